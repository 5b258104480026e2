"""CPU model of the bulge chase's block passing (design check of the GPU
stage-2 algorithm; not the oracle).

The GPU kernel reduces a symmetric band matrix of half-bandwidth 32 to
tridiagonal form by Householder bulge chasing.  Sweep s removes column s below
the subdiagonal; step t of the sweep works on the 32 x 32 blocks B (below the
previous diagonal block) and D (the next diagonal block).  The kernel runs
sweeps in chains of three: sweep s + 1 never loads its blocks, it builds them
from the blocks of sweep s (shifted down and right by one) plus the first row
of sweep s's next step; only the last sweep of a chain stores its blocks, and
the others store just what leaves their blocks.  This model performs exactly
that block passing in numpy and checks it against plain sequential sweeps:
both must give the same band (to rounding) and the eigenvalues of the input.
"""
import numpy as np
import pytest

B = 32


def house(x):
    """v (v[0] = 1), tau, beta with (I - tau v v^T) x = beta e_0."""
    alpha = x[0]
    sig = float(np.dot(x[1:], x[1:]))
    v = np.zeros_like(x)
    v[0] = 1.0
    if sig == 0.0:
        return v, 0.0, alpha
    nrm = np.sqrt(alpha * alpha + sig)
    beta = -nrm if alpha >= 0 else nrm
    v[1:] = x[1:] / (alpha - beta)
    return v, (beta - alpha) / beta, beta


def sequential_sweep(A, s):
    """Sweep s on the full symmetric matrix A (in place), one step at a time."""
    m = A.shape[0]
    t, prev = 0, None
    while True:
        lo = s + 1 + t * B
        if lo > m - 1:
            break
        hi = min(s + (t + 1) * B, m - 1)
        rows = slice(lo, hi + 1)
        if t == 0:
            col = s
        else:
            plo, phi, vp, taup = prev
            blk = A[rows, plo:phi + 1]
            blk -= taup * np.outer(blk @ vp, vp)
            A[plo:phi + 1, rows] = blk.T
            col = plo
        x = A[rows, col].copy()
        if hi - lo + 1 < 2:
            break
        v, tau, beta = house(x)
        if t == 0:
            A[rows, col] = 0.0
            A[lo, col] = beta
            A[col, rows] = A[rows, col]
        else:
            plo, phi, vp, taup = prev
            blk = A[rows, plo:phi + 1]
            blk -= tau * np.outer(v, v @ blk)
            blk[1:, 0] = 0.0
            A[plo:phi + 1, rows] = blk.T
        D = A[rows, rows]
        w = tau * (D @ v)
        w -= 0.5 * tau * (v @ w) * v
        D -= np.outer(v, w) + np.outer(w, v)
        A[rows, rows] = D
        prev = (lo, hi, v, tau)
        t += 1


# ---- the kernel's block formulation: full 32 x 32 blocks, zero outside the matrix
def step(first, x, Bk, Dk, L, st):
    """One step on blocks: previous reflector from the right on B, new reflector
    from column 0 (or x at the first step), applied to B and two-sidedly to D."""
    if not first:
        u = Bk @ st["vp"]
        Bk -= st["taup"] * np.outer(u, st["vp"])
        x = Bk[:, 0].copy()
    tau = 0.0
    if L >= 2:
        v0, tau, beta = house(x[:L].copy())
        v = np.zeros(B)
        v[:L] = v0
    else:
        beta = x[0]
        v = np.zeros(B)
        v[0] = 1.0
    if not first:
        Bk -= tau * np.outer(v, v @ Bk)
        Bk[:, 0] = 0.0
        Bk[0, 0] = beta
    if L >= 2:
        w = tau * (Dk @ v)
        w -= 0.5 * tau * (v @ w) * v
        Dk -= np.outer(v, w) + np.outer(w, v)
        st["vp"] = v
    st["taup"] = tau
    return beta


def load(mem, r0, c0):
    m = mem.shape[0]
    out = np.zeros((B, B))
    r1, c1 = min(m, r0 + B), min(m, c0 + B)
    out[:r1 - r0, :c1 - c0] = mem[r0:r1, c0:c1]
    return out


def store_sym(mem, r, c, val):
    mem[r, c] = val
    mem[c, r] = val


def shifted(PB, PD, CB, CD):
    """Blocks of the next sweep's step: this sweep's blocks of the same step
    shifted down and right by one, plus the first row of its next step."""
    FB, FD = np.zeros((B, B)), np.zeros((B, B))
    FB[:B - 1, :B - 1] = PB[1:, 1:]
    FB[:B - 1, B - 1] = PD[1:, 0]
    FB[B - 1, B - 1] = CB[0, 0]
    FD[:B - 1, :B - 1] = PD[1:, 1:]
    FD[B - 1, :B - 1] = CB[0, 1:]
    FD[:B - 1, B - 1] = CB[0, 1:]
    FD[B - 1, B - 1] = CD[0, 0]
    return FB, FD


def chain(mem, s, K):
    """Sweeps s .. s + K - 1 as one chain (in place on the symmetric matrix mem)."""
    m = mem.shape[0]
    levels = [l for l in range(K) if s + l + 2 < m]
    last = {l: (m - 2 - (s + l)) // B for l in levels}
    st = {l: {"vp": np.zeros(B), "taup": 0.0} for l in levels}
    zero = (np.zeros((B, B)), np.zeros((B, B)))
    prev = {l: zero for l in levels}
    for t in range(max(l + last[l] for l in levels) + 1):
        cur = {}
        for l in levels:
            tt = t - l
            if tt < 0 or tt > last[l]:
                cur[l] = zero
                continue
            sw, lo = s + l, s + l + 1 + tt * B
            L = min(B, m - lo)
            if l == 0:
                x = np.array([mem[lo + i, s] if lo + i < m else 0.0 for i in range(B)]) if tt == 0 else None
                Bk = load(mem, lo, lo - B) if tt > 0 else np.zeros((B, B))
                Dk = load(mem, lo, lo)
            else:
                Bk, Dk = shifted(prev[l - 1][0], prev[l - 1][1], cur[l - 1][0], cur[l - 1][1])
                x = Bk[:, B - 1].copy() if tt == 0 else None
            beta = step(tt == 0, x, Bk, Dk, L, st[l])
            if l == levels[-1]:          # last sweep of the chain: all it holds is final
                if tt == 0:
                    for i in range(L):
                        store_sym(mem, lo + i, sw, beta if i == 0 else 0.0)
                else:
                    for i in range(L):
                        for j in range(B):
                            store_sym(mem, lo + i, lo - B + j, Bk[i, j])
                for i in range(L):
                    for j in range(i + 1):
                        store_sym(mem, lo + i, lo + j, Dk[i, j])
            elif tt == 0:                # final column sw and the first diagonal entry
                for i in range(L):
                    store_sym(mem, lo + i, sw, beta if i == 0 else 0.0)
                mem[lo, lo] = Dk[0, 0]
            else:                        # annihilated first column of B below its first row
                for i in range(1, L):
                    store_sym(mem, lo + i, lo - B, 0.0)
            cur[l] = (Bk, Dk)
        prev = cur


def random_band(m, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((m, m))
    A = (G + G.T) / np.sqrt(2)
    r = np.arange(m)
    A[np.abs(r[:, None] - r[None, :]) > B] = 0.0
    return A


@pytest.mark.parametrize("K", [1, 2, 3])
@pytest.mark.parametrize("m", [3, 4, 5, 17, 33, 34, 35, 63, 64, 65, 66, 67, 97, 98, 99, 130])
def test_chained_sweeps_match_sequential_sweeps(m, K):
    A = random_band(m, 1000 + m)
    S = A.copy()
    for s in range(m - 2):
        sequential_sweep(S, s)
    P = A.copy()
    for s in range(0, m - 2, K):
        chain(P, s, K)
    scale = np.max(np.abs(np.linalg.eigvalsh(A)))
    assert np.max(np.abs(np.tril(S) - np.tril(P))) < 1e-12 * scale * m
    # the result is tridiagonal and has the eigenvalues of the input
    Tm = np.tril(P, -2)
    assert np.max(np.abs(Tm)) < 1e-12 * scale * m
    d, e = np.diag(P), np.diag(P, -1)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.max(np.abs(np.linalg.eigvalsh(T) - np.linalg.eigvalsh(A))) < 1e-12 * scale * m
