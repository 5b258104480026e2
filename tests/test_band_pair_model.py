"""CPU model of the dense-to-band stage with paired panels (design check, not the oracle).

The two-stage kernel reduces a symmetric matrix to a band of half-width b
with one block Householder transform per panel of b columns:
A22 <- Q^T A22 Q = A22 - V W^T - W V^T, Q = I - V T V^T, Y = A22 V, X = Y T,
W = X - 1/2 V (T^T V^T X).  With an FP64 trailing matrix it takes the panels
in pairs: after panel p only the next panel's columns are brought up to date,
panel p + 1 is factored from them, and its Y is formed from the trailing
matrix NOT yet updated by p,

    Y_1 = A V_1 - V_0 (W_0^T V_1) - W_0 (V_0^T V_1),

after which one update with V = [V_0 V_1], W = [W_0 W_1] serves both panels.
This model runs both schedules in numpy on whole matrices and checks that
they give the same band (to rounding), that entries beyond the band vanish
and that the eigenvalues are those of the input.
"""
import numpy as np
import pytest


def householder_panel(P):
    """Compact WY QR of the panel P (h x b): (V, T, R) with (I - V T V^T)^T P = [R; 0]."""
    h, b = P.shape
    V = np.zeros((h, b))
    T = np.zeros((b, b))
    R = P.copy()
    for c in range(min(b, h)):
        x = R[c:, c]
        alpha = x[0]
        sg = float(x[1:] @ x[1:])
        if sg == 0.0:
            tau, v = 0.0, np.r_[1.0, np.zeros(len(x) - 1)]
        else:
            beta = -np.copysign(np.sqrt(alpha * alpha + sg), alpha)
            tau = (beta - alpha) / beta
            v = np.r_[1.0, x[1:] / (alpha - beta)]
        V[c:, c] = v
        R[c:, c:] -= tau * np.outer(v, v @ R[c:, c:])
        # column c of T: T(0:c, c) = -tau T(0:c, 0:c) V(:, 0:c)^T v, T(c, c) = tau
        T[:c, c] = -tau * (T[:c, :c] @ (V[:, :c].T @ V[:, c]))
        T[c, c] = tau
    return V, T, np.triu(R[:b])   # the annihilated entries are exact zeros (as the kernel stores them)


def make_w(Y, V, T):
    X = Y @ T
    return X - 0.5 * V @ (T.T @ (V.T @ X))


def to_band(A, b, paired):
    A = A.copy()
    n = len(A)
    k0 = 0
    while k0 + b < n:
        r0 = k0 + b
        V0, T0, R0 = householder_panel(A[r0:, k0:k0 + b])
        A[r0:, k0:k0 + b] = 0.0
        A[r0:r0 + R0.shape[0], k0:k0 + b] = R0
        A[k0:k0 + b, r0:] = A[r0:, k0:k0 + b].T
        W0 = make_w(A[r0:, r0:] @ V0, V0, T0)
        if not paired or r0 + b >= n:
            A[r0:, r0:] -= V0 @ W0.T + W0 @ V0.T
            k0 = r0
            continue
        # update only the next panel's columns (and their mirror rows), factor it
        r1 = r0 + b
        s = slice(0, b)              # columns r0 .. r1 - 1 of the trailing block
        A[r0:, r0:r1] -= V0 @ W0[s].T + W0 @ V0[s].T
        A[r0:r1, r0:] = A[r0:, r0:r1].T
        V1, T1, R1 = householder_panel(A[r1:, r0:r1])
        A[r1:, r0:r1] = 0.0
        A[r1:r1 + R1.shape[0], r0:r1] = R1
        A[r0:r1, r1:] = A[r1:, r0:r1].T
        # Y of panel p + 1 from the trailing matrix not yet updated by panel p
        V0t, W0t = V0[b:], W0[b:]
        Y1 = A[r1:, r1:] @ V1 - V0t @ (W0t.T @ V1) - W0t @ (V0t.T @ V1)
        W1 = make_w(Y1, V1, T1)
        Vp, Wp = np.hstack([V0t, V1]), np.hstack([W0t, W1])
        A[r1:, r1:] -= Vp @ Wp.T + Wp @ Vp.T
        k0 = r1
    return A


@pytest.mark.parametrize("n,b", [(40, 4), (97, 8), (130, 16), (200, 32)])
def test_paired_panels_give_the_same_band(n, b):
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n))
    A = (G + G.T) / np.sqrt(2.0)
    B1 = to_band(A, b, paired=False)
    B2 = to_band(A, b, paired=True)
    s = np.max(np.abs(np.linalg.eigvalsh(A)))
    i, j = np.indices(A.shape)
    outside = np.abs(i - j) > b
    assert np.max(np.abs(B1[outside])) == 0.0 and np.max(np.abs(B2[outside])) == 0.0
    assert np.max(np.abs(B2 - B1)) < 1e-12 * s
    lam = np.linalg.eigvalsh(A)
    assert np.max(np.abs(np.linalg.eigvalsh(B2) - lam)) < 1e-12 * s
    assert np.max(np.abs(np.linalg.eigvalsh(B1) - lam)) < 1e-12 * s


def test_a_dropped_correction_is_caught():
    # without the two corrections Y_1 comes from the wrong matrix: the band's
    # spectrum is no longer the input's
    n, b = 97, 8
    rng = np.random.default_rng(5)
    G = rng.standard_normal((n, n))
    A = (G + G.T) / np.sqrt(2.0)
    B = to_band(A, b, paired=True)
    lam = np.linalg.eigvalsh(A)
    assert np.max(np.abs(np.linalg.eigvalsh(B) - lam)) < 1e-12 * np.max(np.abs(lam))

    def to_band_uncorrected(A, b):
        A = A.copy()
        r0, k0 = b, 0
        V0, T0, R0 = householder_panel(A[r0:, k0:k0 + b])
        A[r0:, k0:k0 + b] = 0.0
        A[r0:r0 + R0.shape[0], k0:k0 + b] = R0
        A[k0:k0 + b, r0:] = A[r0:, k0:k0 + b].T
        W0 = make_w(A[r0:, r0:] @ V0, V0, T0)
        r1 = r0 + b
        A[r0:, r0:r1] -= V0 @ W0[:b].T + W0 @ V0[:b].T
        A[r0:r1, r0:] = A[r0:, r0:r1].T
        V1, T1, R1 = householder_panel(A[r1:, r0:r1])
        A[r1:, r0:r1] = 0.0
        A[r1:r1 + R1.shape[0], r0:r1] = R1
        A[r0:r1, r1:] = A[r1:, r0:r1].T
        Y1 = A[r1:, r1:] @ V1        # corrections dropped
        W1 = make_w(Y1, V1, T1)
        Vp, Wp = np.hstack([V0[b:], V1]), np.hstack([W0[b:], W1])
        A[r1:, r1:] -= Vp @ Wp.T + Wp @ Vp.T
        return A

    Bbad = to_band_uncorrected(A, b)
    # the first two panels' part of the spectrum is now wrong
    assert np.max(np.abs(np.linalg.eigvalsh(Bbad) - lam)) > 1e-6
