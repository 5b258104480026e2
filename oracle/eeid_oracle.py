"""CPU FP64 oracle for the eigenvector-eigenvalue identity.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library never
calls it and shares no code with it.

What the paper fixes (Section 2, Eq. (2)): for an n x n Hermitian A with
ascending eigenvalues lambda_1..lambda_n and M_j the minor of A with row j
*and* column j removed,

    |v_ij|^2 = prod_{k=1}^{n-1} (lambda_i(A) - lambda_k(M_j))
               / prod_{k != i} (lambda_i(A) - lambda_k(A)),

where v_i is the unit eigenvector of lambda_i.  Algorithm 2 (Section 3)
computes the spectrum of A once and the spectrum of each minor once and then
forms the ratio of products.

Two routes are provided:

* the method (``components_identity``): EigenValues(A), EigenValues(M_j) for
  every j, then the ratio above evaluated as a sum of logarithms of
  |differences| with Neumaier-compensated summation (the paper notes raw
  products over- or underflow for n of order 150 and up, Section 3);
* the plain definition (``components_definition``): a Jacobi
  eigendecomposition with accumulated rotations, W_ij = |V_ji|^2.

Readings of the paper taken here (the text is silent or garbled):

* i indexes the eigenvalue and j the component / deleted row, as in Eq. (2)
  (the algorithms print the two indices the other way round);
* ``del`` removes row and column j (Section 2 says both);
* eigenvalues are ascending (the LAPACK convention of NumPy's routine that
  the paper calls);
* every factor enters through its absolute value;
* an exactly zero factor in the numerator gives W = 0; an exactly repeated
  eigenvalue of A (zero denominator factor) makes row i undefined: it is NaN
  and the matrix is flagged degenerate;
* only the lower triangle of A is read and the imaginary parts of its
  diagonal are ignored.

The EigenValues step is cyclic Jacobi in plain C (``jacobi.c``), carried in
extended precision by default (``method="jacobi"``; ``"jacobi64"`` runs the
same code in double precision).  ``method="lapack"`` swaps in
``numpy.linalg.eigvalsh`` as a library routine for the same step (used where
Jacobi would take hours); it is a cross-check, not the oracle.
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

FLAG_NONFINITE_INPUT = 1
FLAG_DEGENERATE = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}


def _lib(precision: str = "extended"):
    lib = _LIBS.get(precision)
    if lib is None:
        from . import build as _build
        path = _build.build(force=False, precision=precision)
        lib = ctypes.CDLL(path)
        for name in ("oracle_jacobi_r64", "oracle_jacobi_c128"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p]
        _LIBS[precision] = lib
    return lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


# --------------------------------------------------------------------------
# Input convention
# --------------------------------------------------------------------------
def hermitian_from_lower(a: np.ndarray) -> np.ndarray:
    """The Hermitian matrix whose lower triangle is that of ``a`` (diagonal made real)."""
    a = np.asarray(a)
    low = np.tril(a, -1)
    if np.iscomplexobj(a):
        d = np.diag(np.real(np.diag(a))).astype(np.complex128)
        return low + low.conj().T + d
    return low + low.T + np.diag(np.diag(a))


# --------------------------------------------------------------------------
# EigenValues(.) -- Algorithms 1 and 2, Section 3
# --------------------------------------------------------------------------
def _jacobi_call(a, vectors, max_sweeps, precision, max_rounds=0):
    a = np.asarray(a)
    n = a.shape[0]
    lib = _lib(precision)
    w = np.empty(n, dtype=np.float64)
    st = np.zeros(2, dtype=np.int64)
    if np.iscomplexobj(a):
        work = np.ascontiguousarray(a, dtype=np.complex128)
        v = np.empty((n, n), dtype=np.complex128) if vectors else None
        fn = lib.oracle_jacobi_c128
    else:
        work = np.ascontiguousarray(a, dtype=np.float64)
        v = np.empty((n, n), dtype=np.float64) if vectors else None
        fn = lib.oracle_jacobi_r64
    rc = fn(n, work.ctypes.data, w.ctypes.data, v.ctypes.data if vectors else None, max_sweeps,
            max_rounds, st.ctypes.data)
    return rc, w, v, dict(sweeps=int(rc), rotations=int(st[0]), rounds=int(st[1]))


def eigh_jacobi(a: np.ndarray, vectors: bool = True, max_sweeps: int = 60,
                precision: str = "extended", stats: dict | None = None):
    """Jacobi eigen-decomposition: ascending w and (optionally) V with A V = V diag(w).

    ``precision`` is the working precision of the rotations: "extended" (x87,
    64-bit significand; the default) or "double".  Input and output are FP64.
    If ``stats`` is a dict it receives the sweeps, rotations and rounds taken.
    """
    rc, w, v, st = _jacobi_call(a, vectors, max_sweeps, precision)
    if rc < 0:
        raise RuntimeError(f"Jacobi did not converge in {max_sweeps} sweeps (n={np.asarray(a).shape[0]})")
    if stats is not None:
        stats.update(st)
    return (w, v) if vectors else w


def jacobi_rounds_sample(a: np.ndarray, max_rounds: int, precision: str = "extended") -> dict:
    """Time the first ``max_rounds`` rounds of the Jacobi iteration on ``a``.

    Only a timing aid for bounded samples of problems too large to finish
    (the benchmark's CPU baseline): returns the wall seconds, rounds and
    rotations of the capped run; its eigenvalue output is discarded.
    """
    import time
    t0 = time.perf_counter()
    rc, _, _, st = _jacobi_call(a, False, 60, precision, max_rounds=max_rounds)
    st["seconds"] = time.perf_counter() - t0
    st["capped"] = rc == -2
    return st


# EigenValues methods: "jacobi" (extended-precision Jacobi, the oracle),
# "jacobi64" (the same code in double precision) and "lapack" (numpy's
# eigvalsh, a library routine, not the oracle).
METHODS = ("jacobi", "jacobi64", "lapack")


def eigvalsh(a: np.ndarray, method: str = "jacobi", stats: dict | None = None) -> np.ndarray:
    """Ascending eigenvalues of the Hermitian matrix given by the lower triangle of ``a``."""
    a = np.asarray(a)
    if a.shape[0] == 0:
        return np.zeros(0)
    if method == "jacobi":
        return eigh_jacobi(a, vectors=False, precision="extended", stats=stats)
    if method == "jacobi64":
        return eigh_jacobi(a, vectors=False, precision="double", stats=stats)
    if method == "lapack":
        return np.linalg.eigvalsh(a, UPLO="L").astype(np.float64)
    raise ValueError(method)


def minor(a: np.ndarray, j: int) -> np.ndarray:
    """M_j: A with row j and column j removed (Section 2, the text around Eq. (2))."""
    keep = np.r_[0:j, j + 1:a.shape[0]]
    return np.ascontiguousarray(a[np.ix_(keep, keep)])


def minor_spectra(a: np.ndarray, js=None, method: str = "jacobi", threads: int | None = None):
    """Rows mu[t] = ascending eigenvalues of M_{js[t]} (all minors when js is None)."""
    n = a.shape[0]
    js = list(range(n)) if js is None else [int(j) for j in js]
    mu = np.empty((len(js), max(n - 1, 0)), dtype=np.float64)
    if n == 1:
        return mu
    threads = threads or default_threads()

    def one(t):
        mu[t] = eigvalsh(minor(a, js[t]), method)

    if threads == 1 or len(js) == 1:
        for t in range(len(js)):
            one(t)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(len(js))))
    return mu


# --------------------------------------------------------------------------
# The ratio of products of Eq. (2), in the log domain
# --------------------------------------------------------------------------
def neumaier_sum(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """Neumaier-compensated sum along ``axis`` (sequential in the summation index)."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, 0)
    s = np.zeros(x.shape[1:])
    c = np.zeros(x.shape[1:])
    for k in range(x.shape[0]):
        xk = x[k]
        t = s + xk
        big = np.abs(s) >= np.abs(xk)
        c += np.where(big, (s - t) + xk, (xk - t) + s)
        s = t
    return s + c


def log_abs_sum(diff: np.ndarray, axis: int = -1) -> np.ndarray:
    """sum_k log|diff_k| along ``axis``; -inf where some factor is exactly zero."""
    diff = np.asarray(diff, dtype=np.float64)
    zero = np.any(diff == 0.0, axis=axis)
    with np.errstate(divide="ignore"):
        logs = np.log(np.abs(np.where(diff == 0.0, 1.0, diff)))
    out = neumaier_sum(logs, axis=axis)
    return np.where(zero, -np.inf, out)


def denominators(lam: np.ndarray):
    """D_i = sum_{k != i} log|lambda_i - lambda_k| (denominator of Eq. (2)).

    Returns (D, degenerate) where degenerate[i] is True when some k != i has
    lambda_k == lambda_i exactly.
    """
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    if n <= 1:
        return np.zeros(n), np.zeros(n, dtype=bool)
    diff = lam[:, None] - lam[None, :]
    off = ~np.eye(n, dtype=bool)
    diff_off = diff[off].reshape(n, n - 1)
    degenerate = np.any(diff_off == 0.0, axis=1)
    return log_abs_sum(diff_off, axis=1), degenerate


def numerators(lam: np.ndarray, mu_rows: np.ndarray) -> np.ndarray:
    """N[i, t] = sum_k log|lambda_i - mu_rows[t, k]| (numerator of Eq. (2))."""
    lam = np.asarray(lam, dtype=np.float64)
    mu_rows = np.asarray(mu_rows, dtype=np.float64)
    diff = lam[:, None, None] - mu_rows[None, :, :]          # (n, T, m)
    return log_abs_sum(diff, axis=2)


def identity_from_spectra(lam: np.ndarray, mu_rows: np.ndarray):
    """W[i, t] = exp(N[i, t] - D_i): column t holds |v_i(j_t)|^2 for the minor whose spectrum is mu_rows[t].

    Returns (W, flags) with flags bit FLAG_DEGENERATE set when a row is NaN.
    """
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    mu_rows = np.asarray(mu_rows, dtype=np.float64)
    if n == 1:
        return np.ones((1, mu_rows.shape[0])), 0
    mu_rows = mu_rows.reshape(-1, n - 1)
    D, degenerate = denominators(lam)
    N = numerators(lam, mu_rows)
    with np.errstate(invalid="ignore"):
        W = np.exp(N - D[:, None])
    W[degenerate, :] = np.nan
    flags = FLAG_DEGENERATE if degenerate.any() else 0
    return W, flags


def components_identity(a: np.ndarray, js=None, method: str = "jacobi",
                        threads: int | None = None):
    """The method end to end (Algorithm 2 with the readings above).

    Returns (lam, mu, W, flags): lam ascending (n,), mu[t] the ascending
    spectrum of M_{js[t]}, W[i, t] = |v_i(js[t])|^2 (all j when js is None, so
    W is n x n), flags as in the library.
    """
    a = hermitian_from_lower(np.asarray(a))
    n = a.shape[0]
    js = list(range(n)) if js is None else [int(j) for j in js]
    if not np.all(np.isfinite(a)):
        nan = np.full
        return (nan(n, np.nan), nan((len(js), n - 1), np.nan),
                nan((n, len(js)), np.nan), FLAG_NONFINITE_INPUT)
    lam = eigvalsh(a, method)
    mu = minor_spectra(a, js, method, threads)
    W, flags = identity_from_spectra(lam, mu)
    return lam, mu, W, flags


def components_definition(a: np.ndarray):
    """The plain definition: W[i, j] = |V[j, i]|^2 from a Jacobi eigendecomposition."""
    a = hermitian_from_lower(np.asarray(a))
    w, v = eigh_jacobi(a, vectors=True)
    return w, (np.abs(v) ** 2).T.copy()


# --------------------------------------------------------------------------
# Signs of the eigenvector components: Eq. (2) in other bases (Section 2)
# --------------------------------------------------------------------------
def signed_eigenvectors_definition(a: np.ndarray, r: int):
    """The plain definition: (lam, V) with row i of V the unit eigenvector of
    the i-th smallest eigenvalue of the Hermitian A, its sign (real A) or phase
    (complex A) fixed so that V[i, r] is real and >= 0 (a row with V[i, r] == 0
    keeps the Jacobi phase)."""
    a = hermitian_from_lower(np.asarray(a))
    w, v = eigh_jacobi(a, vectors=True)
    V = v.T.copy()
    ref = V[:, r]
    mag = np.abs(ref)
    ph = np.where(mag > 0, np.conj(ref) / np.where(mag > 0, mag, 1.0), 1.0)
    V *= ph[:, None]
    if not np.iscomplexobj(a):
        V = V.real.copy()
    return w, V


def rotation(n: int, r: int, k: int, rot: int = 0) -> np.ndarray:
    """R with columns the new basis: rot 0: e'_r = (e_r + e_k)/sqrt2, e'_k = (e_k - e_r)/sqrt2;
    rot 1: e'_r = (e_r + i e_k)/sqrt2, e'_k = (e_k + i e_r)/sqrt2; e'_p = e_p otherwise."""
    h = 1.0 / np.sqrt(2.0)
    if rot == 0:
        R = np.eye(n)
        R[r, r], R[k, r] = h, h
        R[r, k], R[k, k] = -h, h
    else:
        R = np.eye(n, dtype=np.complex128)
        R[r, r], R[k, r] = h, 1j * h
        R[r, k], R[k, k] = 1j * h, h
    return R


def rotated_minor(a: np.ndarray, r: int, k: int, rot: int = 0) -> np.ndarray:
    """The minor at r of B = R^H A R (R = rotation(n, r, k, rot)): B has A's
    eigenvalues and component r of its eigenvector i is (v_ir + v_ik)/sqrt2
    (rot 0) or (v_ir - i v_ik)/sqrt2 (rot 1)."""
    a = hermitian_from_lower(np.asarray(a))
    R = rotation(a.shape[0], r, k, rot)
    return minor(R.conj().T @ a @ R, r)


def signed_eigenvectors_identity(a: np.ndarray, r: int, method: str = "jacobi"):
    """The method: eigenvectors with signs (phases) from Eq. (2) in the
    original basis and in rotated bases of the (r, k) planes.

    W_ik = |v_ik|^2 from the minors of A; from the minor at r of R^H A R (same
    eigenvalues, so the same denominators) Eq. (2) gives
    S_ik = (W_ir + W_ik)/2 + Re(conj(v_ir) v_ik) for the real rotation and, for
    complex A, (W_ir + W_ik)/2 + Im(conj(v_ir) v_ik) for the imaginary one; with
    v_ir = sqrt(W_ir) real >= 0, v_ik = conj(v_ir) v_ik / sqrt(W_ir).  Rows with
    W_ir = 0 are NaN.  Returns (lam, V) with V as in signed_eigenvectors_definition.
    """
    a = hermitian_from_lower(np.asarray(a))
    cplx = np.iscomplexobj(a)
    n = a.shape[0]
    lam, _, W, _ = components_identity(a, method=method)
    if n == 1:
        return lam, np.ones((1, 1), dtype=a.dtype)
    ks = [k for k in range(n) if k != r]
    sr = np.sqrt(W[:, r])
    V = np.empty((n, n), dtype=np.complex128 if cplx else np.float64)
    parts = []
    for rot in ((0, 1) if cplx else (0,)):
        mu_rot = np.array([eigvalsh(rotated_minor(a, r, k, rot), method) for k in ks])
        S, _ = identity_from_spectra(lam, mu_rot)
        parts.append(S)
    with np.errstate(divide="ignore", invalid="ignore"):
        for q, k in enumerate(ks):
            half = 0.5 * (W[:, r] + W[:, k])
            val = parts[0][:, q] - half
            if cplx:
                val = val + 1j * (parts[1][:, q] - half)
            V[:, k] = val / sr
    V[:, r] = sr
    V[W[:, r] == 0.0] = np.nan
    return lam, V


# --------------------------------------------------------------------------
# Invariants every exact W satisfies (used as pins and as large-n checks)
# --------------------------------------------------------------------------
def invariants(a: np.ndarray, lam: np.ndarray, W: np.ndarray) -> dict:
    """Residuals of identities that hold for the exact W of a Hermitian A.

    rows:   max_i |sum_j W_ij - 1|           (unit eigenvectors)
    cols:   max_j |sum_i W_ij - 1|           (orthonormal basis)
    diag:   max_j |sum_i lam_i W_ij - A_jj|  (A_jj = e_j^H A e_j)
    frob:   max_j |sum_i lam_i^2 W_ij - sum_k |A_jk|^2|
    range:  how far W leaves [0, 1]
    """
    a = hermitian_from_lower(np.asarray(a))
    lam = np.asarray(lam, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    rows = np.max(np.abs(W.sum(axis=1) - 1.0))
    cols = np.max(np.abs(W.sum(axis=0) - 1.0))
    diag = np.max(np.abs(lam @ W - np.real(np.diag(a))))
    frob = np.max(np.abs((lam ** 2) @ W - np.sum(np.abs(a) ** 2, axis=1)))
    rng = max(0.0, -float(W.min()), float(W.max()) - 1.0)
    return dict(rows=float(rows), cols=float(cols), diag=float(diag), frob=float(frob), range=rng)


def minor_invariants(a: np.ndarray, lam: np.ndarray, mu: np.ndarray, js) -> dict:
    """Cauchy interlacing and trace identities for the minor spectra.

    interlace: worst violation of lam_k <= mu_jk <= lam_{k+1}
    trace:     max_j |sum_k mu_jk - (tr A - A_jj)|
    frob:      max_j |sum_k mu_jk^2 - ||M_j||_F^2|
    """
    a = hermitian_from_lower(np.asarray(a))
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    d = np.real(np.diag(a))
    tr = d.sum()
    fro2 = np.sum(np.abs(a) ** 2)
    row2 = np.sum(np.abs(a) ** 2, axis=1)
    worst_il = 0.0
    worst_tr = 0.0
    worst_fr = 0.0
    for t, j in enumerate(js):
        m = mu[t]
        lo = lam[:-1] - m
        hi = m - lam[1:]
        worst_il = max(worst_il, float(np.max(np.maximum(lo, hi), initial=0.0)))
        worst_tr = max(worst_tr, abs(m.sum() - (tr - d[j])))
        worst_fr = max(worst_fr, abs(np.sum(m ** 2) - (fro2 - 2 * row2[j] + d[j] ** 2)))
    return dict(interlace=worst_il, trace=worst_tr, frob=worst_fr)
