"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds only input construction (random draws, symmetrisation,
packing of a batch into one buffer).  It contains none of the method's
arithmetic, and both the CPU oracle and the HIP path consume exactly the
bytes it produces.

The paper states the domain (Hermitian matrices, real symmetric as a special
case; Section 2, around Eq. (2)) but no distribution or seed.  The recipes
below are this project's choice:

* ``goe(n, seed)``      -- G i.i.d. N(0,1), A = (G + G^T)/sqrt(2)
* ``wishart(n, seed)``  -- X (2n x n) i.i.d. N(0,1), A = X^T X / (2n), symmetrised
* ``gue(n, seed)``      -- G with real and imaginary parts i.i.d. N(0,1)
                           (real part drawn first), A = (G + G^H)/2
* ``clustered(n, ...)`` -- A = Q diag(lam) Q^T with Q Haar-orthogonal
                           (QR of a Gaussian matrix, columns sign-fixed by
                           diag(R)) and lam in clusters with a tiny gap.  The
                           exact |v_ij|^2 are Q[j, i]^2 by construction.
* ``uneven_batch(...)`` -- sizes uniform in [32, 384]; even members GOE, odd
                           members Wishart.

All generators use ``numpy.random.default_rng`` (PCG64) so the bytes are the
same on every host running this numpy.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "goe", "wishart", "gue", "clustered", "laplacian", "uneven_batch",
    "pack_batch", "WORKLOADS", "make_workload",
]


def goe(n: int, seed) -> np.ndarray:
    """Symmetrised Gaussian: A = (G + G^T)/sqrt(2), G i.i.d. N(0,1)."""
    g = np.random.default_rng(seed).standard_normal((n, n))
    a = (g + g.T) / np.sqrt(2.0)
    return np.ascontiguousarray(a)


def wishart(n: int, seed) -> np.ndarray:
    """Wishart X^T X / (2n), X of shape (2n, n) i.i.d. N(0,1), made exactly symmetric."""
    x = np.random.default_rng(seed).standard_normal((2 * n, n))
    a = (x.T @ x) / (2 * n)
    a = (a + a.T) / 2.0
    return np.ascontiguousarray(a)


def gue(n: int, seed) -> np.ndarray:
    """Complex Hermitian: A = (G + G^H)/2 with Re G, Im G i.i.d. N(0,1)."""
    r = np.random.default_rng(seed)
    re = r.standard_normal((n, n))
    im = r.standard_normal((n, n))
    g = re + 1j * im
    a = (g + g.conj().T) / 2.0
    return np.ascontiguousarray(a.astype(np.complex128))


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal Q: QR of a Gaussian matrix, Q * sign(diag R)."""
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    q = q * np.sign(np.diag(r))[None, :]
    return q


def clustered(n: int = 2048, clusters: int = 16, gap: float = 1e-6, seed: int = 40):
    """Q diag(lam) Q^T with ``clusters`` groups of n/clusters eigenvalues.

    Cluster centres are sorted draws from U(-1, 1), redrawn (seed sequence
    [seed, attempt]) until every pair of centres is at least twice a cluster's
    width apart.  Inside a cluster the eigenvalues are spaced ``gap`` apart.

    Returns (A, lam, Q): lam ascending, column i of Q is the unit eigenvector
    of lam[i], so the exact squared components are Q[j, i]**2.
    """
    if n % clusters:
        raise ValueError("n must be a multiple of clusters")
    per = n // clusters
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(n, rng)
    width = gap * (per - 1)
    attempt = 0
    while True:
        c = np.sort(np.random.default_rng([seed, attempt]).uniform(-1.0, 1.0, clusters))
        if clusters == 1 or np.min(np.diff(c)) >= 2.0 * width + 1e-12:
            break
        attempt += 1
    t = np.arange(per, dtype=np.float64) - (per - 1) / 2.0
    lam = (c[:, None] + gap * t[None, :]).reshape(-1)
    a = (q * lam[None, :]) @ q.T
    a = (a + a.T) / 2.0
    return np.ascontiguousarray(a), lam, q


def laplacian(n: int) -> np.ndarray:
    """Discrete 1-D Laplacian tridiag(-1, 2, -1) of order n."""
    a = 2.0 * np.eye(n)
    if n > 1:
        idx = np.arange(n - 1)
        a[idx, idx + 1] = -1.0
        a[idx + 1, idx] = -1.0
    return a


def uneven_batch(count: int = 256, lo: int = 32, hi: int = 384, seed: int = 3):
    """List of ``count`` real symmetric matrices with sizes uniform in [lo, hi].

    Member b is GOE for even b and Wishart for odd b, each drawn from its own
    seed sequence [seed, b], so the families interleave across the size range.
    """
    sizes = np.random.default_rng(seed).integers(lo, hi + 1, count)
    mats = []
    for b, nb in enumerate(sizes):
        nb = int(nb)
        mats.append(goe(nb, [seed, b]) if b % 2 == 0 else wishart(nb, [seed, b]))
    return mats


def pack_batch(mats):
    """Concatenate row-major matrices into one flat buffer.

    Returns (flat, n, offset): ``n[b]`` is the order of member b and
    ``offset[b]`` the element offset of its (0, 0) entry in ``flat``.
    """
    n = np.array([m.shape[0] for m in mats], dtype=np.int64)
    sizes = n * n
    offset = np.zeros(len(mats), dtype=np.int64)
    if len(mats) > 1:
        offset[1:] = np.cumsum(sizes)[:-1]
    dtype = np.complex128 if any(np.iscomplexobj(m) for m in mats) else np.float64
    flat = np.empty(int(sizes.sum()), dtype=dtype)
    for m, o, s in zip(mats, offset, sizes):
        flat[o:o + s] = np.asarray(m, dtype=dtype).reshape(-1)
    return flat, n, offset


# The five workloads (sizes, families, precision forms), by name.
# ``make_workload`` builds the matrices; forms are "fp64" (plain) and "fp32"
# (FP32 trailing storage and FP32 matrix-core trailing update).
WORKLOADS = {
    "goe64": dict(family="goe", n=64, seed=1, dtype="r64", forms=("fp64",)),
    "goe512": dict(family="goe", n=512, seed=2, dtype="r64", forms=("fp64",)),
    "uneven256": dict(family="uneven", count=256, seed=3, dtype="r64", forms=("fp64",)),
    "pair2048": dict(family="goe+clustered", n=2048, seed=4, dtype="r64", forms=("fp64", "fp32")),
    "gue4096": dict(family="gue", n=4096, seed=5, dtype="c128", forms=("fp64", "fp32")),
}


def make_workload(name: str):
    """Matrices of a workload (a list; pair2048 holds the GOE and the clustered matrix)."""
    c = WORKLOADS[name]
    if c["family"] == "goe":
        return [goe(c["n"], c["seed"])]
    if c["family"] == "uneven":
        return uneven_batch(c["count"], 32, 384, c["seed"])
    if c["family"] == "goe+clustered":
        a_clu, _, _ = clustered(c["n"], 16, 1e-6, 40)
        return [goe(c["n"], c["seed"]), a_clu]
    if c["family"] == "gue":
        return [gue(c["n"], c["seed"])]
    raise KeyError(name)
