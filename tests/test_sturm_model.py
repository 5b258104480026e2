"""CPU model of the bisection's Sturm count (design check, not the oracle).

Each Sturm step is q_i = (d_i - x) - e_{i-1}^2 / q_{i-1}; the count of
negative q_i is the number of eigenvalues below x.  Bisection is provably
right only if the computed count is monotone in x, which holds when every
operation is correctly rounded (a monotone function of its operands).  A
cheaper reciprocal (the hardware reciprocal refined by one Newton step,
within about 11 ulp of 1/q) is not monotone in q; this model replaces 1/q by
fl(1/q) (1 + delta(q)) with |delta| <= 12 eps, delta a pseudo-random function
of q's bits, and shows on GOE, clustered, Laplacian and Wilkinson-type
tridiagonals that

* with correctly rounded division the count never decreases on a fine grid
  and within a few ulp of every eigenvalue;
* with the perturbed reciprocal it does decrease, a few ulp from some
  eigenvalues, although the bisection's results stay within its stopping
  width;
* the kernel's scheme -- halvings with the fast count, then a bracket of four
  stopping widths around the result certified by two correctly rounded
  counts and halved back with them -- needs no fallback on these inputs and
  returns the eigenvalues of the all-correctly-rounded bisection.
"""
import numpy as np
import pytest

EPS = np.finfo(np.float64).eps
TINY = np.finfo(np.float64).tiny


def perturbed_reciprocal(q, ulps=12):
    """fl(1/q) (1 + delta), |delta| <= ulps * eps, delta a hash of q's bits."""
    bits = q.view(np.uint64)
    h = (bits * np.uint64(0x9E3779B97F4A7C15)) ^ (bits >> np.uint64(29))
    h = h * np.uint64(0xBF58476D1CE4E5B9)
    u = (h >> np.uint64(11)).astype(np.float64) / 2.0 ** 53 * 2.0 - 1.0
    return (1.0 / q) * (1.0 + ulps * EPS * u)


def sturm_count(d, e2, x, pivmin, exact=False):
    """#{i : q_i < 0} for every x (vectorised over x), as the kernel computes it."""
    x = np.asarray(x, dtype=np.float64)
    q = np.ones_like(x)
    cnt = np.zeros(x.shape, dtype=np.int64)
    with np.errstate(over="ignore", invalid="ignore"):
        for i in range(len(d)):
            # the kernel's step: one correctly rounded division; the model's alternative
            v = (d[i] - x) - (e2[i] / q if exact else e2[i] * perturbed_reciprocal(q))
            v = np.where(np.abs(v) < pivmin, -pivmin, v)
            cnt += v < 0.0
            q = v
    return cnt


def bisect_all(d, e, exact, certify=False):
    """Every eigenvalue by bisection with the kernel's stopping rule.

    certify: as the kernel, halve with the fast (inexact-reciprocal) count,
    then certify a bracket of four stopping widths on either side of the
    result with two correctly rounded counts (a 64 times wider one, or the
    Gershgorin interval, where that fails) and halve it back to the stopping
    width with correctly rounded counts.  Returns (eigenvalues, atol[, redone])."""
    m = len(d)
    el = np.r_[0.0, np.abs(e)]
    er = np.r_[np.abs(e), 0.0]
    e2 = el * el
    gl, gu = np.min(d - el - er), np.max(d + el + er)
    pivmin = TINY * max(1.0, float(np.max(e2)))
    tnorm = max(abs(gl), abs(gu))
    pad = 2.0 * EPS * tnorm * m + 4.0 * pivmin
    gl, gu = gl - pad, gu + pad
    atol = EPS * tnorm
    idx = np.arange(m)
    lo, hi = np.full(m, gl), np.full(m, gu)

    def halve(lo, hi, done, ex):
        for _ in range(80):
            if done.all():
                break
            x = 0.5 * (lo + hi)
            c = sturm_count(d, e2, x, pivmin, ex)
            up = c > idx
            hi = np.where(~done & up, x, hi)
            lo = np.where(~done & ~up, x, lo)
            w = hi - lo
            mid = 0.5 * (lo + hi)
            done = done | (w <= np.maximum(2.0 * EPS * np.maximum(np.abs(lo), np.abs(hi)), atol)) | (mid <= lo) \
                | (mid >= hi)
        return lo, hi

    lo, hi = halve(lo, hi, np.zeros(m, dtype=bool), exact and not certify)
    if not certify:
        return 0.5 * (lo + hi), atol
    mid = 0.5 * (lo + hi)
    sw = np.maximum(2.0 * EPS * np.maximum(np.abs(lo), np.abs(hi)), atol)
    lo, hi = np.maximum(gl, mid - 4 * sw), np.minimum(gu, mid + 4 * sw)
    ok = (sturm_count(d, e2, lo, pivmin, True) <= idx) & (sturm_count(d, e2, hi, pivmin, True) > idx)
    redone = int(np.count_nonzero(~ok))
    if redone:
        wl, wh = np.maximum(gl, mid - 256 * sw), np.minimum(gu, mid + 256 * sw)
        wok = (sturm_count(d, e2, wl, pivmin, True) <= idx) & (sturm_count(d, e2, wh, pivmin, True) > idx)
        lo = np.where(ok, lo, np.where(wok, wl, gl))
        hi = np.where(ok, hi, np.where(wok, wh, gu))
    lo, hi = halve(lo, hi, np.zeros(m, dtype=bool), True)
    # every bracket now passes the monotone count
    assert np.all(sturm_count(d, e2, lo, pivmin, True) <= idx)
    assert np.all(sturm_count(d, e2, hi, pivmin, True) > idx)
    return 0.5 * (lo + hi), atol, redone


def goe_tridiagonal(n, seed):
    # Dumitriu-Edelman: the tridiagonal model of the GOE (beta = 1)
    r = np.random.default_rng(seed)
    d = r.standard_normal(n) * np.sqrt(2.0)
    e = np.sqrt(r.chisquare(np.arange(n - 1, 0, -1)))
    return d / np.sqrt(2.0), e / np.sqrt(2.0)


def clustered_tridiagonal(n, seed):
    # tridiagonal form of Q diag(lambda) Q^T with clusters 1e-6 wide (Householder, scipy)
    from scipy.linalg import hessenberg
    r = np.random.default_rng(seed)
    q, rr = np.linalg.qr(r.standard_normal((n, n)))
    q = q * np.sign(np.diag(rr))
    c = np.sort(r.uniform(-1, 1, 8))
    lam = np.repeat(c, n // 8) + 1e-6 * np.tile(np.arange(n // 8) - n / 16, 8)
    a = (q * lam) @ q.T
    h = hessenberg((a + a.T) / 2)
    return np.diag(h).copy(), np.diag(h, -1).copy()


def laplacian(n):
    return np.full(n, 2.0), np.full(n - 1, -1.0)


def wilkinson(m):
    # W_{2m+1}^+: pairs of eigenvalues agreeing to many digits
    return np.abs(np.arange(-m, m + 1)).astype(np.float64), np.ones(2 * m)


CASES = {
    "goe300": lambda: goe_tridiagonal(300, 1),
    "clustered256": lambda: clustered_tridiagonal(256, 2),
    "laplacian200": lambda: laplacian(200),
    "wilkinson21": lambda: wilkinson(10),
    "wilkinson101": lambda: wilkinson(50),
}


def grid_near_eigenvalues(d, e):
    lam = np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
    x = np.linspace(lam[0] - 1.0, lam[-1] + 1.0, 4001)
    near = (lam[:, None] * (1.0 + EPS * np.arange(-6, 7)[None, :])).ravel()
    near = np.r_[near, (lam[:, None] + EPS * np.max(np.abs(lam)) * np.arange(-6, 7)[None, :]).ravel()]
    return lam, np.unique(np.r_[x, near])


@pytest.mark.parametrize("name", list(CASES))
def test_count_is_monotone_with_correctly_rounded_division(name):
    d, e = CASES[name]()
    e2 = np.r_[0.0, e * e]
    lam, x = grid_near_eigenvalues(d, e)
    pivmin = TINY * max(1.0, float(np.max(e2)))
    c = sturm_count(d, e2, x, pivmin, exact=True)
    assert np.all(np.diff(c) >= 0), f"count decreases at {x[np.flatnonzero(np.diff(c) < 0)][:4]}"
    assert c[0] == 0 and c[-1] == len(d)


def test_an_inexact_reciprocal_breaks_monotonicity_near_eigenvalues():
    violations = {}
    for name, make in CASES.items():
        d, e = make()
        e2 = np.r_[0.0, e * e]
        lam, x = grid_near_eigenvalues(d, e)
        pivmin = TINY * max(1.0, float(np.max(e2)))
        c = sturm_count(d, e2, x, pivmin)
        bad = np.flatnonzero(np.diff(c) < 0)
        violations[name] = len(bad)
        if len(bad):
            # only ever a few ulp from an eigenvalue
            dist = np.min(np.abs(x[bad][:, None] - lam[None, :]), axis=1)
            assert np.all(dist <= 16 * EPS * np.max(np.abs(lam))), (name, dist.max())
    assert sum(violations.values()) > 0, violations


@pytest.mark.parametrize("name", list(CASES))
def test_bisection_unchanged_by_the_inexact_reciprocal(name):
    d, e = CASES[name]()
    w_model, atol = bisect_all(d, e, exact=False)
    w_exact, _ = bisect_all(d, e, exact=True)
    lam = np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
    width = np.maximum(2 * EPS * np.abs(w_exact), atol)
    assert np.all(np.abs(w_model - w_exact) <= 2 * width)
    assert np.all(np.diff(w_model) >= 0)
    assert np.max(np.abs(w_model - lam)) < 64 * EPS * np.max(np.abs(lam)) * np.sqrt(len(d))


def test_the_perturbation_model_spans_its_bound():
    q = np.random.default_rng(3).standard_normal(100000) * 10.0 ** np.random.default_rng(4).uniform(-300, 300, 100000)
    rel = perturbed_reciprocal(q) * q - 1.0
    assert np.max(np.abs(rel)) <= 14 * EPS and np.max(np.abs(rel)) > 10 * EPS


@pytest.mark.parametrize("name", list(CASES))
def test_certified_fast_bisection_matches_the_exact_one(name):
    # the kernel's scheme: fast halvings, then every bracket certified by the
    # monotone count (redone with it where the certificate fails)
    d, e = CASES[name]()
    w_cert, atol, redone = bisect_all(d, e, exact=True, certify=True)
    w_exact, _ = bisect_all(d, e, exact=True)
    width = np.maximum(2 * EPS * np.abs(w_exact), atol)
    assert np.all(np.abs(w_cert - w_exact) <= 2 * width)
    assert redone == 0
