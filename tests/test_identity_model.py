"""CPU model of the identity kernel's arithmetic (design check; not the oracle).

The GPU kernel evaluates Eq. (2) as two products, each carried as a mantissa
and a separate integer exponent.  Every factor |lambda_i - x| is split by
frexp into a mantissa in [1/2, 1) and an exponent before it is multiplied in;
the running mantissa is renormalised after every eighth factor (the numerator
also at the end of every LDS chunk of 256 minor eigenvalues, the denominator
at its end), and W = ldexp(P / Q, e_P - e_Q).  The eigenvalues are scaled by
a power of two only when the largest |lambda| reaches 2^1021.

This model performs the same IEEE operations in the same order, so it gives
the kernel's results bit for bit; the tests check it against the oracle's
compensated log sums (an independent formulation), at scales where plain
products overflow or underflow, and on graded spectra whose single factors
lie far outside the range where a product of two of them stays normal.
"""
import math

import numpy as np
import pytest

import oracle

RENORM = 8
KC = 256


def spectrum_exponent(lam) -> int:
    big = max(abs(lam[0]), abs(lam[-1]))
    e = math.frexp(big)[1] - 1 if big > 0 else 0          # ilogb
    return e - 1020 if e >= 1021 else 0


def mul_factor(pm, pe, f):
    fm, fe = math.frexp(f)
    return pm * fm, pe + fe


def renormalise(pm, pe):
    m, e = math.frexp(pm)
    return m, pe + e


def denominator(ls, i):
    q, qe, cnt = 1.0, 0, 0
    zero = False
    for k in range(len(ls)):
        if k == i:
            continue
        d = ls[i] - ls[k]
        zero = zero or d == 0.0
        q, qe = mul_factor(q, qe, abs(d))
        cnt += 1
        if cnt == RENORM:
            q, qe = renormalise(q, qe)
            cnt = 0
    q, qe = renormalise(q, qe)
    return (math.nan, 0) if zero else (q, qe)


def numerator(li, mus):
    pm, pe = 1.0, 0
    for kc in range(0, len(mus), KC):
        chunk = mus[kc:kc + KC]
        kk = 0
        while kk + RENORM <= len(chunk):
            for u in range(RENORM):
                pm, pe = mul_factor(pm, pe, abs(li - chunk[kk + u]))
            pm, pe = renormalise(pm, pe)
            kk += RENORM
        for u in range(kk, len(chunk)):
            pm, pe = mul_factor(pm, pe, abs(li - chunk[u]))
        pm, pe = renormalise(pm, pe)
    return pm, pe


def identity_model(lam, mu_rows):
    """W[i, t] for the minor spectra mu_rows[t], step by step as the kernel."""
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    E = spectrum_exponent(lam)
    ls = [math.ldexp(float(x), -E) for x in lam]
    W = np.empty((n, len(mu_rows)))
    for i in range(n):
        qm, qe = denominator(ls, i)
        for t, mu in enumerate(mu_rows):
            pm, pe = numerator(ls[i], [math.ldexp(float(v), -E) for v in mu])
            W[i, t] = math.ldexp(pm / qm, pe - qe) if not math.isnan(qm) else math.nan
    return W


def paired_factors(lam, mu, i):
    """Algorithm 2's paired factors |lambda_i - mu_k| / |lambda_i - lambda'_k|,
    lambda' = lambda without lambda_i, both ascending (scaled as the kernel)."""
    lam = np.asarray(lam, dtype=np.float64)
    E = spectrum_exponent(lam)
    ls = [math.ldexp(float(x), -E) for x in lam]
    ms = [math.ldexp(float(x), -E) for x in mu]
    m = len(ls) - 1
    return [abs(ls[i] - ms[k]) / abs(ls[i] - ls[k + (1 if k >= i else 0)]) for k in range(m)]


def paired_model(lam, mu_rows):
    """The paired kernel's W[i, t]: the factors multiplied in ascending k."""
    n = len(lam)
    W = np.empty((n, len(mu_rows)))
    for i in range(n):
        lam_ = np.asarray(lam, dtype=np.float64)
        lam_other = np.delete(lam_, i)
        if np.any(lam_other == lam_[i]):
            W[i, :] = math.nan
            continue
        for t, mu in enumerate(mu_rows):
            r = 1.0
            for f in paired_factors(lam, mu, i):
                r *= f
            W[i, t] = r
    return W


@pytest.mark.parametrize("n, seed", [(2, 1), (17, 2), (64, 3), (150, 4), (300, 6)])
def test_paired_factors_lie_in_the_unit_interval_and_multiply_to_w(n, seed):
    # Cauchy interlacing puts every paired factor in [0, 1] (to rounding), so
    # the running product never grows; it reproduces the oracle's log sums
    a = np.random.default_rng(seed).standard_normal((n, n))
    a = (a + a.T) / np.sqrt(2)
    lam = oracle.eigvalsh(a, "lapack")
    js = list(range(0, n, max(1, n // 6)))
    mu = oracle.minor_spectra(a, js, "lapack")
    fmax = max(max(paired_factors(lam, mu[t], i)) for i in range(n) for t in range(len(js))) if n > 1 else 0.0
    assert fmax <= 1.0 + 1e-9
    W_log, _ = oracle.identity_from_spectra(lam, mu)
    W = paired_model(lam, mu)
    assert np.max(np.abs(W - W_log)) < 1e-13 * max(1, n / 16)


@pytest.mark.parametrize("k", [332, 1020])
def test_paired_form_on_graded_blocks(k):
    lam, mu, W_exp = graded_block_spectra(k)
    W = paired_model(lam, mu)
    assert np.max(np.abs(W - W_exp)) < 1e-13


def test_paired_form_zero_factor_and_degenerate_row():
    W = paired_model(np.array([-1.0, 0.0, 2.0]), np.array([[0.0, 1.0]]))
    assert W[1, 0] == 0.0 and np.all(np.isfinite(W))
    W = paired_model(np.array([1.0, 1.0, 3.0]), np.array([[1.0, 2.0]]))
    assert np.all(np.isnan(W[0])) and np.all(np.isnan(W[1])) and np.isfinite(W[2, 0])


@pytest.mark.parametrize("n, seed", [(2, 1), (17, 2), (64, 3), (150, 4), (300, 6)])
def test_model_matches_the_oracles_log_sums(n, seed):
    a = np.random.default_rng(seed).standard_normal((n, n))
    a = (a + a.T) / np.sqrt(2)
    lam = oracle.eigvalsh(a, "lapack")
    js = list(range(0, n, max(1, n // 6)))
    mu = oracle.minor_spectra(a, js, "lapack")
    W_log, _ = oracle.identity_from_spectra(lam, mu)
    W = identity_model(lam, mu)
    assert np.max(np.abs(W - W_log)) < 1e-13 * max(1, n / 16)


@pytest.mark.parametrize("scale", [1e-250, 1e250, 2.0 ** 1022])
def test_model_at_scales_where_plain_products_fail(scale):
    # n = 300: the plain product of |differences| overflows (or underflows) in
    # FP64 at these scales; the components are invariant under scaling of A.
    # At 2^1022 the eigenvalues themselves are near the top of the range and
    # are scaled down before differences are taken.
    n = 300
    a = np.random.default_rng(5).standard_normal((n, n))
    a = (a + a.T) / np.sqrt(2)
    lam = oracle.eigvalsh(a, "lapack")
    mu = oracle.minor_spectra(a, [0, 150], "lapack")
    lam = lam / np.max(np.abs(lam))
    mu = mu / np.max(np.abs(oracle.eigvalsh(a, "lapack")))
    with np.errstate(over="ignore", under="ignore"):
        plain = np.prod(np.abs(lam[1:] * scale - lam[0] * scale))
    assert plain == 0.0 or not np.isfinite(plain)
    W_ref = identity_model(lam, mu)
    W = identity_model(lam * scale, mu * scale)
    assert np.all(np.isfinite(W))
    assert np.max(np.abs(W - W_ref)) < 1e-12


@pytest.mark.parametrize("g", [1e-150, 1e-158, 1e-160, 1e-165, 1e-200, 1e-300, 5e-320])
def test_graded_diagonal_gives_the_identity(g):
    # diag(g, 2g, 3g, 1): W = I exactly.  Single factors are of order g, so a
    # product of two of them leaves the normal range from g ~ 1e-154 on (and
    # at 5e-320 every factor is itself subnormal).
    a = np.diag([g, 2 * g, 3 * g, 1.0])
    lam, mu, W_o, flags = oracle.components_identity(a)
    assert flags == 0
    W = identity_model(lam, mu)
    np.testing.assert_array_equal(W, np.eye(4))
    np.testing.assert_allclose(W_o, np.eye(4), atol=1e-15)


def graded_block_spectra(k: int, seed: int = 11):
    """Spectra of A = blockdiag(2^-k B, C) (B 5x5, C 6x6 GOE) and of all its
    minors, assembled from those of B, C and their minors at unit scale (the
    power-of-two scale is exact), with the components Eq. (2) must give: the
    rows of the scaled eigenvalues hold B's components on B's indices and 0
    elsewhere, the rows of C's eigenvalues C's components.

    Returns (lam, mu, W_expected) with mu[j] the ascending spectrum of M_j.
    """
    r = np.random.default_rng(seed)
    b = r.standard_normal((5, 5)); b = (b + b.T) / 2
    c = r.standard_normal((6, 6)); c = (c + c.T) / 2
    g = 2.0 ** -k
    lb, mb, Wb, _ = oracle.components_identity(b)
    lc, mc, Wc, _ = oracle.components_identity(c)
    lam_parts = [(g * lb, 0), (lc, 1)]
    lam = np.concatenate([p for p, _ in lam_parts])
    order = np.argsort(lam, kind="stable")
    lam = lam[order]
    mu = np.empty((11, 10))
    for j in range(11):
        if j < 5:
            mu[j] = np.sort(np.concatenate([g * mb[j], lc]))
        else:
            mu[j] = np.sort(np.concatenate([g * lb, mc[j - 5]]))
    W = np.zeros((11, 11))
    W[:5, :5] = Wb
    W[5:, 5:] = Wc
    return lam, mu, W[order]


@pytest.mark.parametrize("k", [332, 531, 830, 1020])
def test_graded_blocks_reduce_to_the_blocks(k):
    # scales 2^-332 ~ 1e-100 ... 2^-1020 ~ 1e-307: the rows of the tiny
    # eigenvalues have numerator and denominator factors of order 2^-k, whose
    # pairwise products leave the normal range; the model and the oracle's
    # log sums must both reproduce B's components computed at unit scale
    lam, mu, W_exp = graded_block_spectra(k)
    W = identity_model(lam, mu)
    W_o, flags = oracle.identity_from_spectra(lam, mu)
    assert flags == 0
    assert np.max(np.abs(W - W_exp)) < 1e-13
    # each logarithm is of order k ln 2 and carries a rounding error of eps times that
    assert np.max(np.abs(W_o - W_exp)) < 10 * 11 * 2.3e-16 * k * math.log(2)


def test_model_zero_factor_and_degenerate_row():
    lam = np.array([-1.0, 0.0, 2.0])
    mu = np.array([[0.0, 1.0]])               # mu hits lambda_1 exactly: W[1, 0] = 0
    W = identity_model(lam, mu)
    assert W[1, 0] == 0.0 and np.all(np.isfinite(W))
    W = identity_model(np.array([1.0, 1.0, 3.0]), np.array([[1.0, 2.0]]))
    assert np.all(np.isnan(W[0])) and np.all(np.isnan(W[1])) and np.isfinite(W[2, 0])
