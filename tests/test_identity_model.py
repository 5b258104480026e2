"""CPU model of the identity kernel's arithmetic (design check; not the oracle).

The GPU kernel evaluates Eq. (2) as two products, each carried as a mantissa
in [1/2, 1) and a separate integer exponent: the eigenvalues of the matrix are
first scaled by 2^-E (E the exponent of the largest |lambda|; exact), every
second factor the mantissa is renormalised with frexp, and
W = ldexp(P / Q, e_P - e_Q).  This model performs the same steps in numpy and
checks them against the oracle's compensated log sums (an independent
formulation), and at scales where plain products overflow or underflow.
"""
import math

import numpy as np
import pytest

import oracle


def scaled_product(factors):
    """Product of the factors (each < 4) as (mantissa, exponent), renormalised
    after every second factor, as the kernel does."""
    m, e = 1.0, 0
    k = 0
    while k + 1 < len(factors):
        m, de = math.frexp(m * (factors[k] * factors[k + 1]))
        e += de
        k += 2
    if k < len(factors):
        m, de = math.frexp(m * factors[k])
        e += de
    return m, e


def identity_model(lam, mu_rows):
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    big = max(abs(lam[0]), abs(lam[-1]))
    E = math.frexp(big)[1] - 1 if big > 0 else 0          # exponent of the largest |lambda|
    ls = np.ldexp(lam, -E)
    W = np.empty((n, len(mu_rows)))
    for i in range(n):
        qf = [abs(ls[i] - ls[k]) for k in range(n) if k != i]
        if any(f == 0.0 for f in qf):
            W[i, :] = np.nan
            continue
        qm, qe = scaled_product(qf)
        for t, mu in enumerate(mu_rows):
            pm, pe = scaled_product([abs(ls[i] - v) for v in np.ldexp(np.asarray(mu), -E)])
            W[i, t] = math.ldexp(pm / qm, pe - qe)
    return W


@pytest.mark.parametrize("n, seed", [(2, 1), (17, 2), (64, 3), (150, 4)])
def test_model_matches_the_oracles_log_sums(n, seed):
    a = np.random.default_rng(seed).standard_normal((n, n))
    a = (a + a.T) / np.sqrt(2)
    lam = oracle.eigvalsh(a, "lapack")
    js = list(range(0, n, max(1, n // 6)))
    mu = oracle.minor_spectra(a, js, "lapack")
    W_log, _ = oracle.identity_from_spectra(lam, mu)
    W = identity_model(lam, mu)
    assert np.max(np.abs(W - W_log)) < 1e-13 * max(1, n / 16)


@pytest.mark.parametrize("scale", [1e-250, 1e250])
def test_model_at_scales_where_plain_products_fail(scale):
    # n = 300: the plain product of |differences| overflows (or underflows) in
    # FP64 at these scales; the components are invariant under scaling of A
    n = 300
    a = np.random.default_rng(5).standard_normal((n, n))
    a = (a + a.T) / np.sqrt(2)
    lam = oracle.eigvalsh(a, "lapack")
    mu = oracle.minor_spectra(a, [0, 150], "lapack")
    with np.errstate(over="ignore", under="ignore"):
        plain = np.prod(np.abs(lam[1:] * scale - lam[0] * scale))
    assert plain == 0.0 or not np.isfinite(plain)
    W_ref = identity_model(lam, mu)
    W = identity_model(lam * scale, mu * scale)
    assert np.all(np.isfinite(W))
    assert np.max(np.abs(W - W_ref)) < 1e-12


def test_model_zero_factor_and_degenerate_row():
    lam = np.array([-1.0, 0.0, 2.0])
    mu = np.array([[0.0, 1.0]])               # mu hits lambda_1 exactly: W[1, 0] = 0
    W = identity_model(lam, mu)
    assert W[1, 0] == 0.0 and np.all(np.isfinite(W))
    W = identity_model(np.array([1.0, 1.0, 3.0]), np.array([[1.0, 2.0]]))
    assert np.all(np.isnan(W[0])) and np.all(np.isnan(W[1])) and np.isfinite(W[2, 0])
