"""GPU identity kernel (Eq. (2)) on given spectra, and the bounded waits.

* The kernel's products are bit for bit those of the step-by-step CPU model
  in tests/test_identity_model.py (same IEEE operations in the same order),
  on GOE spectra that span several LDS chunks of minor eigenvalues and a
  ragged tail.
* The paired form (Algorithm 2's factors in [0, 1]) is bit for bit its own
  CPU model and agrees with the products form.
* Graded spectra: diag(g, 2g, 3g, 1) gives W = I exactly for g down to the
  subnormal range, and blockdiag(2^-k B, C) reproduces the components of B
  and C computed at unit scale, although single factors are of order 2^-k.
* Spectra near the top of the double range (scaled internally) give the
  same components as at unit scale.
* A bounded inter-wave wait whose poll limit is forced to zero from the host
  gives up, flags the problem with EEID_FLAG_WAIT_TIMEOUT and the kernel
  still ends normally.
"""
import ctypes
import math
import os

import numpy as np
import pytest

import oracle
from paper_2002_04989_amd import inputs
from tests.gpu_util import announce
from tests.test_identity_model import graded_block_spectra, identity_model, paired_model

pytestmark = pytest.mark.gpu


def gpu_components(lam, mu_rows, form="products"):
    import torch
    from paper_2002_04989_amd import eeid
    n = len(lam)
    dl = torch.from_numpy(np.ascontiguousarray(lam, dtype=np.float64)).to("cuda:0")
    dm = torch.from_numpy(np.ascontiguousarray(np.asarray(mu_rows, dtype=np.float64).reshape(-1))).to("cuda:0")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    eeid.set_identity_form(form)
    try:
        V2 = eeid.components(dl, dm, [n], flags)
        torch.cuda.synchronize()
    finally:
        eeid.set_identity_form("products")
    return V2.cpu().numpy().reshape(n, n), int(flags.cpu()[0])


@pytest.mark.parametrize("n", [2, 9, 300, 517])
def test_paired_kernel_is_the_model_bit_for_bit(n):
    announce(f"paired identity kernel vs model, GOE spectra n={n}")
    A = inputs.goe(n, 300 + n)
    lam = oracle.eigvalsh(A, "lapack")
    mu = oracle.minor_spectra(A, range(n), "lapack")
    W, flag = gpu_components(lam, mu, "paired")
    assert flag == 0
    js = sorted(set([0, n // 2, n - 1]))
    np.testing.assert_array_equal(W[:, js], paired_model(lam, mu[js]))
    W_prod, _ = gpu_components(lam, mu)
    assert np.max(np.abs(W - W_prod)) < 1e-13 * max(1, n / 16)


@pytest.mark.parametrize("k", [332, 1020])
def test_paired_graded_block_spectra(k):
    announce(f"paired identity kernel, graded blocks 2^-{k}")
    lam, mu, W_exp = graded_block_spectra(k)
    W, flag = gpu_components(lam, mu, "paired")
    assert flag == 0
    np.testing.assert_array_equal(W, paired_model(lam, mu))
    assert np.max(np.abs(W - W_exp)) < 1e-13


def test_paired_conventions():
    announce("paired identity kernel: zero factor, degenerate row")
    W, flag = gpu_components(np.array([-1.0, 0.0, 2.0]), np.array([[0.0, 2.0], [-1.0, 2.0], [-1.0, 0.0]]), "paired")
    assert flag == 0 and np.all(np.isfinite(W))
    np.testing.assert_array_equal(W, np.eye(3))
    W, flag = gpu_components(np.array([1.0, 1.0, 3.0]), np.array([[1.0, 3.0], [1.0, 3.0], [1.0, 1.0]]), "paired")
    assert flag & 2 and np.all(np.isnan(W[:2])) and np.all(np.isfinite(W[2]))


@pytest.mark.parametrize("n", [2, 9, 300, 517])
def test_identity_kernel_is_the_model_bit_for_bit(n):
    announce(f"identity kernel vs model, GOE spectra n={n}")
    A = inputs.goe(n, 300 + n)
    lam = oracle.eigvalsh(A, "lapack")
    mu = oracle.minor_spectra(A, range(n), "lapack")
    W, flag = gpu_components(lam, mu)
    assert flag == 0
    js = sorted(set([0, n // 2, n - 1]))
    W_model = identity_model(lam, mu[js])
    np.testing.assert_array_equal(W[:, js], W_model)
    W_log, _ = oracle.identity_from_spectra(lam, mu[js])
    assert np.max(np.abs(W[:, js] - W_log)) < 1e-13 * max(1, n / 16)


@pytest.mark.parametrize("g", [1e-150, 1e-160, 1e-200, 1e-300, 5e-320])
def test_graded_diagonal_spectra(g):
    announce(f"identity kernel, graded diagonal g={g}")
    lam = np.array([g, 2 * g, 3 * g, 1.0])
    mu = np.array([np.delete(lam, j) for j in range(4)])
    W, flag = gpu_components(lam, mu)
    assert flag == 0
    np.testing.assert_array_equal(W, np.eye(4))


@pytest.mark.parametrize("k", [332, 531, 830, 1020])
def test_graded_block_spectra(k):
    announce(f"identity kernel, graded blocks 2^-{k}")
    lam, mu, W_exp = graded_block_spectra(k)
    W, flag = gpu_components(lam, mu)
    assert flag == 0
    np.testing.assert_array_equal(W, identity_model(lam, mu))
    assert np.max(np.abs(W - W_exp)) < 1e-13
    W_o, _ = oracle.identity_from_spectra(lam, mu)
    assert np.max(np.abs(W - W_o)) < 10 * 11 * 2.3e-16 * k * math.log(2)   # the log sums' own rounding


def test_spectra_near_the_top_of_the_range():
    announce("identity kernel, spectra scaled by 2^1022")
    n = 40
    A = inputs.goe(n, 77)
    lam = oracle.eigvalsh(A, "lapack")
    mu = oracle.minor_spectra(A, range(n), "lapack")
    s = 2.0 ** 1022 / np.max(np.abs(lam))
    s = 2.0 ** np.floor(np.log2(s))              # a power of two: the scaled spectra are exact
    W1, _ = gpu_components(lam, mu)
    W2, flag = gpu_components(lam * s, mu * s)
    assert flag == 0 and np.all(np.isfinite(W2))
    np.testing.assert_array_equal(W2[:, [0, n - 1]], identity_model(lam * s, (mu * s)[[0, n - 1]]))
    assert np.max(np.abs(W2 - W1)) < 1e-13


def test_bounded_wait_gives_up_and_flags():
    """EEID_SPIN_LIMIT=0 (read by eeid_create): the first wait of the bulge
    chase that is not satisfied at once gives up; the launch ends normally and
    the matrix is flagged."""
    import torch
    from paper_2002_04989_amd import eeid
    lib = eeid.load_library()
    announce("bounded wait: spin limit 0 on a fresh handle, band32_nt256x2, GOE n=256")
    old = os.environ.get("EEID_SPIN_LIMIT")
    os.environ["EEID_SPIN_LIMIT"] = "0"
    h = ctypes.c_void_p()
    try:
        assert lib.eeid_create(ctypes.byref(h), 0) == 0
    finally:
        if old is None:
            del os.environ["EEID_SPIN_LIMIT"]
        else:
            os.environ["EEID_SPIN_LIMIT"] = old
    try:
        assert lib.eeid_set_variant(h, eeid.VARIANTS.index("band32_nt256x2")) == 0
        n = 256
        A = torch.from_numpy(inputs.goe(n, 9)).to("cuda:0")
        lam = torch.empty(n, dtype=torch.float64, device="cuda:0")
        mu = torch.empty(n * (n - 1), dtype=torch.float64, device="cuda:0")
        flags = torch.empty(1, dtype=torch.int32, device="cuda:0")
        torch.cuda.synchronize()
        nn, off = (ctypes.c_int64 * 1)(n), (ctypes.c_int64 * 1)(0)
        st = lib.eeid_minor_eigvals(h, eeid.R64, eeid.PREC["fp64"], 1, nn, off, A.data_ptr(), lam.data_ptr(),
                                    mu.data_ptr(), flags.data_ptr())
        assert st == 0
        assert lib.eeid_destroy(h) == 0      # synchronises the handle's stream
        h = None
        torch.cuda.synchronize()
        assert int(flags.cpu()[0]) & eeid.FLAG_WAIT_TIMEOUT
    finally:
        if h is not None:
            lib.eeid_destroy(h)
    # the default handle (spin limit 2^26) is unaffected
    from tests.gpu_util import run_all
    _, _, _, flag = run_all([inputs.goe(n, 9)])[0]
    assert flag == 0


@pytest.mark.parametrize("form", ["products", "paired"])
@pytest.mark.parametrize("n", [2, 300, 517])
def test_eigenvector_sq_is_the_row_of_w(n, form):
    import torch
    from paper_2002_04989_amd import eeid
    announce(f"eigenvector_sq n={n} {form}")
    A = inputs.goe(n, 900 + n)
    lam = oracle.eigvalsh(A, "lapack")
    mu = oracle.minor_spectra(A, range(n), "lapack")
    W, _ = gpu_components(lam, mu, form)
    dl = torch.from_numpy(lam).to("cuda:0")
    dm = torch.from_numpy(mu.reshape(-1)).to("cuda:0")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    eeid.set_identity_form(form)
    try:
        rows = {i: eeid.eigenvector_sq(dl, dm, i, flag) for i in sorted({0, n // 2, n - 1})}
        torch.cuda.synchronize()
    finally:
        eeid.set_identity_form("products")
    assert int(flag.cpu()[0]) == 0
    for i, row in rows.items():
        np.testing.assert_array_equal(row.cpu().numpy(), W[i])
    W_log, _ = oracle.identity_from_spectra(lam, mu)
    for i, row in rows.items():
        assert np.max(np.abs(row.cpu().numpy() - W_log[i])) < 1e-13 * max(1, n / 16)


def test_eigenvector_sq_degenerate_row():
    import torch
    from paper_2002_04989_amd import eeid
    announce("eigenvector_sq degenerate")
    lam = torch.tensor([1.0, 1.0, 3.0], dtype=torch.float64, device="cuda:0")
    mu = torch.tensor([1.0, 3.0, 1.0, 3.0, 1.0, 1.0], dtype=torch.float64, device="cuda:0")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    r0 = eeid.eigenvector_sq(lam, mu, 0, flag).cpu().numpy()
    r2 = eeid.eigenvector_sq(lam, mu, 2, flag).cpu().numpy()
    assert np.all(np.isnan(r0)) and np.all(np.isfinite(r2)) and int(flag.cpu()[0]) & 2
