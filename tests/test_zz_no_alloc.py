"""eeid_components_noalloc: the identity with the library's scratch in a fixed
device array instead of allocated workspace.

Through the C ABI, against eeid_components on the same spectra (the same
kernels, so bit for bit), on two calls in a row with the second smaller than
the first (the scratch keeps the first call's contents), a batch of several
matrices, and the size limits (refused with EEID_ERR_UNSUPPORTED, nothing
enqueued).
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2002_04989_amd import eeid, inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def spectra(n, seed):
    A = inputs.goe(n, seed)
    return oracle.eigvalsh(A, "lapack"), oracle.minor_spectra(A, range(n), "lapack")


def run_both(mats_spectra):
    import torch
    n = [len(lam) for lam, _ in mats_spectra]
    lam = torch.from_numpy(np.concatenate([lam for lam, _ in mats_spectra])).to("cuda:0")
    mu = torch.from_numpy(np.concatenate([mu.reshape(-1) for _, mu in mats_spectra])).to("cuda:0")
    f1 = torch.zeros(len(n), dtype=torch.int32, device="cuda:0")
    f2 = torch.zeros(len(n), dtype=torch.int32, device="cuda:0")
    V_ref = eeid.components(lam, mu, n, f1)
    V = torch.full((sum(k * k for k in n),), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    eeid.components_noalloc(lam, mu, n, f2, V)
    torch.cuda.synchronize()
    return V.cpu().numpy(), V_ref.cpu().numpy(), f2.cpu().numpy(), f1.cpu().numpy()


def test_noalloc_matches_components_on_two_calls_the_second_smaller():
    first = [spectra(700, 1)]
    second = [spectra(129, 2)]
    for label, batch in (("n=700", first), ("n=129 after n=700", second)):
        announce(f"components_noalloc {label}")
        V, V_ref, f, f_ref = run_both(batch)
        np.testing.assert_array_equal(V, V_ref)
        np.testing.assert_array_equal(f, f_ref)
        lam, mu = batch[0]
        W_o, _ = oracle.identity_from_spectra(lam, mu[[0, len(lam) - 1]])
        W = V.reshape(len(lam), len(lam))
        assert np.max(np.abs(W[:, [0, len(lam) - 1]] - W_o)) < 1e-12


def test_noalloc_batch_and_flags():
    announce("components_noalloc batch of 5 (one degenerate)")
    batch = [spectra(n, 10 + n) for n in (1, 2, 33, 64, 300)]
    lam_deg = np.array([1.0, 1.0, 3.0])
    batch.insert(2, (lam_deg, np.array([[1.0, 2.0], [1.0, 2.0], [1.0, 1.0]])))
    V, V_ref, f, f_ref = run_both(batch)
    np.testing.assert_array_equal(V, V_ref)
    np.testing.assert_array_equal(f, f_ref)
    assert f[2] & eeid.FLAG_DEGENERATE and not np.any(np.delete(f, 2))


def test_noalloc_paired_form():
    announce("components_noalloc, paired form")
    eeid.set_identity_form("paired")
    try:
        V, V_ref, f, f_ref = run_both([spectra(300, 5), spectra(41, 6)])
    finally:
        eeid.set_identity_form("products")
    np.testing.assert_array_equal(V, V_ref)
    np.testing.assert_array_equal(f, f_ref)


def test_noalloc_limits_are_refused():
    import torch
    announce("components_noalloc limits")
    lib = eeid.load_library()
    h = eeid.handle(0)
    buf = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    flags = torch.zeros(65, dtype=torch.int32, device="cuda:0")
    ones = (ctypes.c_int64 * 65)(*([1] * 65))
    st = lib.eeid_components_noalloc(h, 65, ones, buf.data_ptr(), buf.data_ptr(), buf.data_ptr(), flags.data_ptr())
    assert st == 5 and b"EEID_NOALLOC_MAX_MATRICES" in lib.eeid_last_error(h)
    big = (ctypes.c_int64 * 3)(8192, 8192, 2)
    st = lib.eeid_components_noalloc(h, 3, big, buf.data_ptr(), buf.data_ptr(), buf.data_ptr(), flags.data_ptr())
    assert st == 5 and b"EEID_NOALLOC_MAX_EIGENVALUES" in lib.eeid_last_error(h)
    st = lib.eeid_components_noalloc(h, 1, (ctypes.c_int64 * 1)(4), None, buf.data_ptr(), buf.data_ptr(),
                                     flags.data_ptr())
    assert st == 1
