"""Thin ctypes binding of libeeid (include/eeid.h).

Argument marshalling only: tensors are passed as device pointers and the
current torch stream is handed to the library; every step of the computation
runs in the library's HIP kernels.  There is no CPU fallback: if the library
cannot be loaded, or no GPU is present, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libeeid.so")
PHASE_LIB_PATH = os.path.join(PKG, "libeeid_phase.so")   # the same library built with phase timers

R64, C128 = 0, 1
PREC = {"fp64": 0, "fp32": 1}
FLAG_NONFINITE_INPUT = 1
FLAG_DEGENERATE = 2
FLAG_WAIT_TIMEOUT = 4
FLAG_NO_REFERENCE = 8
STATUS = {0: "EEID_OK", 1: "EEID_ERR_INVALID_ARG", 2: "EEID_ERR_NO_DEVICE", 3: "EEID_ERR_ALLOC",
          4: "EEID_ERR_HIP", 5: "EEID_ERR_UNSUPPORTED"}

EXPORTS = (
    "eeid_create", "eeid_destroy", "eeid_set_stream", "eeid_status_string", "eeid_last_error",
    "eeid_eigvalsh_batched", "eeid_minor_eigvals", "eeid_minor_eigvals_subset",
    "eeid_components", "eeid_components_noalloc", "eeid_components_subset", "eeid_all_components",
    "eeid_set_graph_mode",
    "eeid_variant_count", "eeid_set_variant", "eeid_set_identity_form",
    "eeid_rotated_minor_eigvals", "eeid_signed_eigenvectors", "eeid_eigenvector_sq",
    "eeid_minor_eigvals_latency", "eeid_component", "eeid_phase_ticks",
    "eeid_autotune",
)
VARIANTS = ("nb32_nt512", "nb32_nt256x2", "nb16_nt512", "band32_nt512", "band32_nt256x2")


class EEIDError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {detail}")


_lib = None
_handles: dict = {}

_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


def load_library(path: str = LIB_PATH):
    """Load libeeid.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libeeid is not built ({path} missing); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    c = ctypes.c_int
    lib.eeid_create.argtypes = [ctypes.POINTER(_vp), c]
    lib.eeid_destroy.argtypes = [_vp]
    lib.eeid_set_stream.argtypes = [_vp, _vp]
    lib.eeid_status_string.argtypes = [c]
    lib.eeid_status_string.restype = ctypes.c_char_p
    lib.eeid_last_error.argtypes = [_vp]
    lib.eeid_last_error.restype = ctypes.c_char_p
    lib.eeid_eigvalsh_batched.argtypes = [_vp, c, c, ctypes.c_int64, _i64p, _i64p, _vp, _vp, _vp]
    lib.eeid_minor_eigvals.argtypes = [_vp, c, c, ctypes.c_int64, _i64p, _i64p, _vp, _vp, _vp, _vp]
    lib.eeid_minor_eigvals_subset.argtypes = [_vp, c, c, ctypes.c_int64, _vp, ctypes.c_int64, _i64p,
                                              _vp, _vp, _vp]
    lib.eeid_components.argtypes = [_vp, ctypes.c_int64, _i64p, _vp, _vp, _vp, _vp]
    lib.eeid_components_noalloc.argtypes = [_vp, ctypes.c_int64, _i64p, _vp, _vp, _vp, _vp]
    lib.eeid_all_components.argtypes = [_vp, c, c, ctypes.c_int64, _i64p, _i64p, _vp, _vp, _vp, _vp, _vp]
    lib.eeid_components_subset.argtypes = [_vp, ctypes.c_int64, _vp, ctypes.c_int64, _vp, _vp, _vp]
    lib.eeid_set_graph_mode.argtypes = [_vp, c]
    lib.eeid_set_identity_form.argtypes = [_vp, c]
    lib.eeid_minor_eigvals_latency.argtypes = [_vp, c, c, ctypes.c_int64, _vp, ctypes.c_int64, _i64p,
                                               _vp, _vp, _vp]
    lib.eeid_component.argtypes = [_vp, c, c, ctypes.c_int64, _vp, ctypes.c_int64, ctypes.c_int64, _vp, _vp]
    lib.eeid_phase_ticks.argtypes = [ctypes.POINTER(ctypes.c_ulonglong), c]
    lib.eeid_eigenvector_sq.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int64, _vp, _vp]
    lib.eeid_rotated_minor_eigvals.argtypes = [_vp, c, c, ctypes.c_int64, _vp, ctypes.c_int64, _vp, _vp]
    lib.eeid_signed_eigenvectors.argtypes = [_vp, c, ctypes.c_int64, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
    lib.eeid_variant_count.argtypes = []
    lib.eeid_variant_count.restype = c
    lib.eeid_set_variant.argtypes = [_vp, c]
    lib.eeid_autotune.argtypes = [_vp, c, c, ctypes.c_int64, _i64p, _i64p, _vp, _vp, _vp, _vp,
                                  ctypes.POINTER(c), ctypes.POINTER(ctypes.c_double)]
    for name in EXPORTS:
        if name not in ("eeid_status_string", "eeid_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, h=None):
    if status != 0:
        detail = load_library().eeid_last_error(h).decode() if h else ""
        raise EEIDError(status, detail)


def handle(device: int | None = None):
    """The library handle of a device, bound to torch's current stream."""
    import torch
    lib = load_library()
    dev = torch.cuda.current_device() if device is None else int(device)
    h = _handles.get(dev)
    if h is None:
        hp = _vp()
        _check(lib.eeid_create(ctypes.byref(hp), dev))
        h = hp
        _handles[dev] = h
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib.eeid_set_stream(h, _vp(stream)), h)
    return h


def _i64(values: Sequence[int]):
    arr = (ctypes.c_int64 * len(values))(*[int(v) for v in values])
    return arr


def _dtype_code(A):
    import torch
    if A.dtype == torch.float64:
        return R64
    if A.dtype == torch.complex128:
        return C128
    raise TypeError(f"A must be float64 or complex128, got {A.dtype}")


class Packed:
    """A batch packed once (one flat device buffer, orders, offsets), so that
    repeated calls pass the same pointers (graph mode replays them)."""

    def __init__(self, flat, n, offs):
        self.flat, self.n, self.offs = flat, n, offs


def pack(mats) -> Packed:
    return Packed(*_batch(mats))


def _batch(mats):
    """Accept one square tensor, a list of them or a Packed batch; returns (flat, n, offsets)."""
    import torch
    if isinstance(mats, Packed):
        return mats.flat, mats.n, mats.offs
    if isinstance(mats, torch.Tensor):
        mats = [mats]
    n = [int(m.shape[0]) for m in mats]
    for m in mats:
        if m.dim() != 2 or m.shape[0] != m.shape[1]:
            raise ValueError("matrices must be square")
        if not m.is_cuda:
            raise ValueError("matrices must be on a GPU")
    offs, o = [], 0
    for k in n:
        offs.append(o)
        o += k * k
    flat = mats[0].reshape(-1).contiguous() if len(mats) == 1 else torch.cat([m.reshape(-1) for m in mats])
    return flat, n, offs


def sizes(n: Sequence[int]):
    """Element counts of lambda, mu and V2 for a batch of orders n."""
    return sum(n), sum(k * (k - 1) for k in n), sum(k * k for k in n)


def eigvalsh_batched(mats, prec: str = "fp64"):
    """Ascending eigenvalues of each matrix: (lambda [sum n], flags [count])."""
    import torch
    flat, n, offs = _batch(mats)
    dev = flat.device
    lam = torch.empty(sum(n), dtype=torch.float64, device=dev)
    flags = torch.empty(len(n), dtype=torch.int32, device=dev)
    h = handle(dev.index)
    _check(load_library().eeid_eigvalsh_batched(h, _dtype_code(flat), PREC[prec], len(n), _i64(n), _i64(offs),
                                                 flat.data_ptr(), lam.data_ptr(), flags.data_ptr()), h)
    return lam, flags


def minor_eigvals(mats, prec: str = "fp64", out=None):
    """lambda(A_b) and the spectra of all minors: (lambda [sum n], mu [sum n(n-1)], flags).
    out: optional (lambda, mu, flags) tensors to write into (mu of at least one element)."""
    import torch
    flat, n, offs = _batch(mats)
    dev = flat.device
    nl, nm, _ = sizes(n)
    if out is not None:
        lam, mu, flags = out
    else:
        lam = torch.empty(nl, dtype=torch.float64, device=dev)
        mu = torch.empty(max(nm, 1), dtype=torch.float64, device=dev)
        flags = torch.empty(len(n), dtype=torch.int32, device=dev)
    h = handle(dev.index)
    _check(load_library().eeid_minor_eigvals(h, _dtype_code(flat), PREC[prec], len(n), _i64(n), _i64(offs),
                                              flat.data_ptr(), lam.data_ptr(), mu.data_ptr(), flags.data_ptr()), h)
    return lam, mu[:nm], flags


def minor_eigvals_subset(A, js: Sequence[int], prec: str = "fp64", with_lambda: bool = True):
    """lambda(A) (or None) and the spectra of the minors M_j, j in js: (lambda, mu [len(js), n-1], flag)."""
    import torch
    if not A.is_cuda or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square GPU tensor")
    A = A.contiguous()
    n = int(A.shape[0])
    dev = A.device
    lam = torch.empty(n, dtype=torch.float64, device=dev) if with_lambda else None
    mu = torch.empty((len(js), max(n - 1, 1)), dtype=torch.float64, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    h = handle(dev.index)
    _check(load_library().eeid_minor_eigvals_subset(
        h, _dtype_code(A), PREC[prec], n, A.data_ptr(), len(js), _i64(js),
        lam.data_ptr() if lam is not None else None, mu.data_ptr(), flag.data_ptr()), h)
    return lam, mu[:, :n - 1], flag


def minor_eigvals_latency(A, js: Sequence[int], prec: str = "fp64", with_lambda: bool = True):
    """As minor_eigvals_subset, each problem spread over many workgroups (few problems, low latency)."""
    import torch
    if not A.is_cuda or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square GPU tensor")
    A = A.contiguous()
    n = int(A.shape[0])
    dev = A.device
    lam = torch.empty(n, dtype=torch.float64, device=dev) if with_lambda else None
    mu = torch.empty((max(len(js), 1), max(n - 1, 1)), dtype=torch.float64, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    h = handle(dev.index)
    _check(load_library().eeid_minor_eigvals_latency(
        h, _dtype_code(A), PREC[prec], n, A.data_ptr(), len(js), _i64(js) if len(js) else None,
        lam.data_ptr() if lam is not None else None, mu.data_ptr(), flag.data_ptr()), h)
    return lam, mu[:len(js), :n - 1], flag


def component(A, i: int, j: int, prec: str = "fp64"):
    """|v_ij|^2 of one real symmetric matrix (the paper's EigenComponent(matrix, i, j)):
    (a one-element device tensor, flag)."""
    import torch
    if not A.is_cuda or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square GPU tensor")
    A = A.contiguous()
    n = int(A.shape[0])
    out = torch.empty(1, dtype=torch.float64, device=A.device)
    flag = torch.empty(1, dtype=torch.int32, device=A.device)
    h = handle(A.device.index)
    _check(load_library().eeid_component(h, _dtype_code(A), PREC[prec], n, A.data_ptr(), int(i), int(j),
                                         out.data_ptr(), flag.data_ptr()), h)
    return out, flag


def component_column(A, j: int):
    """|v_ij|^2 for every i and one j (the single-component query of Algorithm 2 for
    all i at once): lambda(A) and the spectrum of M_j on the latency path, then Eq. (2)."""
    lam, mu, flag = minor_eigvals_latency(A, [int(j)])
    W = components_subset(lam, mu, flag)
    return W[:, 0], lam, mu[0], flag


def components(lam, mu, n: Sequence[int], flags, out=None):
    """V2 [sum n^2] with V2_b[i*n_b + j] = |v_ij|^2 (Eq. (2)); updates flags in place.
    out: optional V2 tensor to write into."""
    import torch
    n = [int(k) for k in n]
    V2 = out if out is not None else torch.empty(sizes(n)[2], dtype=torch.float64, device=lam.device)
    h = handle(lam.device.index)
    _check(load_library().eeid_components(h, len(n), _i64(n), lam.data_ptr(),
                                           mu.data_ptr() if mu.numel() else None, V2.data_ptr(),
                                           flags.data_ptr()), h)
    return V2


def components_noalloc(lam, mu, n: Sequence[int], flags, V2):
    """eeid_components into a caller-provided V2, with the library allocating nothing."""
    n = [int(k) for k in n]
    h = handle(lam.device.index)
    _check(load_library().eeid_components_noalloc(h, len(n), _i64(n), lam.data_ptr(),
                                                   mu.data_ptr() if mu.numel() else None, V2.data_ptr(),
                                                   flags.data_ptr()), h)
    return V2


def components_subset(lam, mu_sel, flag):
    """Columns of Eq. (2) for selected minors of one matrix: W_sel [n, nsel], W_sel[i, s] = |v_i(j_s)|^2."""
    import torch
    n = int(lam.numel())
    nsel = int(mu_sel.shape[0])
    V2 = torch.empty((n, nsel), dtype=torch.float64, device=lam.device)
    h = handle(lam.device.index)
    mu_c = mu_sel.contiguous()
    _check(load_library().eeid_components_subset(h, n, lam.data_ptr(), nsel,
                                                  mu_c.data_ptr() if mu_c.numel() else None, V2.data_ptr(),
                                                  flag.data_ptr()), h)
    return V2


def set_graph_mode(enable: bool, device: int | None = None):
    """Graph mode for minor_eigvals, components and all_components: each argument
    set (pointers, orders, kernel configuration) is recorded into a hipGraph once
    and replayed afterwards (pass a pack()ed batch and out= buffers so that
    repeated calls present the same pointers)."""
    h = handle(device)
    _check(load_library().eeid_set_graph_mode(h, 1 if enable else 0), h)


IDENTITY_FORMS = ("products", "paired")


def set_identity_form(form: str, device: int | None = None):
    """Evaluate Eq. (2) as two products with exponents ("products", default) or
    with Algorithm 2's paired factors in [0, 1] ("paired")."""
    h = handle(device)
    _check(load_library().eeid_set_identity_form(h, IDENTITY_FORMS.index(form)), h)


def set_variant(variant, device: int | None = None):
    """Force a real-kernel configuration (name from VARIANTS or index), or None for automatic."""
    h = handle(device)
    v = -1 if variant is None else (VARIANTS.index(variant) if isinstance(variant, str) else int(variant))
    _check(load_library().eeid_set_variant(h, v), h)


def autotune(mats, prec: str = "fp64"):
    """Time every kernel configuration on this batch; the fastest is used from then on.

    Returns (variant name, milliseconds)."""
    import torch
    flat, n, offs = _batch(mats)
    dev = flat.device
    nl, nm, _ = sizes(n)
    lam = torch.empty(nl, dtype=torch.float64, device=dev)
    mu = torch.empty(max(nm, 1), dtype=torch.float64, device=dev)
    flags = torch.empty(len(n), dtype=torch.int32, device=dev)
    best = ctypes.c_int(-1)
    ms = ctypes.c_double(0.0)
    h = handle(dev.index)
    _check(load_library().eeid_autotune(h, _dtype_code(flat), PREC[prec], len(n), _i64(n), _i64(offs),
                                         flat.data_ptr(), lam.data_ptr(), mu.data_ptr(), flags.data_ptr(),
                                         ctypes.byref(best), ctypes.byref(ms)), h)
    name = "complex" if _dtype_code(flat) == C128 else VARIANTS[best.value]
    return name, ms.value


def all_components(mats, prec: str = "fp64"):
    """Every |v_ij|^2 of every matrix: (lambda, mu, V2, flags), all on the GPU."""
    import torch
    flat, n, offs = _batch(mats)
    dev = flat.device
    nl, nm, nv = sizes(n)
    lam = torch.empty(nl, dtype=torch.float64, device=dev)
    mu = torch.empty(max(nm, 1), dtype=torch.float64, device=dev)
    V2 = torch.empty(nv, dtype=torch.float64, device=dev)
    flags = torch.empty(len(n), dtype=torch.int32, device=dev)
    h = handle(dev.index)
    _check(load_library().eeid_all_components(h, _dtype_code(flat), PREC[prec], len(n), _i64(n), _i64(offs),
                                               flat.data_ptr(), lam.data_ptr(), mu.data_ptr(), V2.data_ptr(),
                                               flags.data_ptr()), h)
    return lam, mu[:nm], V2, flags


def eigenvector_sq(lam, mu, i: int, flag):
    """Row i of Eq. (2): |v_ij|^2 for every j, from lambda and all minors' spectra of one matrix."""
    import torch
    n = int(lam.numel())
    row = torch.empty(n, dtype=torch.float64, device=lam.device)
    h = handle(lam.device.index)
    _check(load_library().eeid_eigenvector_sq(h, n, lam.data_ptr(), mu.data_ptr() if mu.numel() else None, int(i),
                                               row.data_ptr(), flag.data_ptr()), h)
    return row


def rotated_minor_eigvals(A, r: int, prec: str = "fp64"):
    """Spectra of the minors at r of the n - 1 rotated matrices R^T A R: (mu_rot [n-1, n-1], flag)."""
    import torch
    if not A.is_cuda or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square GPU tensor")
    A = A.contiguous()
    n = int(A.shape[0])
    fam = 2 if _dtype_code(A) == C128 else 1
    mu_rot = torch.empty((max(fam * (n - 1), 1), max(n - 1, 1)), dtype=torch.float64, device=A.device)
    flag = torch.empty(1, dtype=torch.int32, device=A.device)
    h = handle(A.device.index)
    _check(load_library().eeid_rotated_minor_eigvals(h, _dtype_code(A), PREC[prec], n, A.data_ptr(), int(r),
                                                      mu_rot.data_ptr(), flag.data_ptr()), h)
    return mu_rot[:fam * (n - 1), :n - 1], flag


def signed_eigenvectors(A, r: int = 0, prec: str = "fp64"):
    """Unit eigenvectors with signs (phases for complex A; v_ir real >= 0) from
    Eq. (2) in the original and the rotated bases: (lambda, V [n, n] with row i
    the i-th eigenvector, float64 or complex128 like A, flags)."""
    import torch
    n = int(A.shape[0])
    t = _dtype_code(A)
    lam, mu, V2, flags = all_components(A, prec)
    mu_rot, flag_rot = rotated_minor_eigvals(A, r, prec)
    V = torch.empty((n, n), dtype=torch.complex128 if t == C128 else torch.float64, device=A.device)
    h = handle(A.device.index)
    _check(load_library().eeid_signed_eigenvectors(h, t, n, int(r), lam.data_ptr(), V2.data_ptr(),
                                                    mu_rot.data_ptr() if n > 1 else None, V.data_ptr(),
                                                    flags.data_ptr()), h)
    return lam, V, flags | flag_rot


def split(vec, n: Sequence[int], kind: str):
    """Views of a packed output per matrix: kind in {"lambda", "mu", "V2"}."""
    out, o = [], 0
    for k in n:
        if kind == "lambda":
            out.append(vec[o:o + k]); o += k
        elif kind == "mu":
            out.append(vec[o:o + k * (k - 1)].reshape(k, k - 1)); o += k * (k - 1)
        else:
            out.append(vec[o:o + k * k].reshape(k, k)); o += k * k
    return out
