"""Host-only checks of the C ABI boundary (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2002_04989_amd import eeid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eeid.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const char \*|eeid_status_t|int)\s*(eeid_\w+)\s*\(", text, re.M)))


def test_header_compiles_as_c99(tmp_path):
    src = tmp_path / "use.c"
    src.write_text('#include "eeid.h"\nint main(void){ eeid_handle_t h = 0; (void)h; return EEID_OK; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    "-c", str(src), "-o", str(tmp_path / "use.o")], check=True)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(eeid.EXPORTS), names
    lib = eeid.load_library()
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", eeid.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    for name in names:
        assert re.search(rf"\bT {name}$", out, re.M), name


def test_library_is_gfx950():
    """The fat binary of our own build carries a gfx950 code object."""
    data = open(eeid.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_status_strings_cover_every_code():
    lib = eeid.load_library()
    for code in range(6):
        s = lib.eeid_status_string(code).decode()
        assert s.startswith(eeid.STATUS[code]), s
    assert b"unknown" in lib.eeid_status_string(99)


def test_null_handle_is_invalid_argument():
    lib = eeid.load_library()
    n = (ctypes.c_int64 * 1)(4)
    off = (ctypes.c_int64 * 1)(0)
    assert lib.eeid_minor_eigvals(None, 0, 0, 1, n, off, None, None, None, None) == 1
    assert lib.eeid_components(None, 1, n, None, None, None, None) == 1
    assert lib.eeid_destroy(None) == 1
    assert lib.eeid_set_stream(None, None) == 1
    assert lib.eeid_last_error(None) == b""
    assert lib.eeid_create(None, 0) == 1
    assert lib.eeid_set_variant(None, 0) == 1


def test_variant_table_matches_binding():
    lib = eeid.load_library()
    assert lib.eeid_variant_count() == len(eeid.VARIANTS)


def test_no_device_is_reported(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = eeid.load_library()
    h = ctypes.c_void_p()
    assert lib.eeid_create(ctypes.byref(h), 0) == 2
    assert not h.value


def test_no_cpu_fallback_in_binding():
    """The binding is marshalling only: it must not import the oracle or numpy linear algebra."""
    src = open(eeid.__file__).read()
    assert "oracle" not in src and "linalg" not in src and "numpy" not in src
