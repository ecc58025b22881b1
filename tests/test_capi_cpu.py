"""CPU-side checks of the C ABI: the library loads and exports every declared entry
point (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srw.h")
LIB = os.path.join(ROOT, "paper_math_0609672_amd", "libsrw.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("srw_build_factor", "srw_pcg_solve", "srw_factor_free", "srw_factor_info",
                 "srw_factor_export", "srw_tally_export", "srw_status_string"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrw.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrw.so not built")
def test_status_strings_and_argument_checks_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.srw_status_string.restype = ctypes.c_char_p
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.srw_status_string(code).startswith(b"SRW_")
    # null output handle / null matrix are rejected before any device call
    assert lib.srw_build_factor(None, 64, ctypes.c_double(0.0), ctypes.c_uint64(0), None, None, None) == -1
    out = ctypes.c_void_p(0)
    assert lib.srw_build_factor(None, 64, ctypes.c_double(0.0), ctypes.c_uint64(0), None,
                                ctypes.byref(out), None) == -1
    assert lib.srw_factor_info(None, None, None, None, None, None, None, None, None) == -1
