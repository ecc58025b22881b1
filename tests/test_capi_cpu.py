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
    # batched apply: null factor, nrhs and schedule out of range
    for nrhs, sched in ((1, 0), (9, 0), (1, 3)):
        assert lib.srw_apply_batched(None, nrhs, None, None, sched, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrw.so not built")
def test_budget_entry_points_reject_bad_arguments_without_gpu():
    lib = ctypes.CDLL(LIB)
    P, I64, I32, D, F = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_float
    lib.srw_ordering.argtypes = [I64, ctypes.c_uint64, P, P]
    lib.srw_mlp_budgets.argtypes = [P, I64, D, I32, I32, P, P]
    lib.srw_mlp_train_step.argtypes = [P, P, P, I32, F, P, P, P, I64, P, P, P]
    lib.srw_mlp_forward.argtypes = [P, P, P, I64, P, P]
    lib.srw_budget_labels.argtypes = [P, I32, P, P]
    lib.srw_row_features.argtypes = [P, P, P, P]
    assert lib.srw_ordering(-1, 0, None, None) == -1
    assert lib.srw_ordering(10, 0, None, None) == -1          # no output
    assert lib.srw_ordering(0, 0, None, None) == 0            # empty: nothing to do
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails its checks first
    assert lib.srw_mlp_budgets(fake, 4, 0.0, 1, 8, fake, None) == -1   # eps <= 0
    assert lib.srw_mlp_budgets(fake, 4, 0.1, 0, 8, fake, None) == -1   # lo < 1
    assert lib.srw_mlp_budgets(fake, 4, 0.1, 9, 8, fake, None) == -1   # hi < lo
    assert lib.srw_mlp_budgets(fake, 4, 0.1, 1, 9000, fake, None) == -1  # hi > 8192
    assert lib.srw_mlp_budgets(None, 4, 0.1, 1, 8, fake, None) == -1
    # Adam moments must come as a pair, with step >= 1 and lr > 0
    assert lib.srw_mlp_train_step(fake, fake, None, 1, 1e-3, fake, fake, fake, 4, None, None, None) == -1
    assert lib.srw_mlp_train_step(fake, fake, fake, 0, 1e-3, fake, fake, fake, 4, None, None, None) == -1
    assert lib.srw_mlp_train_step(fake, fake, fake, 1, 0.0, fake, fake, fake, 4, None, None, None) == -1
    assert lib.srw_mlp_train_step(fake, None, None, 1, 1e-3, fake, None, fake, 4, None, None, None) == -1
    assert lib.srw_mlp_forward(fake, fake, fake, -1, fake, None) == -1
    assert lib.srw_mlp_forward(fake, None, fake, 4, fake, None) == -1
    assert lib.srw_budget_labels(None, 0, fake, None) == -1
    assert lib.srw_row_features(None, fake, fake, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrw.so not built")
def test_walk_reuse_options_rejected_without_gpu():
    """srw_options.reuse: only 0 or 1, and not with per-walk records (keep = 2) or a
    refill period other than 8; checked before any device call."""
    from paper_math_0609672_amd import srw
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p

    class Csr(ctypes.Structure):
        _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", P), ("col", P),
                    ("val", P)]

    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the option checks fail first
    A = Csr(4, 4, fake, fake, fake)
    out = ctypes.c_void_p(0)
    for fields in (dict(reuse=2), dict(reuse=-1), dict(reuse=1, keep=2),
                   dict(reuse=1, refill_period=4), dict(reuse=1, refill_period=1)):
        opt = srw._Options()
        lib.srw_default_options(ctypes.byref(opt))
        assert opt.reuse == 0
        for k, v in fields.items():
            setattr(opt, k, v)
        st = lib.srw_build_factor(ctypes.byref(A), 8, ctypes.c_double(0.0), ctypes.c_uint64(0),
                                  ctypes.byref(opt), ctypes.byref(out), None)
        assert st == -1, fields


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrw.so not built")
def test_walk_waves_option_range_without_gpu():
    """srw_options.walk_waves: 0 (default) or 4..64 waves per CU; others rejected
    before any device call."""
    from paper_math_0609672_amd import srw
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p

    class Csr(ctypes.Structure):
        _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", P), ("col", P),
                    ("val", P)]

    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the option checks fail first
    A = Csr(4, 4, fake, fake, fake)
    out = ctypes.c_void_p(0)
    opt = srw._Options()
    lib.srw_default_options(ctypes.byref(opt))
    assert opt.walk_waves == 0
    for w in (-1, 1, 3, 65, 1 << 20):
        opt.walk_waves = w
        st = lib.srw_build_factor(ctypes.byref(A), 8, ctypes.c_double(0.0), ctypes.c_uint64(0),
                                  ctypes.byref(opt), ctypes.byref(out), None)
        assert st == -1, w


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsrw.so not built")
def test_solve_order_option_range_without_gpu():
    """srw_options.solve_order: 0 rank, 1 level, 2 automatic (the default)."""
    from paper_math_0609672_amd import srw
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p

    class Csr(ctypes.Structure):
        _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", P), ("col", P),
                    ("val", P)]

    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the option checks fail first
    A = Csr(4, 4, fake, fake, fake)
    out = ctypes.c_void_p(0)
    opt = srw._Options()
    lib.srw_default_options(ctypes.byref(opt))
    assert opt.solve_order == 2
    for v in (-1, 3, 7):
        opt.solve_order = v
        st = lib.srw_build_factor(ctypes.byref(A), 8, ctypes.c_double(0.0), ctypes.c_uint64(0),
                                  ctypes.byref(opt), ctypes.byref(out), None)
        assert st == -1, v
