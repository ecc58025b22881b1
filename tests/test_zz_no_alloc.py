"""srw_apply_noalloc against srw_apply (through the C ABI).

The allocation-free entry point runs the same kernels as srw_apply with its work
vectors in the library's static scratch, so its result must equal srw_apply's bit for
bit.  Two calls in a row, the second on a smaller factor (the scratch keeps the first
call's contents), then a two-game factor and an FP32 factor, then a factor over the
size limit, which must be refused with SRW_E_ARG before any work.
"""
import numpy as np
import pytest

from paper_math_0609672_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def srw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_math_0609672_amd import srw as s
    return s


def np_(t):
    return t.detach().cpu().numpy()


def test_noalloc_apply_equals_apply(srw):
    big = W.grid((40, 40, 40), g=("loguniform", 1e-2, 1e2), ground_frac=0.01,
                 excess=("uniform", 0.01, 1.0), seed=3)
    small = W.config_grid2d_32(0)
    asym = W.config_grid3d_asym(16, 0)
    cases = [(big, "sym", "fp64"), (small, "sym", "fp64"), (asym, "ldu", "fp64"),
             (small, "sym", "fp32")]
    for i, (A, kind, prec) in enumerate(cases):
        M = srw.Matrix.from_host(A, DEV)
        build = srw.build_factor_ldu if kind == "ldu" else srw.build_factor
        F = build(M, 64, 1e-4, 7 + i, precision=prec)
        r = torch.as_tensor(np.random.default_rng(i).standard_normal(A.n), device=DEV)
        want = np_(srw.apply(F, r))
        for _ in range(2):
            got = np_(srw.apply_noalloc(F, r))
            assert np.array_equal(got, want), (i, kind, prec)
        assert np.all(np.isfinite(got))
        F.free()


def test_noalloc_apply_refuses_factor_over_the_limit(srw):
    n = srw.NOALLOC_MAX_N + 1
    empty = np.zeros(0, np.int64)
    A = W.assemble(n, empty, empty, np.zeros(0), np.ones(n))  # diagonal: no walks
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, 1, 0.0, 0)
    r = torch.ones(n, dtype=torch.float64, device=DEV)
    z = torch.zeros_like(r)
    st = srw._lib.srw_apply_noalloc(F.handle, srw._ptr(r), srw._ptr(z), srw._stream(None))
    assert st == srw.E_ARG
    assert "SRW_NOALLOC_MAX_N" in srw.last_error()
    # the allocating entry point still serves it, and the next allocation-free call on a
    # factor within the limit works
    assert np.array_equal(np_(srw.apply(F, r)), np.ones(n))
    F.free()
    small = W.config_grid2d_32(0)
    Ms = srw.Matrix.from_host(small, DEV)
    Fs = srw.build_factor(Ms, 16, 1e-3, 1)
    rs = torch.as_tensor(np.random.default_rng(9).standard_normal(small.n), device=DEV)
    assert np.array_equal(np_(srw.apply_noalloc(Fs, rs)), np_(srw.apply(Fs, rs)))
    Fs.free()
