"""The triangular solves' dense head (through the C ABI): the lowest-ranked rows solved
with the explicit inverse of their diagonal block of Y.

Bars: the preconditioner matches the oracle's to 1e-12 (relative, as every apply test)
for head sizes from one row to all of them and ragged against the 64-column chunks of
the inverse; with and without the head it agrees to 1e-13 (FP64; 1e-5 with the FP32
factor: two roundings of the same factor), and PCG takes the same iterations with
iterates within 1e-10; head_rows outside its range is refused.
"""
import numpy as np
import pytest

import oracle as O
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


def grid3d(m, seed):
    return W.grid((m, m, m), g=("loguniform", 1e-2, 1e2), ground_frac=0.01,
                  excess=("uniform", 0.01, 1.0), seed=seed)


SMALL = {
    "grid3d_12": (grid3d(12, 3), 256),
    "random_3000": (W.random_graph(3000, 9000, seed=7, ground_frac=0.01), 37),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("head_rows", [-1, 1, 63, 64, 65, 700, 16384])
def test_head_apply_matches_oracle(srw, name, head_rows):
    A, walks = SMALL[name]
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, 1e-3, 2, head_rows=head_rows)
    ref = O.build_factor(A, walks, 1e-3, 2)
    for seed in (4, 5):
        r = W.rhs(A.n, seed=seed)
        z = np_(srw.apply(F, torch.as_tensor(r, device=DEV)))
        zr = O.apply(ref, r)
        assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr), head_rows
    F.free()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
def test_head_agrees_with_substitution_mid_size(srw, precision, tol):
    """24^3 = 13,824 rows: the default head (4,096 rows) against none, in rank and in
    level order."""
    A = grid3d(24, 4)
    M = srw.Matrix.from_host(A, DEV)
    F0 = srw.build_factor(M, 64, 1e-3, 9, precision=precision, head_rows=-1)
    for order in (0, 1):
        F1 = srw.build_factor(M, 64, 1e-3, 9, precision=precision, solve_order=order)
        for seed in (8, 9):
            r = torch.as_tensor(W.rhs(A.n, seed=seed), device=DEV)
            z0, z1 = np_(srw.apply(F0, r)), np_(srw.apply(F1, r))
            assert np.linalg.norm(z1 - z0) <= tol * np.linalg.norm(z0)
        if precision == "fp64":
            b = torch.as_tensor(W.rhs(A.n, seed=10), device=DEV)
            st0, x0, it0, _ = srw.pcg_solve(M, F0, b, 1e-10)
            st1, x1, it1, _ = srw.pcg_solve(M, F1, b, 1e-10)
            assert st0 == st1 == srw.OK and it0 == it1
            x0, x1 = np_(x0), np_(x1)
            assert np.linalg.norm(x1 - x0) <= 1e-10 * np.linalg.norm(x0)
        F1.free()
    F0.free()


def test_head_pcg_matches_oracle_mid_size(srw):
    """PCG with the default head on 13,824 rows: the oracle's iteration count and its
    iterate within 1e-10."""
    A = grid3d(24, 5)
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, 64, 1e-3, 3)
    ref = O.build_factor(A, 64, 1e-3, 3)
    b = W.rhs(A.n, seed=2)
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), 1e-10)
    st_o, x_o, it_o, _ = O.pcg(A, ref, b, 1e-10)
    assert st == st_o == 0 and it == it_o
    assert np.linalg.norm(np_(x) - x_o) <= 1e-10 * np.linalg.norm(x_o)
    F.free()


def test_head_with_ic0_and_noalloc(srw):
    """IC(0) takes the head too (it shares the solve plan), and the allocation-free
    application gives srw_apply's result bit for bit."""
    A = grid3d(16, 6)
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_ic0(M)
    G = srw.build_ic0(M, head_rows=-1)
    r = torch.as_tensor(W.rhs(A.n, seed=3), device=DEV)
    z, zg = np_(srw.apply(F, r)), np_(srw.apply(G, r))
    assert np.linalg.norm(z - zg) <= 1e-13 * np.linalg.norm(zg)
    assert np.array_equal(np_(srw.apply_noalloc(F, r)), z)
    F.free()
    G.free()


def test_head_shortened_by_its_cost(srw):
    """The head's inverse costs about (head rows) x (head entries); a head that would
    pass the bound is shortened (to a multiple of 64 rows), and the preconditioner
    still agrees with the head-less one.  A plain build reports the default head."""
    A = grid3d(40, 7)  # 64,000 rows; 16,384 head rows would hold about 1.4M entries
    M = srw.Matrix.from_host(A, DEV)
    F0 = srw.build_factor(M, 256, 1e-4, 5)
    assert F0.stats()["head_rows"] == 4096
    F = srw.build_factor(M, 256, 1e-4, 5, head_rows=16384)
    G = srw.build_factor(M, 256, 1e-4, 5, head_rows=-1)
    h = F.stats()["head_rows"]
    assert 4096 <= h < 16384 and h % 64 == 0, h
    assert G.stats()["head_rows"] == 0
    r = torch.as_tensor(W.rhs(A.n, seed=6), device=DEV)
    z, zg = np_(srw.apply(F, r)), np_(srw.apply(G, r))
    assert np.linalg.norm(z - zg) <= 1e-13 * np.linalg.norm(zg)
    assert np.linalg.norm(np_(srw.apply(F0, r)) - zg) <= 1e-13 * np.linalg.norm(zg)
    for X in (F0, F, G):
        X.free()


def test_head_rows_out_of_range_refused(srw):
    A, walks = SMALL["grid3d_12"]
    M = srw.Matrix.from_host(A, DEV)
    for bad in (-2, 16385):
        with pytest.raises(srw.SrwError):
            srw.build_factor(M, walks, 1e-3, 2, head_rows=bad)
