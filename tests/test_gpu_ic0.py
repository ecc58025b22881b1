"""The paper's comparison preconditioner and workload family on the GPU (through the C
ABI): IC(0) against the oracle, and the random-walk factor on the 3D Dirichlet
Laplacians of Table 1.

Bars: the IC(0) factor bit-exact with the oracle's (both evaluate the same sums in
row k's CSR order without contraction) in natural, random and given orderings; PCG
with it takes the oracle's iterations with iterates within 1e-10.  On the 3D
Dirichlet Laplacian (diagonal 6, off-diagonal -1, excess only next to the boundary,
so every interior row is ungrounded), right-hand side all ones, tolerance 1e-6 as in
Section 6: the random-walk factor bit-exact with the oracle's and PCG iterates within
1e-10, and IC(0)-PCG likewise.
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


MATS = {
    "grid3d_12": lambda: W.grid((12, 12, 12), g=("loguniform", 1e-2, 1e2), ground_frac=0.01,
                                excess=("uniform", 0.01, 1.0), seed=3),
    "random_3000": lambda: W.random_graph(3000, 9000, seed=7, ground_frac=0.01),
    "laplace_14": lambda: W.laplace3d_dirichlet(m=14),
}


def pcg_parity(srw, A, M, F, ref, b, tol):
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), tol)
    st_o, x_o, it_o, _ = O.pcg(A, ref, b, tol)
    assert st == st_o == 0 and rel <= tol
    assert it == it_o, (it, it_o)
    assert np.linalg.norm(np_(x) - x_o) <= 1e-10 * np.linalg.norm(x_o)
    return it


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("order", ["natural", "random", "given"])
def test_ic0_bit_exact_and_pcg(srw, name, order):
    A = MATS[name]()
    M = srw.Matrix.from_host(A, DEV)
    if order == "natural":
        F = srw.build_ic0(M)
        rk = np.arange(A.n, dtype=np.int32)
    elif order == "random":
        F = srw.build_ic0(M, 5, rank=None)
        rk = O.rank(A.n, 5)
    else:
        rk = np.random.default_rng(2).permutation(A.n).astype(np.int32)
        F = srw.build_ic0(M, rank=torch.as_tensor(rk, device=DEV))
    ref = O.ic0(A, rk)
    got = {k: np_(v) for k, v in F.export().items()}
    assert np.array_equal(got["rank"], rk)
    assert np.array_equal(got["yptr"], ref.yptr) and np.array_equal(got["ycol"], ref.ycol)
    assert np.array_equal(got["yval"], ref.yval)
    assert np.array_equal(got["d"], ref.d)
    b = W.rhs(A.n, seed=1)
    pcg_parity(srw, A, M, F, ref, b, 1e-8)
    F.free()


def test_ic0_refuses_walk_options(srw):
    A = MATS["grid3d_12"]()
    M = srw.Matrix.from_host(A, DEV)
    import ctypes
    opt = srw._options("natural", None, "fp32", 0, 0, 0, False, 1, 2, False)
    h = ctypes.c_void_p(0)
    csr = M.c()
    st = srw._lib.srw_build_ic0(ctypes.byref(csr), 0, ctypes.byref(opt), ctypes.byref(h), None)
    assert st == srw.E_ARG


@pytest.mark.parametrize("m", [12, 20])
def test_laplacian_table1_family_random_walk_and_ic0(srw, m):
    A = W.laplace3d_dirichlet(m=m)
    M = srw.Matrix.from_host(A, DEV)
    b = np.ones(A.n)
    # random-walk factor, 24 walks per row, no drop (the Table 1 rerun's settings)
    F = srw.build_factor(M, 24, 0.0, 0)
    ref = O.build_factor(A, 24, 0.0, 0)
    got = {k: np_(v) for k, v in F.export().items()}
    for k in ("yptr", "ycol", "yval", "d"):
        assert np.array_equal(got[k], getattr(ref, k)), k
    it_rw = pcg_parity(srw, A, M, F, ref, b, 1e-6)
    F.free()
    # IC(0) in natural ordering, as the conventional ICCG
    G = srw.build_ic0(M)
    it_ic = pcg_parity(srw, A, M, G, O.ic0(A), b, 1e-6)
    G.free()
    assert it_rw < it_ic  # the random-walk factor, about 13 entries per row, beats IC(0)
