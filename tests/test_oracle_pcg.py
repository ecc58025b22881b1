"""Pins of the oracle's preconditioner application and PCG (Algorithm 1, Section 6)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle import dense
from paper_math_0609672_amd import metrics, workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_oracle_factor(A, rk):
    """Oracle Factor whose Y, D are the dense exact factor (no walks)."""
    Ye, De = dense.exact_factor_schur(A.dense(), rk)
    n = A.n
    yptr = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for k in range(n):
        nz = [i for i in range(n) if i != k and Ye[k, i] != 0.0]
        cols += nz
        vals += [Ye[k, i] for i in nz]
        yptr[k + 1] = len(cols)
    return O.Factor(n, rk, yptr, np.array(cols, np.int32), np.array(vals), De)


def test_exact_preconditioner_converges_in_one_iteration():
    A = W.random_graph(30, 60, seed=2)
    rk = O.rank(A.n, 1)
    F = exact_oracle_factor(A, rk)
    b = W.rhs(A.n, seed=3)
    z = O.apply(F, b)
    assert np.allclose(A.dense() @ z, b, atol=1e-11)
    st, x, it, rr = O.pcg(A, F, b, 1e-10)
    assert st == 0 and it == 1 and rr < 1e-10


def test_identity_preconditioner_is_cg():
    A = W.config_grid2d_32()
    b = W.rhs(A.n, seed=0)
    xs = []
    spla.cg(A.to_scipy(), b, x0=np.zeros(A.n), rtol=1e-30, atol=0.0, maxiter=12,
            callback=lambda xk: xs.append(xk.copy()))
    for k in (1, 2, 5, 12):
        st, x, it, rr = O.pcg(A, None, b, 1e-30, max_iter=k)
        assert st == O.NOT_CONVERGED and it == k
        assert np.linalg.norm(x - xs[k - 1]) <= 1e-12 * np.linalg.norm(xs[k - 1])


@pytest.mark.parametrize("tol", [1e-6, 1e-8, 1e-10])
def test_pcg_solution_against_direct_solve(tol):
    A = W.config_grid2d_32()
    F = O.build_factor(A, 64, 1e-3, 0)
    b = W.rhs(A.n, seed=0)
    st, x, it, rr = O.pcg(A, F, b, tol)
    Ad = A.dense()
    xd = np.linalg.solve(Ad, b)
    assert st == 0 and rr <= tol
    assert np.isclose(rr, np.linalg.norm(b - Ad @ x) / np.linalg.norm(b), rtol=1e-6)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(x - xd) <= kappa * tol * np.linalg.norm(xd)
    # the walk preconditioner beats plain CG by a wide margin
    _, _, it_cg, _ = O.pcg(A, None, b, tol)
    assert it < it_cg / 4


def test_zero_rhs_and_iteration_cap():
    A = W.config_grid2d_32()
    F = O.build_factor(A, 8, 0.0, 0)
    st, x, it, rr = O.pcg(A, F, np.zeros(A.n), 1e-8)
    assert st == 0 and it == 0 and rr == 0.0 and not x.any()
    st, x, it, rr = O.pcg(A, F, W.rhs(A.n), 1e-14, max_iter=3)
    assert st == O.NOT_CONVERGED and it == 3 and rr > 1e-14


def test_table1_arithmetic():
    """N, E of the 3D Dirichlet grids, C of ILU(0) = (E+N)/2 and eq. m1 reproduce the
    printed Table 1 entries to their two significant digits."""
    g = json.load(open(os.path.join(GOLDEN, "table1_3d_grids.json")))
    for row in g["rows"]:
        m = row["grid"]
        if m <= 60:
            A = W.laplace3d_dirichlet(m)
            N, E = A.n, A.nnz
        else:
            N, E = m ** 3, 7 * m ** 3 - 6 * m ** 2
        C = metrics.factor_size((E - N) // 2, N)
        for got, want in [(N, row["N"]), (E, row["E"]), (C, row["C_ilu0"]),
                          (metrics.m1(C, E, N), row["M1_ilu0"])]:
            assert abs(got - want) <= 0.05 * want, (row["name"], got, want)
    h = g["hybrid_m1_formula_check"]
    assert abs(metrics.m1(h["C"], h["E"], h["N"]) - h["M1_printed"]) <= 0.05 * h["M1_printed"]
