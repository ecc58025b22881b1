"""Pins of the oracle's IC(0), the incomplete Cholesky preconditioner of the paper's
ICCG comparisons (Section 6, Tables 1-2), held in the factor's form A ~ Y^T D Y.

What fixes IC(0) independently of how it is computed:
  - zero fill-in: Y keeps exactly the lower-ranked neighbours of each row;
  - the defining property of the incomplete factorization: (Y^T D Y)_ij = A_ij on
    every position of A's pattern, diagonal included (the error lives only off it);
  - a tree (a path in any ordering, eliminated leaves first) has no fill, so there
    IC(0) is the complete factorization: Y^T D Y = A;
  - the classical constant-coefficient limits: far from the boundary the pivots of
    the 2D 5-point and 3D 7-point Laplacians in natural ordering solve d = 4 - 2/d and
    d = 6 - 3/d, i.e. d = 2 + sqrt(2) and d = 3 + sqrt(6);
  - an M-matrix keeps its sign pattern: D > 0, Y <= 0.
"""
import numpy as np
import pytest

import oracle as O
from paper_math_0609672_amd import workloads as W


def check_pattern_property(A, F, tol=1e-13):
    Ad = A.dense()
    Y = F.dense_y()
    M = Y.T @ np.diag(F.d) @ Y
    mask = Ad != 0
    scale = np.abs(Ad).max()
    assert np.max(np.abs(M - Ad)[mask]) <= tol * scale
    return M, Ad


@pytest.mark.parametrize("case", ["grid2d", "grid3d", "random", "laplace"])
@pytest.mark.parametrize("order", ["natural", "random"])
def test_ic0_matches_A_on_its_pattern(case, order):
    A = {"grid2d": lambda: W.grid((9, 7), g=("uniform", 0.1, 10.0), ground_frac=0.05,
                                  excess=("uniform", 0.1, 1.0), seed=1),
         "grid3d": lambda: W.grid((5, 4, 6), g=("loguniform", 1e-2, 1e2), ground_frac=0.05,
                                  excess=("uniform", 0.01, 1.0), seed=2),
         "random": lambda: W.random_graph(60, 200, seed=3, ground_frac=0.1),
         "laplace": lambda: W.laplace3d_dirichlet(m=5)}[case]()
    rk = None if order == "natural" else O.rank(A.n, 5)
    F = O.ic0(A, rk)
    rank = np.arange(A.n) if rk is None else rk
    # zero fill-in: row k holds exactly its lower-ranked neighbours
    for k in range(A.n):
        nb = [j for j in A.col[A.rowptr[k]:A.rowptr[k + 1]] if j != k and rank[j] < rank[k]]
        assert list(F.ycol[F.yptr[k]:F.yptr[k + 1]]) == sorted(nb)
    check_pattern_property(A, F)
    assert np.all(F.d > 0) and np.all(F.yval <= 0)


def test_ic0_of_a_path_is_the_complete_factorization():
    # natural ordering eliminates from node n-1 down: each eliminated node is the end
    # of the remaining path, a leaf, so nothing fills in and IC(0) is complete
    n = 40
    rng = np.random.default_rng(0)
    g = rng.uniform(0.5, 2.0, n - 1)
    i = np.arange(n - 1)
    exc = np.zeros(n)
    exc[[0, 17]] = [0.3, 0.2]
    A = W.assemble(n, i, i + 1, g, exc)
    F = O.ic0(A)
    Y = F.dense_y()
    Ad = A.dense()
    assert np.allclose(Y.T @ np.diag(F.d) @ Y, Ad, rtol=0, atol=1e-13 * np.abs(Ad).max())
    # with a random ordering the path fills in: only the pattern property holds
    check_pattern_property(A, O.ic0(A, O.rank(n, 1)))


@pytest.mark.parametrize("dims,limit", [((60, 60), 2.0 + np.sqrt(2.0)), ((24, 24, 24), 3.0 + np.sqrt(6.0))])
def test_ic0_interior_pivots_reach_the_constant_coefficient_limit(dims, limit):
    A = laplace2d(dims[0]) if len(dims) == 2 else W.laplace3d_dirichlet(m=dims[0])
    F = O.ic0(A)
    # the first-eliminated (highest) nodes carry the boundary; the pivots deep inside
    # the elimination have converged to the fixed point
    d = F.d.reshape(dims)
    inner = d[tuple(slice(2, 6) for _ in dims)]
    assert np.all(np.abs(inner - limit) <= 1e-10 * limit), (inner.min(), inner.max(), limit)


def laplace2d(m):
    """5-point Dirichlet Laplacian on an m x m grid: diagonal 4, off-diagonal -1."""
    idx = np.arange(m * m).reshape(m, m)
    src = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    dst = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    deg = np.zeros(m * m)
    np.add.at(deg, src, 1)
    np.add.at(deg, dst, 1)
    return W.assemble(m * m, src, dst, np.ones(src.size), 4.0 - deg)


def test_ic0_pcg_converges_faster_than_cg():
    A = W.laplace3d_dirichlet(m=12)
    b = np.ones(A.n)
    F = O.ic0(A)
    st, x, it, rel = O.pcg(A, F, b, 1e-6)
    st0, x0, it0, rel0 = O.pcg(A, None, b, 1e-6)
    assert st == st0 == 0 and rel <= 1e-6
    assert it < it0
