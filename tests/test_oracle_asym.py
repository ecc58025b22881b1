"""Pins of the oracle's asymmetric path (Section 7.1): two walk games, the LDU of
rev(A), and BiCGSTAB.

References independent of the walk code: dense Schur complements and scipy's LU of
the reverse-ordered matrix (the exact factors and eqs. y2 / y3), the absorbing
chains of both games (oracle/dense.py), scipy's BiCGSTAB iterates, direct solves.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as O
from oracle import dense
from paper_math_0609672_amd import workloads as W

Z = 5.0


def small_asym(dims=(4, 3, 3), seed=1, ground_frac=0.1, skew=0.6):
    return W.grid_asym(dims, g=("uniform", 0.5, 2.0), skew=skew, ground_frac=ground_frac,
                       excess=("uniform", 0.2, 1.0), seed=seed)


def exact_ldu_by_lu(A: np.ndarray, rk: np.ndarray):
    """(Y_A, D, Y_T) from scipy's LU of rev(P A P^T), P sorting nodes by rank: rev = L U,
    D = diag(U); in rank order A = (J L J)(J D J)(J D^{-1} U J)."""
    n = A.shape[0]
    by_rank = np.argsort(rk)
    B = dense.rev(A[np.ix_(by_rank, by_rank)])
    P, L, U = sla.lu(B)
    assert np.allclose(P, np.eye(n))  # diagonally dominant by columns: no pivoting
    d = np.diag(U).copy()
    U1 = U / d[:, None]
    node = by_rank[::-1]
    # A[node[a], node[b]] = sum_c L[a, c] d[c] U1[c, b] = sum_m Y_T[m, i] D[m] Y_A[m, j]
    Ya, Yt, D = np.eye(n), np.eye(n), np.zeros(n)
    for c in range(n):
        D[node[c]] = d[c]
        for a in range(c + 1, n):
            Ya[node[c], node[a]] = U1[c, a]
            Yt[node[c], node[a]] = L[a, c]
    return Ya, D, Yt


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_two_game_factors(seed):
    """Eqs. y2 and y3: the limit of the game of A gives the unit lower factor Y_A and D,
    the limit of the game of A^T the factor Y_T with A = Y_T^T D Y_A in rank order; the
    two games' D agree (Section 7.1 footnote); scipy's LU gives the same factors."""
    A = small_asym(seed=seed).dense()
    assert not np.allclose(A, A.T)
    rk = O.rank(A.shape[0], seed + 3)
    Ya, Da = dense.exact_factor_schur(A, rk)
    Yt, Dt = dense.exact_factor_schur(A.T, rk)
    assert np.allclose(Da, Dt, rtol=1e-12)
    assert np.allclose(Yt.T @ np.diag(Da) @ Ya, A, atol=1e-12 * np.abs(A).max())
    La, Dl, Lt = exact_ldu_by_lu(A, rk)
    assert np.allclose(La, Ya, atol=1e-12) and np.allclose(Lt, Yt, atol=1e-12)
    assert np.allclose(Dl, Da, rtol=1e-12)


def test_validate_asym():
    A = small_asym()
    assert O.validate_asym(A) == O.OK
    assert O.validate(A) == O.E_NOT_RMATRIX  # the symmetric check rejects it
    S = W.config_grid2d_32(0)
    assert O.validate_asym(S) == O.OK        # a symmetric R-matrix passes both
    D = A.dense()
    # a column sum above the diagonal (rows still dominant)
    B = D.copy()
    j = 5
    i = next(i for i in range(B.shape[0]) if i != j and B[i, j] != 0)
    B[i, j] -= 10.0
    B[i, i] += 10.0
    assert O.validate_asym(W.from_dense(B)) == O.E_NOT_RMATRIX
    # a row sum above the diagonal
    assert O.validate_asym(W.from_dense(B.T.copy())) == O.E_NOT_RMATRIX
    # a structurally asymmetric entry
    C = D.copy()
    i, j = np.argwhere((C == 0))[0]
    C[i, j] = -1e-3
    C[i, i] += 1.0
    C[j, j] += 1.0
    assert O.validate_asym(W.from_dense(C)) == O.E_NOT_RMATRIX
    # no positive column excess anywhere (rows still have it): singular game of A^T
    n = 4
    E = np.array([[3.0, -1.0, 0, 0], [-2.0, 3.0, -1.0, 0], [0, -2.0, 3.0, -1.0], [0, 0, -2.0, 2.0]])
    # column sums: 3-2 = 1 (excess 1), 3-1-2 = 0, 3-1-2 = 0, 2-1 = 1 -> make all zero
    E[0, 0] = 2.0
    E[3, 3] = 1.0 + 1e-9
    assert O.validate_asym(W.from_dense(E)) in (O.E_NOT_RMATRIX, O.E_SINGULAR)


def test_symmetric_matrix_gives_one_factor_twice():
    A = W.config_grid2d_32(0)
    F = O.build_factor_ldu(A, 40, 1e-3, 7)
    for f in ("yptr", "ycol", "yval", "d"):
        assert np.array_equal(getattr(F.a, f), getattr(F.t, f))
    P = O.build_factor(A, 40, 1e-3, 7)
    r = np.random.default_rng(0).standard_normal(A.n)
    assert np.array_equal(O.apply_ldu(F, r), O.apply(P, r))


@pytest.mark.parametrize("seed", [0, 5])
def test_ldu_factor_converges_to_exact(seed):
    A = small_asym(seed=seed)
    Ad = A.dense()
    rk = O.rank(A.n, seed)
    M = 40000
    F = O.build_factor_ldu(A, M, 0.0, seed + 1, rk=rk)
    for Fg, Ag in ((F.a, Ad), (F.t, Ad.T)):
        Ye, De = dense.exact_factor_schur(Ag, rk)
        Y = Fg.dense_y()
        tau = Fg.table.tau
        for k in range(A.n):
            lim = dense.walk_limits(Ag, rk, k)
            for i in range(A.n):
                if rk[i] >= rk[k]:
                    assert Y[k, i] == (1.0 if i == k else 0.0)
                    continue
                p = lim["p"][i] if lim["p"] is not None else 0.0
                sd = tau[k] * np.sqrt(max(p * (1 - p), 1e-12) / M)
                assert abs(Y[k, i] - Ye[k, i]) <= Z * sd + 1e-13, (k, i)
    # and the preconditioner approaches A^{-1}
    r = np.random.default_rng(1).standard_normal(A.n)
    z = O.apply_ldu(F, r)
    assert np.linalg.norm(Ad @ z - r) <= 0.05 * np.linalg.norm(r)


def test_bicgstab_matches_scipy_iterates():
    A = small_asym(dims=(6, 5, 4), seed=3, ground_frac=0.05)
    S = A.to_scipy()
    b = np.random.default_rng(4).standard_normal(A.n)
    F = O.build_factor_ldu(A, 64, 1e-3, 2)
    for pre in (None, F):
        xs = []
        M = None if pre is None else spla.LinearOperator((A.n, A.n), matvec=lambda v: O.apply_ldu(F, v))
        spla.bicgstab(S, b, rtol=0.0, atol=1e-300, maxiter=6, M=M, callback=lambda xk: xs.append(xk.copy()))
        for k in range(1, 6):
            st, x, it, _ = O.bicgstab(A, pre, b, 0.0, k)
            assert it == k and st == O.NOT_CONVERGED
            assert np.allclose(x, xs[k - 1], rtol=1e-11, atol=1e-12 * np.abs(xs[k - 1]).max())


def test_bicgstab_solutions():
    A = small_asym(dims=(7, 6, 5), seed=4, ground_frac=0.05)
    Ad = A.dense()
    b = np.random.default_rng(5).standard_normal(A.n)
    xd = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    st, x, it, rel = O.bicgstab(A, None, b, 1e-10)
    assert st == O.OK and rel <= 1e-10
    assert np.linalg.norm(x - xd) <= kappa * 1e-10 * np.linalg.norm(xd) * 10
    F = O.build_factor_ldu(A, 128, 1e-4, 1)
    st2, x2, it2, rel2 = O.bicgstab(A, F, b, 1e-10)
    assert st2 == O.OK and rel2 <= 1e-10 and it2 < it
    # the exact factors as preconditioner: one (half) iteration
    rk = O.rank(A.n, 1)
    E = O.build_factor_ldu(A, 1, 0.0, 1, rk=rk)
    Ya, Da = dense.exact_factor_schur(Ad, rk)
    Yt, _ = dense.exact_factor_schur(Ad.T, rk)
    for Fg, Y in ((E.a, Ya), (E.t, Yt)):
        rows, cols = np.nonzero((np.abs(Y) > 0) & ~np.eye(A.n, dtype=bool))
        Fg.yptr = np.zeros(A.n + 1, np.int64)
        np.cumsum(np.bincount(rows, minlength=A.n), out=Fg.yptr[1:])
        order = np.lexsort((cols, rows))
        Fg.ycol = cols[order].astype(np.int32)
        Fg.yval = Y[rows[order], cols[order]]
    E.a.d = Da.copy()
    st3, x3, it3, rel3 = O.bicgstab(A, E, b, 1e-10)
    assert st3 == O.OK and it3 == 1


def test_zero_rhs():
    A = small_asym()
    st, x, it, rel = O.bicgstab(A, None, np.zeros(A.n), 1e-10)
    assert st == O.OK and it == 0 and not x.any()
