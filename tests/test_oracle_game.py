"""Pins of the oracle's validation, walks, tallies and factor.

References are independent of the walk code: the absorbing Markov chain of the game
solved densely (oracle/dense.py), dense Schur complements and numpy's Cholesky of the
reverse-ordered matrix, a two-node closed form, and graph reachability.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import dense
from paper_math_0609672_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
Z = 5.0  # two-sided 5-sigma bands: ~6e-7 false-alarm rate per compared quantity


def small(n=9, edges=16, seed=3, **kw):
    return W.random_graph(n, edges, seed=seed, **kw)


# ----------------------------------------------------------------------- validation
def test_validate_accepts_r_matrices():
    assert O.validate(W.config_grid2d_32()) == O.OK
    assert O.validate(small()) == O.OK
    assert O.validate(W.laplace3d_dirichlet(4)) == O.OK


def _mut(A, fn):
    B = W.CSR(A.n, A.rowptr.copy(), A.col.copy(), A.val.copy())
    fn(B)
    return B


def test_validate_rejects():
    A = small()
    D = A.dense()
    # positive off-diagonal (kept symmetric)
    Dp = D.copy()
    i, j = np.argwhere((Dp < 0))[0]
    Dp[i, j] = Dp[j, i] = 0.5
    assert O.validate(W.from_dense(Dp)) == O.E_NOT_RMATRIX
    # asymmetric value
    Da = D.copy()
    Da[i, j] *= 1.5
    assert O.validate(W.from_dense(Da)) == O.E_NOT_RMATRIX
    # negative excess
    Dn = D.copy()
    Dn[i, i] = -Dn[i][np.arange(A.n) != i].sum() * 0.9
    assert O.validate(W.from_dense(Dn)) == O.E_NOT_RMATRIX
    # non-positive diagonal on an isolated node
    Dz = np.zeros((3, 3)); Dz[0, 0] = 1.0; Dz[1, 1] = 1.0
    assert O.validate(W.from_dense(Dz)) == O.E_NOT_RMATRIX
    # a component with no path to ground: two disconnected pairs, one ungrounded
    Ds = np.array([[2.0, -1, 0, 0], [-1, 2.0, 0, 0], [0, 0, 1.0, -1], [0, 0, -1, 1.0]])
    assert O.validate(W.from_dense(Ds)) == O.E_SINGULAR
    # unsorted columns / missing diagonal
    bad = _mut(A, lambda B: B.col.__setitem__(slice(0, 2), B.col[0:2][::-1]))
    assert O.validate(bad) == O.E_ARG
    nodiag = W.from_dense(np.array([[0.0, -1.0], [-1.0, 2.0]]))
    nodiag = W.CSR(2, np.array([0, 1, 3]), np.array([1, 0, 1], np.int32), np.array([-1.0, -1.0, 2.0]))
    assert O.validate(nodiag) == O.E_ARG


# ---------------------------------------------------------------------- dense pins
def test_rev_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "rev_example.json")))
    assert np.array_equal(dense.rev(np.array(g["input"])), np.array(g["rev"]))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_factor_two_routes_agree(seed):
    A = small(10, 18, seed=seed).dense()
    rk = O.rank(10, seed)
    Ys, Ds = dense.exact_factor_schur(A, rk)
    Yc, Dc = dense.exact_factor_cholesky(A, rk)
    assert np.allclose(Ys, Yc, atol=1e-13) and np.allclose(Ds, Dc, rtol=1e-13)
    # and A = Y^T D Y exactly in the limit (the preconditioner is A itself)
    assert np.allclose(Ys.T @ np.diag(Ds) @ Ys, A, atol=1e-12 * np.abs(A).max())
    # -Y_ki is the absorption probability at i of an unconditioned walk from k
    for k in range(10):
        lim = dense.walk_limits(A, rk, k)
        lower = rk < rk[k]
        assert np.allclose(-Ys[k, lower], lim["q"][lower], atol=1e-12)
        assert np.isclose(Ds[k], A[k, k] / lim["visits"], rtol=1e-12)


# ---------------------------------------------------------------- walk statistics
@pytest.mark.parametrize("seed", [0, 7])
def test_walk_distribution_matches_absorbing_chain(seed):
    """Ends, stays at the start and lengths of simulated walks (first step among
    motels, Section 5.2) match the absorbing chain's limits within 5 sigma."""
    A = small(9, 15, seed=seed)
    Ad = A.dense()
    rk = O.rank(A.n, seed + 100)
    tb = O.table(A, rk)
    M = 40000
    rows = np.arange(A.n)
    wk = O.walk_rows(A, rk, tb, 99, rows, M)
    checked = 0
    for r, k in enumerate(rows):
        lim = dense.walk_limits(Ad, rk, k)
        if lim["p"] is None:
            assert wk.budget[r] == 0
            continue
        s = slice(wk.rec_off[r], wk.rec_off[r + 1])
        end, vis, ln = wk.end[s], wk.visits[s].astype(float), wk.length[s].astype(float)
        for i in range(A.n):
            p = lim["p"][i]
            h = np.mean(end == i)
            assert abs(h - p) <= Z * np.sqrt(max(p * (1 - p), 1e-12) / M) + 1e-12, (k, i, h, p)
        pg = lim["p_ground"]
        assert abs(np.mean(end == -1) - pg) <= Z * np.sqrt(max(pg * (1 - pg), 1e-12) / M) + 1e-12
        assert abs(vis.mean() - lim["visits_motel"]) <= Z * vis.std() / np.sqrt(M) + 1e-12
        assert abs(ln.mean() - lim["length_motel"]) <= Z * ln.std() / np.sqrt(M) + 1e-12
        checked += 1
    assert checked >= 4


def test_tally_identities_config_grid2d():
    A = W.config_grid2d_32()
    F = O.build_factor(A, 64, 1e-3, 0)
    wk, tl, rk = F.walks, F.tallies, F.rank
    walking = F.table.tau > 0
    assert np.array_equal(wk.budget > 0, walking)
    assert np.all(wk.length >= 2)
    ends = wk.end
    starts = np.repeat(wk.rows, wk.budget)
    ok = (ends == -1) | (rk[np.maximum(ends, 0)] < rk[starts])
    assert np.all(ok)
    assert np.all(wk.visits >= 1)
    for r in np.flatnonzero(walking)[:200]:
        hs = slice(tl.h_off[r], tl.h_off[r] + tl.hlen[r])
        assert tl.walks[r] == tl.h_cnt[hs].sum() + tl.G[r]
        assert tl.J[r] >= tl.walks[r]
        assert np.all(np.diff(tl.h_end[hs]) > 0)


def test_two_node_closed_form():
    a, c, d = 3.0, 1.0, 2.0
    A = W.from_dense(np.array([[a, -c], [-c, d]]))
    rk = np.array([0, 1], np.int32)  # node 0 processed first
    M = 200000
    F = O.build_factor(A, M, 0.0, 11, rk=rk)
    Y = F.dense_y()
    assert Y[1, 0] == -c / d and F.d[1] == d  # all neighbours are homes: exact
    assert F.yptr[1] == 0  # row 0 has no lower-ranked node
    vis = F.walks.visits.astype(float)
    tau = c / a
    sd = a * tau * vis.std() / np.sqrt(M) / (1 + tau * (vis.mean() - 1)) ** 2
    assert abs(F.d[0] - (a - c * c / d)) <= Z * sd


# ------------------------------------------------------------------ factor pins
@pytest.mark.parametrize("seed", [1, 4])
def test_factor_converges_to_exact_ldl(seed):
    A = small(10, 17, seed=seed)
    Ad = A.dense()
    rk = O.rank(A.n, seed)
    M = 60000
    F = O.build_factor(A, M, 0.0, seed + 1, rk=rk)
    Ye, De = dense.exact_factor_schur(Ad, rk)
    Y = F.dense_y()
    tau = F.table.tau
    for k in range(A.n):
        lim = dense.walk_limits(Ad, rk, k)
        for i in range(A.n):
            if rk[i] >= rk[k]:
                assert Y[k, i] == (1.0 if i == k else 0.0)
                continue
            p = lim["p"][i] if lim["p"] is not None else 0.0
            sd = tau[k] * np.sqrt(max(p * (1 - p), 1e-12) / M)
            assert abs(Y[k, i] - Ye[k, i]) <= Z * sd + 1e-13, (k, i)
        r = np.searchsorted(F.walks.rows, k)
        s = slice(F.walks.rec_off[r], F.walks.rec_off[r + 1])
        v = F.walks.visits[s].astype(float)
        if v.size:
            sd = Ad[k, k] * tau[k] * v.std() / np.sqrt(v.size) / (1 + tau[k] * (v.mean() - 1)) ** 2
            assert abs(F.d[k] - De[k]) <= Z * sd + 1e-13
        else:
            assert np.isclose(F.d[k], De[k], rtol=1e-14)


def test_exact_rows_need_no_walks():
    """Rows whose neighbours all rank lower are exact (Section 5.2)."""
    A = W.config_grid2d_32()
    F = O.build_factor(A, 8, 0.0, 3)
    Ad = A.dense()
    rk = F.rank
    exact = np.flatnonzero(F.table.tau == 0)
    assert exact.size > 10
    Y = F.dense_y()
    for k in exact[:40]:
        nb = np.flatnonzero((Ad[k] != 0) & (np.arange(A.n) != k))
        assert np.all(rk[nb] < rk[k])
        assert np.allclose(Y[k, nb], Ad[k, nb] / Ad[k, k], rtol=0, atol=0)
        assert F.d[k] == Ad[k, k]
    # the highest-ranked node is always exact
    top = int(np.argmax(rk))
    assert F.table.tau[top] == 0


def test_pattern_within_reachable_set():
    """Stored Y_ki needs i reachable from k through higher-ranked nodes (Section 3.2)."""
    A = small(12, 20, seed=5)
    Ad = A.dense()
    F = O.build_factor(A, 500, 0.0, 5)
    for k in range(A.n):
        reach = dense.reachable_through_higher(Ad, F.rank, k)
        cols = set(F.ycol[F.yptr[k]:F.yptr[k + 1]].tolist())
        assert cols <= reach


def test_invariants_and_row_sum_identity():
    A = W.config_grid2d_32()
    F = O.build_factor(A, 64, 0.0, 2)
    Ad = A.dense()
    a = np.diag(Ad)
    assert np.all(F.yval < 0)
    assert np.all(F.d > 0) and np.all(F.d <= a * (1 + 1e-15))
    # 1 + sum_i Y_ki = e_k/a_k + tau_k G'_k/M'_k (ground-absorption estimate)
    e = Ad.sum(axis=1)
    Gk = np.zeros(A.n)
    Mk = np.ones(A.n)
    Gk[F.walks.rows] = F.tallies.G
    Mk[F.walks.rows] = np.maximum(F.tallies.walks, 1)
    rs = 1 + np.add.reduceat(np.append(F.yval, 0.0), F.yptr[:-1]) * (np.diff(F.yptr) > 0)
    want = e / a + F.table.tau * Gk / Mk
    assert np.allclose(rs, want, atol=1e-13)
    # the preconditioner Y^T D Y is SPD and the apply is symmetric
    Y = F.dense_y()
    Mdense = Y.T @ np.diag(F.d) @ Y
    np.linalg.cholesky(Mdense)
    rng = np.random.default_rng(0)
    r1, r2 = rng.standard_normal(A.n), rng.standard_normal(A.n)
    z1, z2 = O.apply(F, r1), O.apply(F, r2)
    assert abs(z1 @ r2 - r1 @ z2) <= 1e-13 * abs(z1 @ r2)
    assert np.allclose(Mdense @ z1, r1, atol=1e-11)


def test_drop_removes_exactly_small_entries():
    A = W.config_grid2d_32()
    F0 = O.build_factor(A, 64, 0.0, 0)
    tol = 1e-2
    F1 = O.build_factor(A, 64, tol, 0)
    keep = np.abs(F0.yval) >= tol
    assert np.array_equal(F1.yval, F0.yval[keep])
    assert np.array_equal(F1.ycol, F0.ycol[keep])
    assert np.array_equal(F1.d, F0.d)
    assert F1.yptr[-1] < F0.yptr[-1]


def test_single_node_and_all_grounded():
    A = W.from_dense(np.array([[2.5]]))
    F = O.build_factor(A, 16, 0.0, 0)
    assert F.yptr[-1] == 0 and F.d[0] == 2.5
    st, x, it, rr = O.pcg(A, F, np.array([5.0]), 1e-12)
    assert st == 0 and it == 1 and x[0] == 2.0


def test_length_criterion_against_its_statement():
    # delta * mean * sqrt(M) / sigma > z, sigma the sample standard deviation
    rng = np.random.default_rng(5)
    for _ in range(200):
        L = rng.integers(2, 50, rng.integers(2, 60))
        M = L.size
        mean, sd = L.mean(), L.std(ddof=1)
        delta, z = rng.uniform(0.01, 0.5), rng.uniform(1.0, 3.0)
        expect = True if sd == 0 else delta * mean * np.sqrt(M) / sd > z
        assert O.length_criterion(int(L.sum()), int((L * L).sum()), M, delta, z) == expect
    assert O.length_criterion(5 * 20, 25 * 20, 20, 0.01, 3.0)  # equal lengths pass


def test_adaptive_budgets_match_the_exact_length_variance():
    """Section 5.1 on a two-node game: the walk length from node 0 has exact mean and
    variance from the absorbing chain; the first M with delta*mean*sqrt(M)/sigma > z
    concentrates near M* = z^2 var / (delta mean)^2."""
    g, e0, e1 = 1.0, 0.05, 0.02
    A = W.assemble(2, np.array([0]), np.array([1]), np.array([g]), np.array([e0, e1]))
    a = np.array([g + e0, g + e1])
    # walks from node 0 (rank 0): first step to node 1, then node 1 -> ground w.p.
    # e1/a1 or -> node 0 (stay, the walk continues), node 0 -> ground w.p. e0/a0
    P = np.array([[0.0, g / a[0]], [g / a[1], 0.0]])
    N = np.linalg.inv(np.eye(2) - P)
    t = N @ np.ones(2)                      # expected steps to absorption
    t2 = (2 * N - np.eye(2)) @ t            # second moment of the absorption time
    mean = 1.0 + t[1]                       # first step, then from node 1
    var = t2[1] - t[1] ** 2
    delta, z = 0.05, 2.5758293035489004     # alpha = 99 %
    Mstar = z * z * var / (delta * mean) ** 2
    rk = np.array([0, 1], np.int32)
    tb = O.table(A, rk)
    Ms = [int(O.adaptive_budgets(A, rk, tb, seed, delta, z)[0]) for seed in range(24)]
    assert abs(np.median(Ms) / Mstar - 1.0) < 0.15, (np.median(Ms), Mstar)
