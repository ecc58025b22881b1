"""Pins of the oracle's plain estimator (eq. yzdetail with eq. d, Sections 3.1 and 3.3):
walks step by the full game from the first step on, one-step walks are counted, and
Y_ki = -H_ki / M, D_k = M A_kk / J_k.  It is the form the paper starts from before the
exact one-step treatment of Section 5.2; both must reach the same limit, the complete
LDL^T factor of rev(A).

Independent pins:
  - the unconditioned walk of the absorbing chain (fundamental matrix computed from A):
    end probabilities q_ki, ground, expected stays at the start (= A_kk [A_TT^{-1}]_kk)
    match 40,000 simulated walks per row within 5 sigma;
  - the factor of 60,000 walks per row lies within 5 sigma of the dense exact factor
    (the same limit as the Section 5.2 estimator, whose pin is in test_oracle_game);
  - integer identities: M = sum H + G, every walk of length >= 1 ending at ground or a
    lower-ranked node; a row whose neighbours all rank lower takes only one-step walks;
  - the two-node closed form.
"""
import numpy as np

import oracle as O
from oracle import dense
from paper_math_0609672_amd import workloads as W

Z = 5.0


def small(n, m, seed):
    return W.random_graph(n, m, seed=seed, ground_frac=0.2)


def test_plain_walks_match_unconditioned_chain():
    A = small(9, 15, seed=2)
    Ad = A.dense()
    rk = O.rank(A.n, 102)
    tb = O.table(A, rk)
    M = 40000
    rows = np.arange(A.n)
    wk = O.walk_rows_plain(A, rk, tb, 99, rows, M)
    assert np.all(wk.budget == M)  # every row walks, exact or not
    for r, k in enumerate(rows):
        lim = dense.walk_limits(Ad, rk, k)
        s = slice(wk.rec_off[r], wk.rec_off[r + 1])
        end, vis = wk.end[s], wk.visits[s].astype(float)
        for i in range(A.n):
            q = lim["q"][i]
            assert abs(np.mean(end == i) - q) <= Z * np.sqrt(max(q * (1 - q), 1e-12) / M) + 1e-12, (k, i)
        qg = lim["q_ground"]
        assert abs(np.mean(end == -1) - qg) <= Z * np.sqrt(max(qg * (1 - qg), 1e-12) / M) + 1e-12
        assert abs(vis.mean() - lim["visits"]) <= Z * vis.std() / np.sqrt(M) + 1e-12


def test_plain_factor_converges_to_the_exact_factor():
    for seed in (1, 4):
        A = small(10, 17, seed=seed)
        Ad = A.dense()
        rk = O.rank(A.n, seed)
        M = 60000
        F = O.build_factor(A, M, 0.0, seed + 1, rk=rk, one_step_exact=False)
        Ye, De = dense.exact_factor_schur(Ad, rk)
        Y = F.dense_y()
        for k in range(A.n):
            lim = dense.walk_limits(Ad, rk, k)
            for i in range(A.n):
                if rk[i] >= rk[k]:
                    assert Y[k, i] == (1.0 if i == k else 0.0)
                    continue
                q = lim["q"][i]
                assert abs(Y[k, i] - Ye[k, i]) <= Z * np.sqrt(max(q * (1 - q), 1e-12) / M) + 1e-13
            s = slice(F.walks.rec_off[k], F.walks.rec_off[k + 1])
            v = F.walks.visits[s].astype(float)
            # D = a / mean(visits): delta method
            sd = Ad[k, k] * v.std() / np.sqrt(M) / v.mean() ** 2
            assert abs(F.d[k] - De[k]) <= Z * sd + 1e-13


def test_both_estimators_reach_the_same_factor():
    A = small(10, 17, seed=7)
    rk = O.rank(A.n, 3)
    M = 60000
    P = O.build_factor(A, M, 0.0, 5, rk=rk, one_step_exact=False)
    E = O.build_factor(A, M, 0.0, 5, rk=rk)
    Ye, De = dense.exact_factor_schur(A.dense(), rk)
    # both errors shrink like 1/sqrt(M); each is small against the entries themselves
    for F in (P, E):
        assert np.max(np.abs(F.dense_y() - Ye)) < 0.02
        assert np.max(np.abs(F.d - De) / De) < 0.02


def test_plain_identities_and_one_step_rows():
    A = W.config_grid2d_32()
    F = O.build_factor(A, 64, 0.0, 0, one_step_exact=False)
    wk, tl, rk = F.walks, F.tallies, F.rank
    assert np.all(wk.budget == 64) and np.all(wk.length >= 1)
    starts = np.repeat(wk.rows, wk.budget)
    ends = wk.end
    assert np.all((ends == -1) | (rk[np.maximum(ends, 0)] < rk[starts]))
    for k in range(A.n):
        hs = slice(tl.h_off[k], tl.h_off[k] + tl.hlen[k])
        assert tl.walks[k] == tl.h_cnt[hs].sum() + tl.G[k]
        assert np.isclose(F.d[k], 64 * A.dense()[k, k] / tl.J[k], rtol=1e-15)
    # rows with no higher-ranked neighbour: every walk is one step long
    exact = F.table.tau == 0
    lens = wk.length.reshape(A.n, 64)
    assert np.all(lens[exact] == 1)
    # their entries estimate -w/a: multinomial counts over the neighbours and ground
    Ad = A.dense()
    for k in np.flatnonzero(exact)[:20]:
        row = Ad[k]
        for i in np.flatnonzero((row < 0) & (np.arange(A.n) != k)):
            hs = slice(tl.h_off[k], tl.h_off[k] + tl.hlen[k])
            cnt = tl.h_cnt[hs][tl.h_end[hs] == i]
            p = -row[i] / row[k]
            h = cnt[0] / 64 if cnt.size else 0.0
            assert abs(h - p) <= Z * np.sqrt(p * (1 - p) / 64) + 1e-12


def test_plain_two_node_closed_form():
    a, c, d = 3.0, 1.0, 2.0
    A = W.from_dense(np.array([[a, -c], [-c, d]]))
    rk = np.array([0, 1], np.int32)
    M = 200000
    F = O.build_factor(A, M, 0.0, 11, rk=rk, one_step_exact=False)
    # row 1 (rank 1): every walk ends after one step, at node 0 (probability c/d) or at
    # ground; J = M, so D = d exactly, and Y_10 estimates -c/d
    p = c / d
    assert abs(F.dense_y()[1, 0] + p) <= Z * np.sqrt(p * (1 - p) / M) and F.d[1] == d
    # row 0: D -> a - c^2 / d, and the walks from it never reach a lower-ranked node
    v = F.walks.visits[:M].astype(float)
    sd = a * v.std() / np.sqrt(M) / v.mean() ** 2
    assert abs(F.d[0] - (a - c * c / d)) <= Z * sd
