"""Input generators: the synthetic matrices are R-matrices of the stated shape and
distribution (host only; these generators hold none of the method's arithmetic)."""
import numpy as np
import pytest

from paper_math_0609672_amd import workloads as W


def _is_r_matrix(A):
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0
    d = S.diagonal()
    off = S - np.diag(d)
    assert np.all(d > 0) and off.max() <= 0
    excess = d + np.asarray(off.sum(axis=1)).ravel()
    assert np.all(excess >= -1e-9 * d)
    return np.where(excess > 1e-9 * d, excess, 0.0)  # rounding of the row sums


def test_rgg_pairs_equal_brute_force():
    rng = np.random.default_rng(3)
    pts = rng.random((1500, 3))
    for r in (0.05, 0.13, 0.31):
        u, v, d = W._rgg_pairs(pts, r)
        D = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
        bf = {tuple(p) for p in np.argwhere(np.triu(D < r, 1)).tolist()}
        assert bf == set(zip(u.tolist(), v.tolist()))
        assert np.allclose(d, D[u, v])


def test_rgg_connect_probability_monte_carlo():
    # the closed form against sampled pairs of uniform points
    rng = np.random.default_rng(5)
    a, b = rng.random((400000, 3)), rng.random((400000, 3))
    dist = np.sqrt(((a - b) ** 2).sum(1))
    for r in (0.1, 0.3, 0.6):
        p = W.rgg_connect_probability(r)
        emp = np.mean(dist < r)
        assert abs(emp - p) < 4 * np.sqrt(p * (1 - p) / a.shape[0]) + 1e-4


def test_rgg_shape_and_distribution():
    A, info = W.rgg(20000, 24.0, seed=2, return_info=True)
    assert abs(info["mean_degree"] - 24.0) <= 0.1
    excess = _is_r_matrix(A)
    off = -A.val[A.col != np.repeat(np.arange(A.n), np.diff(A.rowptr))]
    assert off.min() >= 1.0 and off.max() <= 1e3
    assert (excess > 0).sum() >= round(0.005 * A.n)
    # every connected component holds a grounded node
    from scipy.sparse.csgraph import connected_components
    nc, lab = connected_components(A.to_scipy(), directed=False)
    assert set(np.unique(lab[excess > 0])) == set(range(nc))


def test_rgg_grounds_isolated_components():
    # small radius: many components, each must receive a grounded node
    A, info = W.rgg(3000, 2.0, ground_frac=0.001, seed=4, return_info=True, tol=0.5)
    assert info["components"] > 1 and info["grounds_added"] > 0
    excess = _is_r_matrix(A)
    from scipy.sparse.csgraph import connected_components
    nc, lab = connected_components(A.to_scipy(), directed=False)
    assert set(np.unique(lab[excess > 0])) == set(range(nc))


@pytest.mark.parametrize("m", [4, 9])
def test_grid3d_shape(m):
    A = W.config_grid3d(m, seed=1)
    excess = _is_r_matrix(A)
    assert A.n == m ** 3 and A.nnz == m ** 3 + 2 * 3 * m * m * (m - 1)
    assert (excess > 0).sum() == max(round(0.01 * A.n), 1)
