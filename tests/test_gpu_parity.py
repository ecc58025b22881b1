"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: ranks, transition table, per-walk records and tallies bit-exact; the FP64
factor bit-exact (both sides evaluate eqs. newy/newz/d in the same operation order
without contraction); one preconditioner application within 1e-12 and PCG iterates
within 1e-10 relative after the same number of iterations (dot products are summed
in different orders).
"""
import numpy as np
import pytest

import oracle as O
from paper_math_0609672_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def srw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_math_0609672_amd import srw as s
    return s


DEV = "cuda:0"


def np_(t):
    return t.detach().cpu().numpy()


def cases():
    return {
        "grid2d_32": (W.config_grid2d_32(0), 64),
        "grid3d_12": (W.grid((12, 12, 12), g=("loguniform", 1e-2, 1e2), ground_frac=0.01,
                             excess=("uniform", 0.01, 1.0), seed=3), 256),
        "grid2d_37x29": (W.grid((37, 29), g=("uniform", 0.1, 10.0), ground_frac=0.02,
                                excess=("uniform", 0.1, 10.0), seed=5), 100),
        "random_3000": (W.random_graph(3000, 9000, seed=7, ground_frac=0.01), 37),
    }


CASES = cases()


def gpu_build(srw, A, walks, drop, seed, **kw):
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, drop, seed, **kw)
    return M, F


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 9), (1000, 0), (4097, 123456789), (300001, 77)])
def test_rank_bit_exact(srw, n, seed):
    # a diagonal matrix: the ordering is exercised without any walk
    empty = np.zeros(0, np.int64)
    A = W.assemble(n, empty, empty, np.zeros(0), np.ones(n))
    _, F = gpu_build(srw, A, 1, 0.0, seed)
    assert np.array_equal(np_(F.export()["rank"]), O.rank(n, seed))


@pytest.mark.parametrize("name", list(CASES))
def test_table_bit_exact(srw, name):
    A, walks = CASES[name]
    M, F = gpu_build(srw, A, walks, 0.0, 11, keep=1)
    tb = F.table(A.nnz)
    ref = O.table(A, O.rank(A.n, 11))
    assert np.array_equal(np_(tb["nbr"]), ref.nbr)
    assert np.array_equal(np_(tb["thr"]).view(np.uint32), ref.thr)
    assert np.array_equal(np_(tb["mthr"]).view(np.uint32), ref.mthr)
    assert np.array_equal(np_(tb["tau"]), ref.tau)
    assert np.array_equal(np_(tb["grounded"]), ref.grounded)


def compare_walks(srw, A, walks, seed, budget=None, refill=0, schedule=0, walk_waves=0):
    Mx = srw.Matrix.from_host(A, DEV)
    kw = dict(keep=2, refill_period=refill, schedule=schedule, walk_waves=walk_waves)
    if budget is not None:
        kw["walks"] = torch.as_tensor(budget, dtype=torch.int32, device=DEV)
    F = srw.build_factor(Mx, walks, 0.0, seed, **kw)
    rec = {k: np_(v) for k, v in F.records().items()}
    tl = {k: np_(v) for k, v in F.tallies().items()}
    rk = O.rank(A.n, seed)
    tb = O.table(A, rk)
    b = walks if budget is None else np.maximum(np.asarray(budget), 1)
    wk = O.walk_rows(A, rk, tb, seed, np.arange(A.n), b)
    # per-walk records
    assert np.array_equal(rec["rec_off"], wk.rec_off[:-1])
    assert np.array_equal(rec["end"], wk.end)
    assert np.array_equal(rec["visits"].view(np.uint32), wk.visits)
    assert np.array_equal(rec["length"].view(np.uint32), wk.length)
    # tallies
    t = O.tally(wk)
    assert np.array_equal(tl["walks"], wk.budget)
    assert np.array_equal(tl["J"].view(np.uint64), t.J)
    assert np.array_equal(tl["G"].view(np.uint32), t.G)
    assert np.array_equal(tl["steps"].view(np.uint64), t.steps)
    assert np.array_equal(tl["visits_sq"].view(np.uint64), t.visits_sq)
    assert np.array_equal(tl["hlen"], t.hlen)
    valid = np.zeros(tl["h_end"].size, bool)
    idx = np.repeat(t.h_off, t.hlen) + (np.arange(t.hlen.sum()) - np.repeat(np.cumsum(t.hlen) - t.hlen, t.hlen))
    valid[idx] = True
    assert np.array_equal(tl["h_end"][valid], t.h_end[valid])
    assert np.array_equal(tl["h_cnt"].view(np.uint32)[valid], t.h_cnt[valid])
    return F, t


@pytest.mark.parametrize("name", list(CASES))
def test_walks_and_tallies_bit_exact(srw, name):
    A, walks = CASES[name]
    F, t = compare_walks(srw, A, walks, 5)
    assert F.info()["walk_steps"] == int(t.steps.sum())


@pytest.mark.parametrize("refill", [1, 2, 4, 8])
@pytest.mark.parametrize("schedule", [0, 1])
def test_walks_independent_of_scheduling(srw, refill, schedule):
    A, walks = CASES["grid3d_12"]
    compare_walks(srw, A, walks, 21, refill=refill, schedule=schedule)


@pytest.mark.parametrize("walk_waves", [4, 12, 24, 64])
def test_walks_independent_of_walk_waves(srw, walk_waves):
    # the persistent walk grid's size (64: capped at the kernel's occupancy) moves walks
    # between lanes and waves only
    A, walks = CASES["random_3000"]
    F, _ = compare_walks(srw, A, walks, 8, walk_waves=walk_waves)
    ran = F.stats()["walk_waves"]
    assert ran % 4 == 0 and 4 <= ran <= walk_waves
    if walk_waves <= 12:
        assert ran == walk_waves


def test_per_row_budgets_ragged(srw):
    A, _ = CASES["random_3000"]
    rng = np.random.default_rng(0)
    budget = rng.integers(-2, 300, A.n).astype(np.int32)  # < 1 counts as 1
    compare_walks(srw, A, 64, 8, budget=budget)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("drop", [0.0, 1e-3, 2e-2])
def test_factor_bit_exact(srw, name, drop):
    A, walks = CASES[name]
    _, F = gpu_build(srw, A, walks, drop, 3)
    ref = O.build_factor(A, walks, drop, 3)
    got = {k: np_(v) for k, v in F.export().items()}
    assert np.array_equal(got["yptr"], ref.yptr)
    assert np.array_equal(got["ycol"], ref.ycol)
    assert np.array_equal(got["yval"], ref.yval)
    assert np.array_equal(got["d"], ref.d)
    assert F.info()["nnz_y"] == ref.yptr[-1]


def test_fp32_factor_is_rounded_fp64_factor(srw):
    A, walks = CASES["grid2d_37x29"]
    _, F = gpu_build(srw, A, walks, 1e-3, 4, precision="fp32")
    ref = O.build_factor(A, walks, 1e-3, 4)
    got = {k: np_(v) for k, v in F.export().items()}
    assert got["yval"].dtype == np.float32
    assert np.array_equal(got["ycol"], ref.ycol)
    assert np.array_equal(got["yval"], ref.yval.astype(np.float32))
    assert np.array_equal(got["d"], ref.d.astype(np.float32))


@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle(srw, name):
    A, walks = CASES[name]
    _, F = gpu_build(srw, A, walks, 1e-3, 2)
    ref = O.build_factor(A, walks, 1e-3, 2)
    r = W.rhs(A.n, seed=4)
    z = np_(srw.apply(F, torch.as_tensor(r, device=DEV)))
    zr = O.apply(ref, r)
    assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)


@pytest.mark.parametrize("name", list(CASES))
def test_solve_order_does_not_change_results(srw, name):
    """Each row's sum has a fixed order, so the ticket order (rank or level) cannot
    change the preconditioner's result."""
    A, walks = CASES[name]
    M = srw.Matrix.from_host(A, DEV)
    F0 = srw.build_factor(M, walks, 1e-3, 6, solve_order=0)
    F1 = srw.build_factor(M, walks, 1e-3, 6, solve_order=1)
    F2 = srw.build_factor(M, walks, 1e-3, 6, solve_order=2)
    r = torch.as_tensor(W.rhs(A.n, seed=8), device=DEV)
    z0 = srw.apply(F0, r)
    assert torch.equal(z0, srw.apply(F1, r)) and torch.equal(z0, srw.apply(F2, r))
    assert F1.depth() == F0.depth() == F2.depth()


def test_level_order_matches_rank_order_mid_size(srw):
    """13,824 rows (several tiles of every kernel): each row's sum has a fixed order,
    so the level-ordered plan gives the rank-ordered plan's preconditioner and PCG
    iterates bit for bit, and the preconditioner matches the oracle's factor."""
    A = W.grid((24, 24, 24), g=("loguniform", 1e-2, 1e2), ground_frac=0.01,
               excess=("uniform", 0.01, 1.0), seed=4)
    M = srw.Matrix.from_host(A, DEV)
    F0 = srw.build_factor(M, 64, 1e-3, 9, solve_order=0)
    F1 = srw.build_factor(M, 64, 1e-3, 9, solve_order=1)
    for seed in (8, 9):
        r = torch.as_tensor(W.rhs(A.n, seed=seed), device=DEV)
        assert torch.equal(srw.apply(F0, r), srw.apply(F1, r))
    b = torch.as_tensor(W.rhs(A.n, seed=10), device=DEV)
    st0, x0, it0, _ = srw.pcg_solve(M, F0, b, 1e-10)
    st1, x1, it1, _ = srw.pcg_solve(M, F1, b, 1e-10)
    assert st0 == st1 == srw.OK and it0 == it1
    assert torch.equal(x0, x1)
    assert F1.depth() == F0.depth()
    ref = O.build_factor(A, 64, 1e-3, 9)
    r = W.rhs(A.n, seed=8)
    z = np_(srw.apply(F1, torch.as_tensor(r, device=DEV)))
    zr = O.apply(ref, r)
    assert np.linalg.norm(z - zr) <= 1e-12 * np.linalg.norm(zr)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_pcg_matches_oracle(srw, name, tol):
    A, walks = CASES[name]
    M, F = gpu_build(srw, A, walks, 1e-3, 0)
    ref = O.build_factor(A, walks, 1e-3, 0)
    b = W.rhs(A.n, seed=1)
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), tol)
    st_o, x_o, it_o, rel_o = O.pcg(A, ref, b, tol)
    assert st == st_o == 0
    assert it == it_o
    x = np_(x)
    assert np.linalg.norm(x - x_o) <= 1e-10 * np.linalg.norm(x_o)
    # final residual vectors agree: ||(b - A x) - (b - A x_o)|| <= 1e-10 ||b||
    As = A.to_scipy()
    assert np.linalg.norm(As @ (x - x_o)) <= 1e-10 * np.linalg.norm(b)
    # independent check of the returned residual
    true = np.linalg.norm(b - As @ x) / np.linalg.norm(b)
    assert rel <= tol and np.isclose(true, rel, rtol=1e-6)


def test_fp32_factor_pcg_reaches_tolerance(srw):
    A, walks = CASES["grid3d_12"]
    M, F = gpu_build(srw, A, walks, 1e-3, 0, precision="fp32")
    ref = O.build_factor(A, walks, 1e-3, 0)
    b = W.rhs(A.n, seed=1)
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), 1e-10)
    st_o, x_o, it_o, _ = O.pcg(A, ref, b, 1e-10)
    assert st == 0 and rel <= 1e-10
    x = np_(x)
    # the FP32 preconditioner changes the iterates, not the solution tolerance
    assert np.linalg.norm(x - x_o) <= 1e-8 * np.linalg.norm(x_o)
    assert it <= it_o + 3


# -------------------------------------------------------------------- edge cases
def test_diagonal_matrix_all_rows_exact(srw):
    A = W.from_dense(np.diag(np.linspace(1.0, 3.0, 100)))
    M, F = gpu_build(srw, A, 64, 0.0, 0)
    i = F.info()
    assert i["nnz_y"] == 0 and i["walks"] == 0 and F.depth() == 1
    b = W.rhs(100, seed=0)
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), 1e-12)
    assert st == 0 and it == 1
    assert np.allclose(np_(x), b / np.linspace(1.0, 3.0, 100), rtol=1e-15)


def test_single_node_and_two_nodes(srw):
    A1 = W.from_dense(np.array([[2.5]]))
    M, F = gpu_build(srw, A1, 16, 0.0, 0)
    st, x, it, rel = srw.pcg_solve(M, F, torch.tensor([5.0], dtype=torch.float64, device=DEV), 1e-12)
    assert st == 0 and it == 1 and np_(x)[0] == 2.0
    A2 = W.from_dense(np.array([[3.0, -1.0], [-1.0, 2.0]]))
    compare_walks(srw, A2, 1000, 4)


def test_disconnected_grounded_components_and_one_walk(srw):
    Ad = np.zeros((6, 6))
    for (i, j) in [(0, 1), (1, 2), (3, 4)]:
        Ad[i, j] = Ad[j, i] = -1.0
    Ad[np.diag_indices(6)] = -Ad.sum(axis=1) + np.array([0.5, 0, 0, 0, 0.25, 1.0])
    A = W.from_dense(Ad)
    compare_walks(srw, A, 1, 2)
    _, F = gpu_build(srw, A, 1, 0.0, 2)
    ref = O.build_factor(A, 1, 0.0, 2)
    assert np.array_equal(np_(F.export()["yval"]), ref.yval)


def test_zero_rhs_and_iteration_cap(srw):
    A, walks = CASES["grid2d_32"]
    M, F = gpu_build(srw, A, walks, 1e-3, 0)
    st, x, it, rel = srw.pcg_solve(M, F, torch.zeros(A.n, dtype=torch.float64, device=DEV), 1e-8)
    assert st == srw.OK and it == 0 and rel == 0.0 and not np_(x).any()
    b = W.rhs(A.n, seed=1)
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), 1e-14, max_iter=3)
    ref = O.build_factor(A, walks, 1e-3, 0)
    st_o, x_o, it_o, _ = O.pcg(A, ref, b, 1e-14, max_iter=3)
    assert st == srw.NOT_CONVERGED == st_o and it == 3 == it_o
    assert np.linalg.norm(np_(x) - x_o) <= 1e-12 * np.linalg.norm(x_o)


def test_error_statuses(srw):
    good = W.config_grid2d_32()
    D = good.dense()
    i, j = np.argwhere(D < 0)[0]
    bad = D.copy()
    bad[i, j] = bad[j, i] = 0.3
    with pytest.raises(srw.SrwError) as e:
        gpu_build(srw, W.from_dense(bad), 8, 0.0, 0)
    assert e.value.status == srw.E_NOT_RMATRIX
    asym = D.copy()
    asym[i, j] *= 1.01
    with pytest.raises(srw.SrwError) as e:
        gpu_build(srw, W.from_dense(asym), 8, 0.0, 0)
    assert e.value.status == srw.E_NOT_RMATRIX
    ungrounded = np.array([[2.0, -1, 0, 0], [-1, 2.0, 0, 0], [0, 0, 1.0, -1], [0, 0, -1, 1.0]])
    with pytest.raises(srw.SrwError) as e:
        gpu_build(srw, W.from_dense(ungrounded), 8, 0.0, 0)
    assert e.value.status == srw.E_SINGULAR
    unsorted = W.CSR(good.n, good.rowptr.copy(), good.col.copy(), good.val.copy())
    unsorted.col[0:2] = unsorted.col[0:2][::-1]
    with pytest.raises(srw.SrwError) as e:
        gpu_build(srw, unsorted, 8, 0.0, 0)
    assert e.value.status == srw.E_ARG
    with pytest.raises(srw.SrwError) as e:
        gpu_build(srw, good, 64, 0.0, 0, max_steps=2)
    assert e.value.status == srw.E_WALK_LIMIT
    notperm = torch.zeros(good.n, dtype=torch.int32, device=DEV)
    with pytest.raises(srw.SrwError) as e:
        gpu_build(srw, good, 8, 0.0, 0, rank=notperm)
    assert e.value.status == srw.E_ARG


@pytest.mark.parametrize("reuse", [False, True])
def test_per_row_budget_above_limit_is_refused(srw, reuse):
    # a chunk descriptor holds the first walk of a chunk in 16 bits: a budget past the
    # limit (here 65,537 on one row) must fail before any walk runs, with or without reuse
    good = W.config_grid2d_32()
    M = srw.Matrix.from_host(good, DEV)
    budget = np.full(good.n, 8, np.int32)
    k = int(np.flatnonzero(O.table(good, O.rank(good.n, 0)).tau > 0)[0])  # a row that walks
    for over in (65537, 8193):
        budget[k] = over
        with pytest.raises(srw.SrwError) as e:
            srw.build_factor(M, 8, 0.0, 0, walks=torch.as_tensor(budget, device=DEV), reuse=reuse)
        assert e.value.status == srw.E_ARG
    budget[k] = 8192  # the limit itself builds
    F = srw.build_factor(M, 8, 0.0, 0, walks=torch.as_tensor(budget, device=DEV), reuse=reuse)
    F.free()


@pytest.mark.parametrize("name", list(CASES))
def test_plain_estimator_bit_exact(srw, name):
    # one_step_exact = 0: eq. yzdetail with eq. d, every step random, one-step walks
    # counted; every row walks
    A, walks = CASES[name]
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, 1e-3, 21, keep=2, one_step_exact=False)
    ref = O.build_factor(A, walks, 1e-3, 21, one_step_exact=False)
    rec = F.records()
    off = np_(rec["rec_off"])
    assert np.array_equal(off, ref.walks.rec_off[:-1])
    assert np.array_equal(np_(rec["end"]), ref.walks.end)
    assert np.array_equal(np_(rec["visits"]).view(np.uint32), ref.walks.visits)
    assert np.array_equal(np_(rec["length"]).view(np.uint32), ref.walks.length)
    tl = F.tallies()
    assert np.array_equal(np_(tl["walks"]).view(np.uint32), ref.tallies.walks)
    assert np.array_equal(np_(tl["J"]).view(np.uint64), ref.tallies.J)
    got = {k: np_(v) for k, v in F.export().items()}
    for k in ("yptr", "ycol", "yval", "d"):
        assert np.array_equal(got[k], getattr(ref, k)), k
    b = W.rhs(A.n, seed=3)
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), 1e-8)
    st_o, x_o, it_o, _ = O.pcg(A, ref, b, 1e-8)
    assert st == st_o == 0 and it == it_o
    assert np.linalg.norm(np_(x) - x_o) <= 1e-10 * np.linalg.norm(x_o)
    F.free()


@pytest.mark.parametrize("name", ["grid3d_12", "random_3000"])
def test_walk_stats_match_the_records(srw, name):
    # sample variance of the stays and mean length per row, from the tallies on the GPU,
    # against numpy over the oracle's walk records of the same rows
    A, walks = CASES[name]
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, 1e-3, 5, keep=1)
    var, mean = (np_(t) for t in srw.walk_stats(F))
    ref = O.build_factor(A, walks, 1e-3, 5)
    rv, rm = O.walk_stats(ref.walks)
    assert np.array_equal(np.isnan(var), np.isnan(rv)) and np.array_equal(np.isnan(mean), np.isnan(rm))
    ok = ~np.isnan(rv)
    assert np.allclose(var[ok], rv[ok], rtol=1e-12, atol=1e-12)
    ok = ~np.isnan(rm)
    assert np.allclose(mean[ok], rm[ok], rtol=1e-14, atol=0)
    F.free()


def test_plain_estimator_refused_where_it_does_not_apply(srw):
    A, walks = CASES["grid2d_32"]
    M = srw.Matrix.from_host(A, DEV)
    with pytest.raises(srw.SrwError) as e:
        srw.build_factor(M, walks, 1e-3, 1, one_step_exact=False, reuse=True)
    assert e.value.status == srw.E_ARG


def test_natural_ordering_matches_oracle(srw):
    # rank = node id: the ordering the paper's derivations are written in
    A, walks = CASES["grid2d_37x29"]
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, 1e-3, 4, rank="natural")
    ref = O.build_factor(A, walks, 1e-3, 4, rk=np.arange(A.n, dtype=np.int32))
    got = {k: np_(v) for k, v in F.export().items()}
    assert np.array_equal(got["rank"], np.arange(A.n))
    assert np.array_equal(got["yptr"], ref.yptr) and np.array_equal(got["ycol"], ref.ycol)
    assert np.array_equal(got["yval"], ref.yval) and np.array_equal(got["d"], ref.d)
    b = W.rhs(A.n, seed=2)
    st, x, it, rel = srw.pcg_solve(M, F, torch.as_tensor(b, device=DEV), 1e-8)
    st_o, x_o, it_o, _ = O.pcg(A, ref, b, 1e-8)
    assert st == st_o == 0 and it == it_o
    assert np.linalg.norm(np_(x) - x_o) <= 1e-10 * np.linalg.norm(x_o)
    F.free()


def test_given_ordering_matches_oracle(srw):
    A, walks = CASES["grid2d_37x29"]
    rk = np.random.default_rng(3).permutation(A.n).astype(np.int32)
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, 1e-3, 9, rank=torch.as_tensor(rk, device=DEV))
    ref = O.build_factor(A, walks, 1e-3, 9, rk=rk)
    got = {k: np_(v) for k, v in F.export().items()}
    assert np.array_equal(got["rank"], rk)
    assert np.array_equal(got["yval"], ref.yval) and np.array_equal(got["d"], ref.d)


def test_maximum_budget_row(srw):
    # a row with the largest accepted budget (8192 walks: the tally's 64 KiB of LDS)
    A = W.config_grid2d_32(1)
    budget = np.full(A.n, 5, dtype=np.int32)
    budget[[0, 17, 600]] = [8192, 4097, 8191]
    compare_walks(srw, A, 5, 3, budget=budget)


def test_budget_classes_bit_exact(srw):
    # budgets on both sides of every tally class boundary (256, 2048), rows of every
    # class scattered over the matrix, so that each class runs over a row list
    A = W.config_grid2d_32(2)
    rng = np.random.default_rng(11)
    budget = rng.integers(1, 64, A.n).astype(np.int32)
    picks = rng.choice(A.n, 24, replace=False)
    budget[picks] = [255, 256, 257, 258, 511, 1000, 2047, 2048, 2049, 2050, 3000, 4095,
                     4096, 4097, 6000, 8191, 8192, 300, 700, 1500, 1999, 2500, 5000, 7777]
    compare_walks(srw, A, 5, 6, budget=budget)
    # the middle class alone (no row above 2048)
    budget[budget > 2048] = 2048
    compare_walks(srw, A, 5, 6, budget=budget)


@pytest.mark.parametrize("name,delta,max_walks", [("grid2d_32", 0.2, 8192), ("random_3000", 0.3, 8192),
                                                  ("grid2d_37x29", 0.02, 100)])
def test_adaptive_budgets_bit_exact(srw, name, delta, max_walks):
    """Section 5.1 stopping rule: the GPU's walks per row equal the oracle's
    sequential rule (same z), including rows capped at max_walks and exact rows."""
    import statistics
    A, _ = CASES[name]
    alpha = 0.99
    z = statistics.NormalDist().inv_cdf(1.0 - (1.0 - alpha) / 2.0)
    M = srw.Matrix.from_host(A, DEV)
    walks = np_(srw.adaptive_budgets(M, 7, delta, alpha=alpha, max_walks=max_walks))
    rk = O.rank(A.n, 7)
    tb = O.table(A, rk)
    ref = O.adaptive_budgets(A, rk, tb, 7, delta, z, 20, max_walks)
    assert np.array_equal(walks, ref)
    assert np.all((walks == 0) == (tb.tau <= 0))
    # and a factor built with them is the oracle's, bit for bit
    F = srw.build_factor(M, 1, 1e-3, 7, walks=torch.as_tensor(walks, device=DEV))
    ex = {k: np_(v) for k, v in F.export().items()}
    Fo = O.build_factor(A, np.maximum(walks, 1), 1e-3, 7)
    assert np.array_equal(ex["yptr"], Fo.yptr)
    assert np.array_equal(ex["ycol"], Fo.ycol)
    assert np.array_equal(ex["yval"], Fo.yval)
    assert np.array_equal(ex["d"], Fo.d)
    F.free()


def hub_matrix():
    rng = np.random.default_rng(11)
    n = 900
    base = W.random_graph(n, 2500, seed=11, ground_frac=0.02)
    S = base.to_scipy().tocoo()
    eu, ev = S.row[S.row < S.col], S.col[S.row < S.col]
    hubs = {0: 200, 1: 97, 2: 96, 3: 40}
    extra = []
    for h, d in hubs.items():
        others = rng.choice(np.arange(4, n), size=d, replace=False)
        extra += [(h, int(o)) for o in others]
    pairs = set(zip(eu.tolist(), ev.tolist()))
    for a_, b_ in extra:
        pairs.add((min(a_, b_), max(a_, b_)))
    e = np.array(sorted(pairs))
    g = rng.uniform(0.1, 10.0, e.shape[0])
    excess = np.zeros(n)
    excess[rng.choice(n, 20, replace=False)] = rng.uniform(0.1, 1.0, 20)
    return W.assemble(n, e[:, 0], e[:, 1], g, excess)


def test_walks_bit_exact_with_hub_nodes(srw):
    # nodes of degree > 96: the record's line summaries cover twelve lines and the
    # step scans on from the thirteenth; degrees 7..96 use the summaries
    A = hub_matrix()
    deg = np.diff(A.rowptr) - 1
    assert deg.max() > 96
    compare_walks(srw, A, 48, 13)


@pytest.mark.parametrize("drop", [0.0, 1e-3])
def test_factor_bit_exact_with_wide_rows(srw, drop):
    # rows with more than 64 entries and rows with more than 64 distinct walk ends
    A = hub_matrix()
    walks = 160
    _, F = gpu_build(srw, A, walks, drop, 6, keep=2)
    assert (np.diff(A.rowptr) > 64).any()
    assert np_(F.tallies()["hlen"]).max() > 64
    ref = O.build_factor(A, walks, drop, 6)
    got = {k: np_(v) for k, v in F.export().items()}
    assert np.array_equal(got["yptr"], ref.yptr)
    assert np.array_equal(got["ycol"], ref.ycol)
    assert np.array_equal(got["yval"], ref.yval)
    assert np.array_equal(got["d"], ref.d)


@pytest.mark.parametrize("name,A,walks", [
    ("grid2d_32", None, None),
    ("random_50_wide", W.random_graph(50, 400, seed=5, ground_frac=0.05), 40),
])
def test_lds_staged_walks_bit_exact(srw, name, A, walks):
    """Tables that fit in one workgroup's LDS are walked from an LDS copy (narrow
    records, and wide ones with bucket lines): the records and tallies are the
    oracle's, bit for bit."""
    if A is None:
        A, walks = CASES[name]
    assert int(np.diff(A.rowptr).max()) > 7 or name == "grid2d_32"
    F, t = compare_walks(srw, A, walks, 13)
    assert F.stats()["walk_lds"] == 1


def test_large_table_walks_from_memory(srw):
    """A table larger than a workgroup's LDS is read from memory (the 12^3 grid's 3,456
    lines of 64 bytes are 216 KiB)."""
    A, walks = CASES["grid3d_12"]
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, 1e-3, 1)
    assert F.stats()["walk_lds"] == 0
    F.free()
