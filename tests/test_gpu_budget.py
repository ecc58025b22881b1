"""Parity of the learned walk-budget kernels (through the C ABI) with the allocator
oracle (oracle/budget.py).

Bars: ranks bit-exact.  Features: the oracle's float64 values rounded to float32, within
one float32 ulp (the logarithms may differ in the last float64 bit).  Labels: 1e-12
relative (both from bit-identical tallies; the H-list sum runs in another order).
Network output: the oracle evaluates the same bfloat16-rounded operands exactly, the
GPU accumulates in float32; with scale_k = sum_h |W3_h H2_kh| + |b3|, rows agree to
1e-5 scale_k unless a hidden activation lies within float32 error of a bfloat16
rounding midpoint and rounds the other way, which moves a row by at most 2^-7 scale_k;
so >= 99% of rows meet 1e-5 and all rows 2^-7.  Gradients: relative L2 error <= 2e-3
per tensor and loss 1e-4 (float32 sums over the batch, rare rounding flips).  Adam:
the GPU step applied to its own gradient matches the oracle's step on that gradient
to float32 rounding.  Budgets: equal, except where exp(pred) / eps lies within 1e-9
of an integer (then within 1).
"""
import numpy as np
import pytest

import oracle as O
from oracle import budget as B
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


def flat(p: dict) -> np.ndarray:
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"], p["b3"]])


def unflat(v: np.ndarray) -> dict:
    v = np.asarray(v, dtype=np.float64)
    o = 0
    out = {}
    for k, shape in (("W1", (8, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64,)),
                     ("b3", (1,))):
        size = int(np.prod(shape))
        out[k] = v[o:o + size].reshape(shape).copy()
        o += size
    assert o == 4801
    return out


MATRICES = {
    "grid3d_12": lambda: W.grid((12, 12, 12), g=("loguniform", 1e-2, 1e2), ground_frac=0.01,
                                excess=("uniform", 0.01, 1.0), seed=3),
    "random_3000": lambda: W.random_graph(3000, 9000, seed=7, ground_frac=0.01),
    "rgg_2000": lambda: W.rgg(2000, 24.0, seed=4),
}


@pytest.mark.parametrize("n,seed", [(1, 0), (17, 3), (5000, 12345), (300001, 2)])
def test_ordering_bit_exact(srw, n, seed):
    assert np.array_equal(np_(srw.ordering(n, seed, DEV)), O.rank(n, seed))


@pytest.mark.parametrize("name", sorted(MATRICES))
def test_features_match_oracle(srw, name):
    A = MATRICES[name]()
    M = srw.Matrix.from_host(A, DEV)
    rank = srw.ordering(A.n, 11, DEV)
    f = np_(srw.row_features(M, rank))
    ref = B.features(A, O.rank(A.n, 11)).astype(np.float32)
    ulp = np.spacing(np.abs(ref))
    assert np.all(np.abs(f - ref) <= ulp), np.max(np.abs(f - ref) / ulp)


@pytest.mark.parametrize("per_step", [False, True])
@pytest.mark.parametrize("name,walks", [("grid3d_12", 64), ("random_3000", 37), ("rgg_2000", 16)])
def test_labels_match_oracle(srw, name, walks, per_step):
    A = MATRICES[name]()
    M = srw.Matrix.from_host(A, DEV)
    F = srw.build_factor(M, walks, 0.0, 5, keep=1)
    lab = np_(srw.budget_labels(F, per_step=per_step))
    Fo = O.build_factor(A, walks, 0.0, 5)
    ref = B.labels(Fo.table.tau, Fo.tallies, per_step=per_step)
    assert np.array_equal(np.isnan(lab), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.allclose(lab[ok], ref[ok], rtol=1e-12, atol=1e-300)
    F.free()


def random_net(seed):
    rng = np.random.default_rng(seed)
    p = B.init_params(seed)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.2
    # parameters as float32 values (what the device holds)
    return unflat(flat(p).astype(np.float32).astype(np.float64))


def random_inputs(n, seed):
    rng = np.random.default_rng([seed, 1])
    big = max(n, 4096)  # standardization statistics from a larger draw (n may be 1)
    X = (rng.standard_normal((big, 8)) * rng.uniform(0.5, 3.0, 8) + rng.uniform(-2, 2, 8))
    X = X.astype(np.float32)
    mu = X.mean(axis=0).astype(np.float32)
    sd = X.std(axis=0).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    return np.ascontiguousarray(X[:n]), mu, sd, t


def oracle_inputs(X, mu, sd):
    # the GPU standardizes in float32 before rounding to bfloat16
    return ((X - mu) / sd).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", [1, 16, 1009, 20000])
def test_mlp_forward_matches_oracle(srw, n):
    p = random_net(2)
    X, mu, sd, _ = random_inputs(n, 3)
    P = torch.as_tensor(flat(p).astype(np.float32), device=DEV)
    musd = torch.as_tensor(np.concatenate([mu, sd]), device=DEV)
    y = np_(srw.mlp_forward(P, musd, torch.as_tensor(X, device=DEV)))
    ref, cache = B.mlp_forward(p, oracle_inputs(X, mu, sd), round_bf16=True)
    scale = np.abs(cache["h2"]) @ np.abs(cache["W3"]) + abs(p["b3"][0])
    err = np.abs(y - ref) / scale
    assert np.all(err <= 2.0 ** -7), err.max()
    assert np.mean(err <= 1e-5) >= 0.99, np.mean(err <= 1e-5)


@pytest.mark.parametrize("n", [16, 1009, 20000])
def test_mlp_gradients_match_oracle(srw, n):
    p = random_net(5)
    X, mu, sd, t = random_inputs(n, 6)
    P = torch.as_tensor(flat(p).astype(np.float32), device=DEV)
    musd = torch.as_tensor(np.concatenate([mu, sd]), device=DEV)
    grad = torch.empty(4801, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    srw.mlp_train_step(P, musd, torch.as_tensor(X, device=DEV), torch.as_tensor(t, device=DEV),
                       grad=grad, loss=loss)
    torch.cuda.synchronize()
    ref_loss, ref_g = B.loss_and_grads(p, oracle_inputs(X, mu, sd), t.astype(np.float64),
                                       round_bf16=True)
    assert abs(float(np_(loss)[0]) - ref_loss) <= 1e-4 * ref_loss
    g = unflat(np_(grad))
    for k in ref_g:
        d = np.linalg.norm(g[k] - ref_g[k])
        assert d <= 2e-3 * np.linalg.norm(ref_g[k]) + 1e-12, (k, d / np.linalg.norm(ref_g[k]))
    # parameters untouched without Adam moments
    assert np.array_equal(np_(P), flat(p).astype(np.float32))


def test_adam_steps_match_oracle(srw):
    p = random_net(8)
    X, mu, sd, t = random_inputs(3000, 9)
    P = torch.as_tensor(flat(p).astype(np.float32), device=DEV)
    m = torch.zeros(4801, dtype=torch.float32, device=DEV)
    v = torch.zeros(4801, dtype=torch.float32, device=DEV)
    musd = torch.as_tensor(np.concatenate([mu, sd]), device=DEV)
    Xd, td = torch.as_tensor(X, device=DEV), torch.as_tensor(t, device=DEV)
    grad = torch.empty(4801, dtype=torch.float32, device=DEV)
    st = B.adam_state(p)
    q = {k: v_.copy() for k, v_ in p.items()}
    lr = 1e-2
    for step in (1, 2, 3):
        before = np_(P).astype(np.float64)
        srw.mlp_train_step(P, musd, Xd, td, adam_m=m, adam_v=v, step=step, lr=lr, grad=grad)
        torch.cuda.synchronize()
        B.adam_step(q, unflat(np_(grad)), st, lr=lr)
        after = np_(P).astype(np.float64)
        ref = flat(q)
        tol = 3e-5 * lr + 2.0 ** -23 * np.abs(before) * 2  # float32 bias corrections: ~1e-5 relative
        assert np.all(np.abs(after - ref) <= tol), np.max(np.abs(after - ref) - tol)
        q = unflat(after)  # continue from the device's float32 parameters


def test_train_step_rows_equals_gathered_batch(srw):
    """Training on a row list equals training on the gathered copy of those rows, bit
    for bit (same tiles, same order), over three Adam steps; a row outside the arrays is
    refused before anything is queued."""
    p = random_net(11)
    X, mu, sd, t = random_inputs(5000, 12)
    musd = torch.as_tensor(np.concatenate([mu, sd]), device=DEV)
    Xd, td = torch.as_tensor(X, device=DEV), torch.as_tensor(t, device=DEV)
    rows = np.random.default_rng(13).integers(0, 5000, 1777).astype(np.int32)
    rows[:3] = [0, 4999, 0]  # ends of the arrays, and a repeat
    rd = torch.as_tensor(rows, device=DEV)
    Xg, tg = Xd[rd.long()].contiguous(), td[rd.long()].contiguous()
    outs = []
    for gathered in (False, True):
        P = torch.as_tensor(flat(p).astype(np.float32), device=DEV)
        m = torch.zeros(4801, dtype=torch.float32, device=DEV)
        v = torch.zeros(4801, dtype=torch.float32, device=DEV)
        loss = torch.empty(1, dtype=torch.float32, device=DEV)
        for step in (1, 2, 3):
            if gathered:
                srw.mlp_train_step(P, musd, Xg, tg, adam_m=m, adam_v=v, step=step, lr=1e-2, loss=loss)
            else:
                srw.mlp_train_step_rows(P, musd, Xd, td, rd, adam_m=m, adam_v=v, step=step,
                                        lr=1e-2, loss=loss)
        torch.cuda.synchronize()
        outs.append((np_(P), np_(m), np_(v), np_(loss)))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    P = torch.as_tensor(flat(p).astype(np.float32), device=DEV)
    for bad in (-1, 5000):
        rb = rd.clone()
        rb[100] = bad
        with pytest.raises(srw.SrwError):
            srw.mlp_train_step_rows(P, musd, Xd, td, rb)
    assert np.array_equal(np_(P), flat(p).astype(np.float32))


@pytest.mark.parametrize("half", [False, True])
def test_budget_targets_match_definition(srw, half):
    """Rows with a finite positive label, in row order; target log(label), halved on
    request (the square-root and Neyman rules)."""
    rng = np.random.default_rng(21)
    n = 10007
    lab = np.exp(rng.uniform(-20, 5, n))
    lab[rng.random(n) < 0.1] = np.nan
    lab[:6] = [0.0, -1.0, np.inf, -np.inf, np.nan, 5e-324]
    feat = rng.standard_normal((n, 8)).astype(np.float32)
    x, y = srw.budget_targets(torch.as_tensor(lab, device=DEV), torch.as_tensor(feat, device=DEV),
                              half)
    keep = np.isfinite(lab) & (lab > 0)
    ref_y = np.log(lab[keep]) * (0.5 if half else 1.0)
    assert x.shape[0] == keep.sum() and y.shape[0] == keep.sum()
    assert np.array_equal(np_(x), feat[keep])
    assert np.array_equal(np_(y), ref_y.astype(np.float32))
    # nothing kept
    x0, y0 = srw.budget_targets(torch.full((5,), np.nan, dtype=torch.float64, device=DEV),
                                torch.as_tensor(feat[:5], device=DEV), half)
    assert x0.shape[0] == 0 and y0.shape[0] == 0


@pytest.mark.parametrize("n", [1, 2, 777, 300001])
def test_mlp_standardize_matches_definition(srw, n):
    """Per-feature mean and sample standard deviation (n - 1; at least 1e-6; 1 for one
    row) and the target mean, to float32 rounding of the float64 statistics."""
    rng = np.random.default_rng(n)
    X = (rng.standard_normal((n, 8)) * rng.uniform(0.1, 5.0, 8) + rng.uniform(-3, 3, 8))
    X[:, 5] = 2.5  # a constant feature: sd floored at 1e-6
    X = X.astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    mu_sd, tm = srw.mlp_standardize(torch.as_tensor(X, device=DEV), torch.as_tensor(t, device=DEV))
    X64 = X.astype(np.float64)
    mu = X64.mean(axis=0)
    sd = X64.std(axis=0, ddof=1) if n > 1 else np.ones(8)
    sd = np.maximum(sd, 1e-6)
    got = np_(mu_sd).astype(np.float64)
    assert np.allclose(got[:8], mu.astype(np.float32), rtol=2e-7, atol=1e-6 * np.abs(X64).max())
    assert np.allclose(got[8:], sd.astype(np.float32), rtol=2e-6)
    assert abs(float(np_(tm)[0]) - t.astype(np.float64).mean()) <= 1e-6 * (1 + np.abs(t).max())
    assert np.array_equal(np_(srw.mlp_standardize(torch.as_tensor(X, device=DEV))), np_(mu_sd))


def test_budgets_match_oracle(srw):
    rng = np.random.default_rng(4)
    pred = rng.uniform(-8, 6, 5001).astype(np.float32)
    pred[:3] = [np.nan, 50.0, -50.0]
    walks = np_(srw.mlp_budgets(torch.as_tensor(pred, device=DEV), 0.01, 4, 4096))
    p64 = pred.astype(np.float64)
    with np.errstate(invalid="ignore"):
        ref = B.budgets(np.nan_to_num(p64, nan=-np.inf), np.ones(pred.size), 0.01, 4, 4096)
    q = np.exp(p64) / 0.01
    near = np.abs(q - np.round(q)) <= 1e-9 * np.maximum(q, 1)
    assert walks[0] == 4 and walks[1] == 4096 and walks[2] == 4
    assert np.all((walks == ref) | (near & (np.abs(walks - ref) <= 1)))


def test_training_pipeline(srw):
    """Pilot labels -> features -> training on the GPU -> budgets -> a factor that
    PCG converges with (small grids of the evaluation family)."""
    from paper_math_0609672_amd import budget as LB
    Xs, ys = [], []
    for seed in (1, 2):
        A = W.config_grid3d(16, seed)
        X, y = LB.pilot_rows(srw.Matrix.from_host(A, DEV), seed, 64, 1e-4)
        Xs.append(X)
        ys.append(y)
    X, y = torch.cat(Xs), torch.cat(ys)
    model = LB.fit(X, y, epochs=20, batch=2048, lr=3e-3, log_every=1)
    losses = [l for _, l in model.history]
    var = float(y.var())
    assert losses[-1] < 0.8 * var, (losses[0], losses[-1], var)
    A = W.config_grid3d(16, 0)
    M = srw.Matrix.from_host(A, DEV)
    walks = LB.budgets(model, M, 0, eps=0.01, lo=8, hi=4096)
    assert int(walks.min()) >= 8 and int(walks.max()) <= 4096
    F = srw.build_factor(M, 64, 1e-4, 0, walks=walks)
    b = torch.as_tensor(W.rhs(A.n, seed=0), device=DEV)
    st, x, it, rel = srw.pcg_solve(M, F, b, 1e-8, 1000)
    assert st == srw.OK and rel <= 1e-8
    F.free()


def test_learned_budgets_replace_the_pilot(srw):
    """What the trained network gains: budgets for an unseen matrix without a pilot
    factor.  They reach the same PCG iteration count (within 2) as the allocation from
    the matrix's own measured labels at the same eps, and reach the tolerance with fewer
    walk steps than the uniform 256 walks per row."""
    from paper_math_0609672_amd import budget as LB
    Xs, ys = [], []
    for seed in (1, 2, 3):
        A = W.config_grid3d(20, seed)
        X, y = LB.pilot_rows(srw.Matrix.from_host(A, DEV), seed, 256, 1e-4, rule="equal")
        Xs.append(X)
        ys.append(y)
    model = LB.fit(torch.cat(Xs), torch.cat(ys), epochs=40, batch=4096, lr=3e-3)
    A = W.config_grid3d(20, 0)
    M = srw.Matrix.from_host(A, DEV)
    b = torch.as_tensor(W.rhs(A.n, seed=0), device=DEV)

    def solve(walks=None):
        F = srw.build_factor(M, 256, 1e-4, 0, walks=walks)
        st, _, it, rel = srw.pcg_solve(M, F, b, 1e-8, 1000)
        steps = F.stats()["walk_steps"]
        F.free()
        assert st == srw.OK and rel <= 1e-8
        return it, steps

    it_u, steps_u = solve()
    F = srw.build_factor(M, 256, 1e-4, 0, keep=1)
    lab = srw.budget_labels(F)
    F.free()
    eps = 0.01
    label_walks = torch.clamp(torch.ceil(torch.nan_to_num(lab, nan=1.0) / eps), 8, 8192).to(torch.int32)
    it_l, steps_l = solve(label_walks)
    it_n, steps_n = solve(LB.budgets(model, M, 0, eps, lo=8, hi=8192))
    assert abs(it_n - it_l) <= 2, (it_n, it_l)
    assert steps_n < steps_u, (steps_n, steps_u)


def test_square_root_rule_saves_walks_at_equal_iterations(srw):
    """The square-root rule (walks in proportion to the root of the per-walk variance)
    served by the trained network, at the scale of the 128^3 grid: trained on four 64^3
    pilot factors (20 epochs), some eps reaches the uniform 256-walk build's PCG iteration count at
    the same tolerance with at least 10 % fewer walk steps.  (On grids of 32^3 and less
    the iteration counts are too small for the saving to show at equal iterations.)"""
    from paper_math_0609672_amd import budget as LB
    Xs, ys = [], []
    for seed in (1, 2, 3, 4):
        A = W.config_grid3d(64, seed)
        X, y = LB.pilot_rows(srw.Matrix.from_host(A, DEV), seed, 256, 1e-4, rule="sqrt")
        Xs.append(X)
        ys.append(y)
    # about as many Adam steps as the bench's 20 pilots x 4 epochs
    model = LB.fit(torch.cat(Xs), torch.cat(ys), epochs=20, batch=65536, lr=2e-3)
    del Xs, ys
    A = W.config_grid3d(128, 0)
    M = srw.Matrix.from_host(A, DEV)
    b = torch.as_tensor(W.rhs(A.n, seed=0), device=DEV)

    def solve(walks=None):
        F = srw.build_factor(M, 256, 1e-4, 0, walks=walks)
        st, _, it, rel = srw.pcg_solve(M, F, b, 1e-8, 1000)
        steps = F.stats()["walk_steps"]
        F.free()
        assert st == srw.OK and rel <= 1e-8
        return it, steps

    it_u, steps_u = solve()
    found = []
    for eps in np.geomspace(3e-3, 8e-3, 8):
        it, steps = solve(LB.budgets(model, M, 0, float(eps), lo=8, hi=8192))
        found.append((float(eps), it, steps))
        if it <= it_u and steps < 0.9 * steps_u:
            return
    raise AssertionError((it_u, steps_u, found))
