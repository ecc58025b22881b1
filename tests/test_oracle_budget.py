"""Pins of the walk-budget allocator oracle (oracle/budget.py) against things fixed
outside it: hand-computed features, the exact absorbing-chain variance of a row's
walk outcomes, finite differences, bfloat16 rounding of a library, Adam's
constant-gradient step."""
import numpy as np
import pytest

import oracle as O
from oracle import budget as B
from oracle import dense
from paper_math_0609672_amd import workloads as W


def test_features_hand_computed():
    # path 0 - 1 - 2, conductances 2 and 0.5; excess 1 at node 0, 0 at 1, 0.25 at 2
    A = W.assemble(3, np.array([0, 1]), np.array([1, 2]), np.array([2.0, 0.5]),
                   np.array([1.0, 0.0, 0.25]))
    rank = np.array([1, 2, 0])  # node 2 lowest, node 1 highest
    F = B.features(A, rank)
    a = np.array([3.0, 2.5, 0.75])
    exp = np.array([
        # deg, log a, e/a, tau, higher/deg, log spread, log(n/(r+1)), mean nbr e/a
        [1, np.log(3.0), 1 / 3, 2.0 / 3.0, 1.0, 0.0, np.log(3 / 2), 0.0 / 2.5],
        [2, np.log(2.5), 0.0, 0.0, 0.0, np.log(4.0), np.log(3 / 3), (1 / 3 + 0.25 / 0.75) / 2],
        [1, np.log(0.75), 0.25 / 0.75, 0.5 / 0.75, 1.0, 0.0, np.log(3 / 1), 0.0],
    ])
    assert np.allclose(F, exp, rtol=0, atol=1e-15)
    assert np.allclose(a, np.exp(F[:, 1]))


def _exact_label(Ad, rank, k):
    """V_k from the absorbing chain of the game with homes = lower ranks + ground:
    end probabilities p (conditioned on the first step to a motel) and the variance
    of the stays S = 1 + V, where V = 0 if the walk never comes back to k and is
    geometric with mean N_kk once it does (N = fundamental matrix)."""
    lim = dense.walk_limits(Ad, rank, k)
    n = Ad.shape[0]
    a = np.diag(Ad)
    P = -Ad / a[:, None]
    np.fill_diagonal(P, 0.0)
    T = np.flatnonzero(rank >= rank[k])
    N = np.linalg.inv(np.eye(T.size) - P[np.ix_(T, T)])
    pos = {int(v): i for i, v in enumerate(T)}
    kk = pos[k]
    motel = [j for j in T if j != k and Ad[k, j] != 0]
    w = np.array([-Ad[k, j] for j in motel])
    f = w / w.sum()
    hbar = float(f @ N[[pos[int(j)] for j in motel], kk]) / N[kk, kk]
    Nkk = N[kk, kk]
    EV = hbar * Nkk
    EV2 = hbar * (2 * Nkk ** 2 - Nkk)
    var_s = EV2 - EV ** 2
    m = 1.0 + EV
    assert abs(m - lim["visits_motel"]) < 1e-12
    tau = w.sum() / a[k]
    p = lim["p"]
    var_y = float(np.sum(p * (1 - p)))
    c = tau / (1 + tau * (m - 1))
    return tau * tau * var_y + c * c * var_s


@pytest.mark.parametrize("seed", [2, 5])
def test_label_converges_to_exact_chain_variance(seed):
    A = W.random_graph(9, 16, seed=seed, ground_frac=0.2)
    Ad = A.dense()
    rk = O.rank(A.n, seed)
    tb = O.table(A, rk)
    ks = [k for k in range(A.n) if tb.tau[k] > 0]
    M = 1 << 16
    wk = O.walk_rows(A, rk, tb, seed, np.array(ks), M)
    tl = O.tally(wk)
    for r, k in enumerate(ks):
        a = int(tl.h_off[r])
        L = int(tl.hlen[r])
        h = [int(c) for c, e in zip(tl.h_cnt[a:a + L], tl.h_end[a:a + L]) if e >= 0]
        est = B.label(float(tb.tau[k]), int(tl.walks[r]), int(tl.J[r]), int(tl.visits_sq[r]), h)
        ex = _exact_label(Ad, rk, k)
        assert abs(est - ex) <= 0.05 * ex + 1e-4, (k, est, ex)


def test_label_plants():
    # a dropped (1 - p) or a missing stays term moves the value far from the chain
    tau, M = 0.5, 1000
    h = [300, 200]
    v = B.label(tau, M, J=1500, visits_sq=2900, h_cnt=h)
    py = 0.3 * 0.7 + 0.2 * 0.8
    m = 1.5
    s2 = (2900 - M * m * m) / (M - 1)
    assert v == pytest.approx(tau ** 2 * py + (tau / (1 + tau * (m - 1))) ** 2 * s2, rel=1e-15)
    assert B.label(tau, M, J=M, visits_sq=M, h_cnt=[M]) == 0.0  # deterministic row


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(B.bf16(x), ref)


@pytest.mark.parametrize("round_bf16", [False, True])
def test_mlp_gradients_finite_differences(round_bf16):
    rng = np.random.default_rng(3)
    p = B.init_params(4)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((32, B.NF))
    t = rng.standard_normal(32)
    loss, g = B.loss_and_grads(p, X, t, round_bf16=False)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = B.mse(B.mlp_forward(p, X)[0], t)
            flat[idx] = old - h
            lm = B.mse(B.mlp_forward(p, X)[0], t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)
    if round_bf16:
        # rounding the operands changes the loss only at bfloat16 resolution
        loss_b, _ = B.loss_and_grads(p, X, t, round_bf16=True)
        assert abs(loss_b - loss) <= 0.05 * loss


def test_adam_constant_gradient_steps_are_lr():
    # with a constant gradient the bias-corrected moments are g and g^2 at every step
    p = {"w": np.array([1.0, -2.0, 0.5])}
    st = B.adam_state(p)
    g = {"w": np.array([0.3, -4.0, 1e-3])}
    for t in range(1, 6):
        before = p["w"].copy()
        B.adam_step(p, g, st, lr=0.01)
        step = before - p["w"]
        assert np.allclose(step, 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((512, B.NF))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 3] * X[:, 5] - 0.25 * X[:, 6]
    p = B.init_params(1)
    st = B.adam_state(p)
    l0, _ = B.loss_and_grads(p, X, t)
    for _ in range(400):
        _, g = B.loss_and_grads(p, X, t)
        B.adam_step(p, g, st, lr=3e-3)
    l1, _ = B.loss_and_grads(p, X, t)
    assert l1 < 0.1 * l0


def test_budgets():
    pred = np.log(np.array([0.5, 1.0, 30.004, 1e9, 2.0]))
    tau = np.array([0.1, 0.2, 0.3, 0.4, 0.0])
    m = B.budgets(pred, tau, eps=0.01, lo=8, hi=4096)
    assert m.tolist() == [50, 100, 3001, 4096, 0]


def test_label_per_step_and_allocation_optimum():
    # per-step label = label / (steps / M)
    v = B.label(0.5, 1000, 1500, 2900, [300, 200])
    assert B.label(0.5, 1000, 1500, 2900, [300, 200], steps=40000) == pytest.approx(v / 40.0, rel=1e-15)
    # M_k ~ sqrt(V_k / L_k) minimises sum V/M at fixed sum M L: any feasible perturbation
    # of the optimum raises the objective
    rng = np.random.default_rng(2)
    V, L = rng.uniform(0.1, 10, 50), rng.uniform(1, 100, 50)
    budget = 1e5
    M = np.sqrt(V / L)
    M *= budget / np.sum(M * L)
    f0 = np.sum(V / M)
    for _ in range(200):
        d = rng.standard_normal(50) * 0.05 * M
        d -= L * (np.sum(d * L) / np.sum(L * L))  # keep the step budget
        if np.all(M + d > 0):
            assert np.sum(V / (M + d)) >= f0 * (1 - 1e-12)
