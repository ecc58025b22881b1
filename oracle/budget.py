"""CPU oracle of the learned walk-budget allocator (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``; the product path never imports it.  Plain numpy in
float64, one formula per function, no blocking or fusion.

The allocator is not in the paper.  The paper fixes the number of walks per row by a
stopping rule on the sample mean of the walk lengths (Section 5.1); here a small
network predicts, from cheap per-row graph features, the per-walk variance of a
row's estimates, and a row's budget is that variance over a target.  Its parts:

* ``features``: eight per-row quantities of A and the ordering (Section 2.1 game:
  a_k, the conductances w_kj = -A_kj, the excess e_k; Section 5.4 ordering).
* ``label``: the per-walk variance of row k's stochastic estimates, from the tallies
  of a pilot run (Section 3.1 M, H, J and the stays' second moment):
      V_k = tau_k^2 * sum_i p_i (1 - p_i)  +  (tau_k / (1 + tau_k (m - 1)))^2 * s^2
  with p_i = H_ki / M (ground excluded), m = J_k / M the mean stays and s^2 their
  sample variance.  The first term is the variance of one walk's contribution to the
  Y entries of eq. newy (tau_k H / M per entry); the second is the first-order
  relative variance of D_k of eq. d in the mean stays.  A budget M_k = V_k / eps makes
  every row's estimate variance about eps.  Divided by the row's mean walk length L_k
  it is the variance bought per step; budgets M_k proportional to sqrt(V_k / L_k)
  minimise sum_k V_k / M_k at a fixed total sum_k M_k L_k of steps (Lagrange).
* ``mlp_forward`` / ``mlp_backward``: 8 -> 64 -> 64 -> 1 with ReLU, optional rounding
  of the operands to bfloat16 (round to nearest even) as the GPU kernels use them.
* ``adam_step``: Adam (Kingma and Ba) on float64 copies of the parameters.
"""
from __future__ import annotations

import numpy as np

NF = 8          # features per row
H = 64          # hidden width
FEATURE_NAMES = ("degree", "log_diag", "excess_ratio", "tau", "motel_fraction",
                 "log_weight_spread", "log_n_over_rank", "mean_neighbour_excess_ratio")


def features(A, rank: np.ndarray) -> np.ndarray:
    """float64 [n, 8] per-row features, one row at a time:
    0 degree (off-diagonal entries), 1 log a_k, 2 e_k / a_k, 3 tau_k (higher-ranked
    neighbours' conductance over a_k), 4 fraction of neighbours ranked above k,
    5 log(max w / min w) over the row (0 without neighbours), 6 log(n / (rank_k + 1)),
    7 mean over neighbours j of e_j / a_j (0 without neighbours)."""
    n = A.n
    rank = np.asarray(rank)
    diag = np.zeros(n)
    excess = np.zeros(n)
    for k in range(n):
        s = 0.0
        for q in range(A.rowptr[k], A.rowptr[k + 1]):
            j = A.col[q]
            if j == k:
                diag[k] = A.val[q]
            else:
                s += -A.val[q]
        excess[k] = diag[k] - s
    out = np.zeros((n, NF))
    for k in range(n):
        w, higher, ratio = [], 0, []
        motel = 0.0
        for q in range(A.rowptr[k], A.rowptr[k + 1]):
            j = A.col[q]
            if j == k:
                continue
            w.append(-A.val[q])
            if rank[j] > rank[k]:
                higher += 1
                motel += -A.val[q]
            ratio.append(excess[j] / diag[j])
        deg = len(w)
        out[k, 0] = deg
        out[k, 1] = np.log(diag[k])
        out[k, 2] = excess[k] / diag[k]
        out[k, 3] = motel / diag[k]
        out[k, 4] = higher / deg if deg else 0.0
        out[k, 5] = np.log(max(w) / min(w)) if deg else 0.0
        out[k, 6] = np.log(n / (rank[k] + 1.0))
        out[k, 7] = sum(ratio) / deg if deg else 0.0
    return out


def label(tau: float, M: int, J: int, visits_sq: int, h_cnt, steps: int | None = None) -> float:
    """Per-walk variance V_k of one row from its pilot tallies (see module text);
    h_cnt lists H_ki over the row's home nodes (ground excluded).  With `steps` (the
    row's total walk steps) the variance per step: V_k / (steps / M)."""
    M = float(M)
    m = J / M
    s2 = (visits_sq - M * m * m) / (M - 1.0) if M > 1 else 0.0
    if s2 < 0.0:
        s2 = 0.0
    var_y = 0.0
    for h in h_cnt:
        p = h / M
        var_y += p * (1.0 - p)
    c = tau / (1.0 + tau * (m - 1.0))
    v = tau * tau * var_y + c * c * s2
    if steps is not None:
        v = v / (steps / M)
    return v


def labels(tau: np.ndarray, tallies, per_step: bool = False) -> np.ndarray:
    """V_k (or V_k per step) for every row of an all-rows tally (rows without walks
    give NaN)."""
    n = tau.size
    out = np.full(n, np.nan)
    for k in range(n):
        M = int(tallies.walks[k])
        if M == 0:
            continue
        a = int(tallies.h_off[k])
        h = [int(c) for c, e in zip(tallies.h_cnt[a:a + int(tallies.hlen[k])],
                                    tallies.h_end[a:a + int(tallies.hlen[k])]) if e >= 0]
        out[k] = label(float(tau[k]), M, int(tallies.J[k]), int(tallies.visits_sq[k]), h,
                       int(tallies.steps[k]) if per_step else None)
    return out


# ------------------------------------------------------------------ the network
def bf16(x: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (round to nearest, ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def init_params(seed: int = 0) -> dict:
    """He-uniform weights, zero biases; float64."""
    rng = np.random.default_rng([seed, 0xB0D6E7])
    def he(fan_in, shape):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, shape)
    return {"W1": he(NF, (NF, H)), "b1": np.zeros(H), "W2": he(H, (H, H)), "b2": np.zeros(H),
            "W3": he(H, (H,)), "b3": np.zeros(1)}


def standardize(X: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    return (X - mu) / sd


def mlp_forward(p: dict, X: np.ndarray, round_bf16: bool = False):
    """y = W3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 per row of X [B, 8].
    With round_bf16 the inputs, weights and first hidden layer are rounded to
    bfloat16 before each product (products and sums stay exact in float64)."""
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    X = r(X)
    z1 = X @ r(p["W1"]) + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1r = r(h1)
    z2 = h1r @ r(p["W2"]) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    h2r = r(h2)
    y = h2r @ r(p["W3"]) + p["b3"][0]
    cache = {"X": X, "z1": z1, "h1": h1r, "z2": z2, "h2": h2r, "W2": r(p["W2"]), "W3": r(p["W3"]),
             "round": round_bf16}
    return y, cache


def mse(y: np.ndarray, t: np.ndarray) -> float:
    return float(np.mean((y - t) ** 2))


def mlp_backward(p: dict, cache: dict, dy: np.ndarray) -> dict:
    """Gradients of sum(dy * y) with respect to every parameter (chain rule of the
    forward pass above, the rounded operands treated as constants).  When the forward
    pass rounded its operands, the pre-activation gradients dZ2 and dZ1 are rounded to
    bfloat16 too before they enter a product, as the GPU kernels do."""
    r = bf16 if cache.get("round") else (lambda v: v)
    g = {}
    g["W3"] = cache["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = r(np.outer(dy, cache["W3"]) * (cache["z2"] > 0))
    g["W2"] = cache["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = r((dz2 @ cache["W2"].T) * (cache["z1"] > 0))
    g["W1"] = cache["X"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def loss_and_grads(p: dict, X: np.ndarray, t: np.ndarray, round_bf16: bool = False):
    """Mean squared error over the batch and its gradients."""
    y, cache = mlp_forward(p, X, round_bf16)
    dy = 2.0 * (y - t) / y.size
    return mse(y, t), mlp_backward(p, cache, dy)


def adam_state(p: dict) -> dict:
    return {"t": 0, "m": {k: np.zeros_like(v) for k, v in p.items()},
            "v": {k: np.zeros_like(v) for k, v in p.items()}}


def adam_step(p: dict, g: dict, st: dict, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    """One Adam update in place: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
    st["t"] += 1
    t = st["t"]
    for k in p:
        st["m"][k] = beta1 * st["m"][k] + (1.0 - beta1) * g[k]
        st["v"][k] = beta2 * st["v"][k] + (1.0 - beta2) * g[k] * g[k]
        mh = st["m"][k] / (1.0 - beta1 ** t)
        vh = st["v"][k] / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def budgets(pred_log_v: np.ndarray, tau: np.ndarray, eps: float, lo: int, hi: int) -> np.ndarray:
    """Walks per row: ceil(exp(pred) / eps) clamped to [lo, hi]; 0 for rows whose
    factor row is exact (tau = 0, no walks, Section 5.2)."""
    m = np.ceil(np.exp(pred_log_v) / eps)
    m = np.clip(m, lo, hi).astype(np.int64)
    m[tau <= 0.0] = 0
    return m.astype(np.int32)
