"""Learned walk budgets: training data from pilot factors, training and use of the
8 -> 64 -> 64 -> 1 network, all through the C ABI (srw.py); every step of the
arithmetic runs in the library's kernels.

A row's label is the per-walk variance of its estimates measured on a pilot factor
(srw_budget_labels); the network learns a target from the row's features
(srw_row_features) and a row's budget is exp(prediction) / eps (srw_mlp_budgets).
Three rules:
  "equal"   target log V_k: every row gets variance about eps;
  "sqrt"    target (1/2) log V_k: budgets proportional to sqrt(V_k), the least summed
            variance for a given number of walks;
  "neyman"  target (1/2) log(V_k / L_k), L_k the mean walk length: budgets
            proportional to sqrt(V_k / L_k), the least summed variance for a given
            number of walk steps.
The plain method (the same walks for every row) is the fallback and the reference.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import srw


@dataclass
class Model:
    params: torch.Tensor   # float32 [SRW_MLP_PARAMS]
    mu_sd: torch.Tensor    # float32 [16]
    history: list          # (step, loss) pairs

    def predict(self, features: torch.Tensor) -> torch.Tensor:
        return srw.mlp_forward(self.params, self.mu_sd, features)


RULES = ("equal", "sqrt", "neyman")


def pilot_rows(M: srw.Matrix, seed: int, walks: int, drop_tol: float, rule: str = "neyman"):
    """Features and targets of the rows of one matrix with a positive finite label,
    from a pilot factor with `walks` walks per row."""
    if rule not in RULES:
        raise ValueError(rule)
    F = srw.build_factor(M, walks, drop_tol, seed, keep=1)
    lab = srw.budget_labels(F, per_step=rule == "neyman")
    F.free()
    feat = srw.row_features(M, srw.ordering(M.n, seed, M.rowptr.device))
    return srw.budget_targets(lab, feat, rule != "equal")


def init_params(seed: int, device) -> torch.Tensor:
    """He-uniform weights, zero biases (the layout of SRW_MLP_PARAMS)."""
    g = torch.Generator().manual_seed(int(seed))

    def he(fan_in, n):
        lim = math.sqrt(6.0 / fan_in)
        return (torch.rand(n, generator=g, dtype=torch.float64) * 2 - 1) * lim

    parts = [he(8, 8 * 64), torch.zeros(64, dtype=torch.float64), he(64, 64 * 64),
             torch.zeros(64, dtype=torch.float64), he(64, 64), torch.zeros(1, dtype=torch.float64)]
    p = torch.cat(parts).to(torch.float32)
    assert p.numel() == srw.MLP_PARAMS
    return p.to(device)


def fit(X: torch.Tensor, y: torch.Tensor, *, epochs: int = 4, batch: int = 65536,
        lr: float = 2e-3, seed: int = 0, log_every: int = 50) -> Model:
    """Adam on the mean squared error of log(label), minibatches of `batch` rows taken
    in the order of a seeded random permutation per epoch (srw_ordering's ranks, which
    are one) and gathered inside the training kernel.  Input scaling and the output
    bias's start (the mean target) come from srw_mlp_standardize."""
    dev = X.device
    X = X.contiguous()
    y = y.contiguous()
    mu_sd, y_mean = srw.mlp_standardize(X, y)
    P = init_params(seed, dev)
    P[-1:].copy_(y_mean)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    hist = []
    step = 0
    n = X.shape[0]
    for epoch in range(epochs):
        perm = srw.ordering(n, (int(seed) << 16) + epoch + 1, dev)
        for s in range(0, n, batch):
            step += 1
            srw.mlp_train_step_rows(P, mu_sd, X, y, perm[s:s + batch], adam_m=m, adam_v=v,
                                    step=step, lr=lr, loss=loss)
            if step % log_every == 0 or step == 1:
                hist.append((step, float(loss.item())))
    hist.append((step, float(loss.item())))
    return Model(P, mu_sd, hist)


def budgets(model: Model, M: srw.Matrix, seed: int, eps: float, lo: int = 8,
            hi: int = 8192) -> torch.Tensor:
    """Walks per row for the matrix built with `seed`: exp(prediction) / eps, clamped."""
    feat = srw.row_features(M, srw.ordering(M.n, seed, M.rowptr.device))
    return srw.mlp_budgets(model.predict(feat), eps, lo, hi)
