"""Dense closed forms that pin the oracle (test infrastructure only).

Everything here is computed from a small dense matrix by textbook linear algebra,
independently of the walk code:

* ``rev`` -- the reversal operator of the paper's Definition (Section 3.1).
* ``exact_factor_schur`` -- the limit of the random-walk factor: for each node k,
  eliminate every node ranked above k; with S the Schur complement left on the nodes
  of rank <= rank(k), Y_ki -> S_ki / S_kk and D_k -> S_kk.  This is the exact LDL^T of
  the reverse-ordered matrix (eqs. y and d), written out one row at a time.
* ``exact_factor_cholesky`` -- the same factor read off numpy's Cholesky of the
  reverse-ordered matrix (Lemma on UL/LU under rev, Doolittle uniqueness); the two
  routes must agree.
* ``walk_limits`` -- the absorbing Markov chain of the game (Section 2.1) with homes
  at lower ranks and at ground (Section 2.2.1), solved with its fundamental matrix:
  end-node probabilities, expected stays at the start node and expected length,
  unconditionally and conditioned on a first step to a motel (Section 5.2).
"""
from __future__ import annotations

import numpy as np


def rev(M: np.ndarray) -> np.ndarray:
    """rev(M)_{i,j} = M_{N+1-i, N+1-j} (vectors: rev(x)_i = x_{N+1-i})."""
    M = np.asarray(M)
    if M.ndim == 1:
        return M[::-1].copy()
    return M[::-1, ::-1].copy()


def exact_factor_schur(A: np.ndarray, rank: np.ndarray):
    """(Y, D): Y unit lower in rank order (dense, node indices), D diagonal."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Y = np.eye(n)
    D = np.zeros(n)
    for k in range(n):
        E = np.flatnonzero(rank > rank[k])
        R = np.flatnonzero(rank <= rank[k])
        S = A[np.ix_(R, R)]
        if E.size:
            S = S - A[np.ix_(R, E)] @ np.linalg.solve(A[np.ix_(E, E)], A[np.ix_(E, R)])
        kk = int(np.flatnonzero(R == k)[0])
        D[k] = S[kk, kk]
        for a, i in enumerate(R):
            if i != k:
                Y[k, i] = S[kk, a] / S[kk, kk]
    return Y, D


def exact_factor_cholesky(A: np.ndarray, rank: np.ndarray):
    """Same (Y, D) from numpy's Cholesky of rev(P A P^T), P sorting nodes by rank."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    by_rank = np.argsort(rank)
    B = rev(A[np.ix_(by_rank, by_rank)])  # position p <-> node of rank n-1-p
    C = np.linalg.cholesky(B)
    dc = np.diag(C)
    L = C / dc[None, :]
    node = by_rank[::-1]  # node at reversed position p
    Y = np.eye(n)
    D = np.zeros(n)
    for b in range(n):
        D[node[b]] = dc[b] ** 2
        for a in range(b + 1, n):
            Y[node[b], node[a]] = L[a, b]
    return Y, D


def walk_limits(A: np.ndarray, rank: np.ndarray, k: int):
    """Limits for walks from node k with motels {j: rank_j >= rank_k} and homes the
    lower-ranked nodes plus ground.

    Returns a dict with
      q        end-node probabilities of an unconditioned walk (length n, ground in
               key 'q_ground'),
      visits   expected stays at k (start included), unconditioned,
      p, p_ground, visits_motel, length_motel
               the same conditioned on a first step to a motel (None if k has no
               motel neighbour), i.e. what one simulated walk of the exact one-step
               treatment estimates.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    a = np.diag(A).copy()
    P = -A / a[:, None]
    np.fill_diagonal(P, 0.0)
    g = A.sum(axis=1) / a  # probability of a step to ground
    T = np.flatnonzero(rank >= rank[k])
    H = np.flatnonzero(rank < rank[k])
    N = np.linalg.inv(np.eye(T.size) - P[np.ix_(T, T)])  # fundamental matrix
    pos = {int(v): i for i, v in enumerate(T)}
    kk = pos[int(k)]
    absorb = N @ P[np.ix_(T, H)]          # [transient start, home]
    absorb_g = N @ g[T]
    q = np.zeros(n)
    q[H] = absorb[kk]
    out = {"q": q, "q_ground": float(absorb_g[kk]), "visits": float(N[kk, kk])}
    motel_nbrs = [j for j in T if j != k and A[k, j] != 0.0]
    if not motel_nbrs:
        out.update(p=None, p_ground=None, visits_motel=None, length_motel=None)
        return out
    w = np.array([-A[k, j] for j in motel_nbrs])
    f = w / w.sum()
    rows = [pos[int(j)] for j in motel_nbrs]
    p = np.zeros(n)
    p[H] = f @ absorb[rows]
    out["p"] = p
    out["p_ground"] = float(f @ absorb_g[rows])
    out["visits_motel"] = 1.0 + float(f @ N[rows, kk])
    out["length_motel"] = 1.0 + float(f @ N[rows].sum(axis=1))
    return out


def reachable_through_higher(A: np.ndarray, rank: np.ndarray, k: int) -> set:
    """Nodes i with rank_i < rank_k reachable from k through nodes ranked above k
    (Section 3.2, Definition of reachability): the pattern bound of row k."""
    A = np.asarray(A)
    n = A.shape[0]
    seen = {k}
    stack = [k]
    out = set()
    while stack:
        v = stack.pop()
        for j in np.flatnonzero(A[v] != 0):
            j = int(j)
            if j == v or j in seen:
                continue
            seen.add(j)
            if rank[j] < rank[k]:
                out.add(j)
            else:
                stack.append(j)
    return out
