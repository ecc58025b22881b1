"""Seeded synthetic R-matrix workloads.

This module only manufactures inputs: symmetric, irreducibly diagonally dominant
M-matrices ("R-matrices", paper Section 1) in CSR form and right-hand sides.  It
holds none of the preconditioner's arithmetic, so both the CPU oracle tests and
the GPU path may use it.

Every generator is deterministic in its seed (numpy ``default_rng``), and the order
of random draws is fixed: edge conductances in edge order, then the grounded node
set, then the grounding excess.  Right-hand sides come from an independent stream.

Resistor-network reading (paper Section 2.1): an off-diagonal entry A_kj = -g_kj is
the conductance between nodes k and j, the diagonal is the sum of incident
conductances plus a grounding excess e_k >= 0, and a node with e_k > 0 is a path to
ground (an initial home of the walk game).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Square sparse matrix: int64 rowptr[n+1], int32 col[nnz] (sorted per row,
    diagonal stored), float64 val[nnz]."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def assemble(n: int, eu: np.ndarray, ev: np.ndarray, g: np.ndarray, excess: np.ndarray) -> CSR:
    """Symmetric CSR from an undirected edge list (eu[e], ev[e]) with conductance g[e]
    and per-node grounding excess; diagonal = incident conductances + excess."""
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    g = np.asarray(g, dtype=np.float64)
    excess = np.asarray(excess, dtype=np.float64)
    if eu.size and (np.any(eu == ev) or np.any(g <= 0)):
        raise ValueError("edges must join distinct nodes with positive conductance")
    diag = np.bincount(eu, g, minlength=n) + np.bincount(ev, g, minlength=n) + excess
    rows = np.concatenate([eu, ev, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([ev, eu, np.arange(n, dtype=np.int64)])
    vals = np.concatenate([-g, -g, diag])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if np.any(dup):
            raise ValueError("duplicate edge")
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(n, rowptr, cols.astype(np.int32), vals.astype(np.float64))


def assemble_directed(n: int, eu: np.ndarray, ev: np.ndarray, g_uv: np.ndarray, g_vu: np.ndarray,
                      excess: np.ndarray) -> CSR:
    """Structurally symmetric CSR with asymmetric values: A_uv = -g_uv, A_vu = -g_vu for
    every undirected edge (eu[e], ev[e]); the diagonal is the larger of the node's
    off-diagonal row and column sums plus its excess, so the matrix is diagonally
    dominant by rows and by columns (both walk games of the matrix and of its transpose
    are defined), with strict dominance at the nodes of positive excess."""
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    g_uv = np.asarray(g_uv, dtype=np.float64)
    g_vu = np.asarray(g_vu, dtype=np.float64)
    excess = np.asarray(excess, dtype=np.float64)
    if eu.size and (np.any(eu == ev) or np.any(g_uv <= 0) or np.any(g_vu <= 0)):
        raise ValueError("edges must join distinct nodes with positive weights")
    rowsum = np.bincount(eu, g_uv, minlength=n) + np.bincount(ev, g_vu, minlength=n)
    colsum = np.bincount(ev, g_uv, minlength=n) + np.bincount(eu, g_vu, minlength=n)
    diag = np.maximum(rowsum, colsum) + excess
    rows = np.concatenate([eu, ev, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([ev, eu, np.arange(n, dtype=np.int64)])
    vals = np.concatenate([-g_uv, -g_vu, diag])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if np.any(dup):
            raise ValueError("duplicate edge")
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(n, rowptr, cols.astype(np.int32), vals.astype(np.float64))


def grid_asym(dims, *, g=("uniform", 0.5, 1.5), skew=0.5, ground_frac=0.05, min_ground=1,
              excess=("uniform", 0.1, 1.0), seed=0) -> CSR:
    """Grid with asymmetric couplings: each edge's conductance g is split into
    g(1 + t) one way and g(1 - t) the other, t ~ U[-skew, skew] per edge (skew < 1);
    grounded nodes and excess as in `grid`."""
    rng = np.random.default_rng(seed)
    eu, ev = grid_edges(dims)
    n = int(np.prod(dims))
    gv = _draw(rng, g, eu.size)
    t = rng.uniform(-skew, skew, eu.size)
    exc = _ground(rng, n, ground_frac, min_ground, excess)
    return assemble_directed(n, eu, ev, gv * (1.0 + t), gv * (1.0 - t), exc)


def transpose(A: CSR) -> CSR:
    """CSR of A^T (columns sorted per row)."""
    T = A.to_scipy().T.tocsr()
    T.sort_indices()
    return CSR(A.n, T.indptr.astype(np.int64), T.indices.astype(np.int32), T.data.astype(np.float64))


def _draw(rng, spec, size):
    kind, lo, hi = spec
    if kind == "uniform":
        return rng.uniform(lo, hi, size)
    if kind == "loguniform":
        return np.exp(rng.uniform(np.log(lo), np.log(hi), size))
    if kind == "const":
        return np.full(size, float(lo))
    raise ValueError(kind)


def _ground(rng, n, frac, min_count, exc_spec):
    ng = max(int(round(frac * n)), min_count)
    ng = min(ng, n)
    nodes = rng.choice(n, size=ng, replace=False)
    excess = np.zeros(n)
    excess[nodes] = _draw(rng, exc_spec, ng)
    return excess


def grid_edges(dims) -> tuple[np.ndarray, np.ndarray]:
    """Nearest-neighbour edges of a regular grid; node id = x + nx*(y + ny*z).
    Edges are listed direction by direction (x, then y, then z)."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    ids = np.arange(n, dtype=np.int64).reshape(dims[::-1])  # [z][y][x]
    us, vs = [], []
    nd = len(dims)
    for axis in range(nd):
        ax = nd - 1 - axis  # numpy axis of this grid direction
        sl_a = [slice(None)] * nd
        sl_b = [slice(None)] * nd
        sl_a[ax] = slice(0, dims[axis] - 1)
        sl_b[ax] = slice(1, dims[axis])
        us.append(ids[tuple(sl_a)].ravel())
        vs.append(ids[tuple(sl_b)].ravel())
    return np.concatenate(us), np.concatenate(vs)


def grid(dims, *, g=("uniform", 0.5, 1.5), ground_frac=0.05, min_ground=1,
         excess=("uniform", 0.1, 1.0), seed=0) -> CSR:
    """Resistor grid (2D 5-point or 3D 7-point): conductances drawn per edge,
    round(ground_frac*n) (at least min_ground) grounded nodes drawn without
    replacement, each with an excess drawn from `excess`."""
    rng = np.random.default_rng(seed)
    eu, ev = grid_edges(dims)
    n = int(np.prod(dims))
    gv = _draw(rng, g, eu.size)
    exc = _ground(rng, n, ground_frac, min_ground, excess)
    return assemble(n, eu, ev, gv, exc)


def laplace3d_dirichlet(m: int) -> CSR:
    """7-point finite-difference Laplacian on an m^3 interior grid with Dirichlet
    boundary: diagonal 6, off-diagonal -1 (the paper's m1-m6 family, Section 6)."""
    eu, ev = grid_edges((m, m, m))
    n = m ** 3
    deg = np.bincount(eu, minlength=n) + np.bincount(ev, minlength=n)
    return assemble(n, eu, ev, np.ones(eu.size), (6 - deg).astype(np.float64))


def from_dense(a: np.ndarray) -> CSR:
    """CSR of a small dense matrix (stored pattern = nonzeros + diagonal)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    mask = (a != 0) | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(n, rowptr, cols.astype(np.int32), a[rows, cols].copy())


def random_graph(n: int, n_edges: int, *, g=("uniform", 0.1, 10.0), ground_frac=0.05,
                 min_ground=1, excess=("uniform", 0.1, 1.0), seed=0, connected=True) -> CSR:
    """Random sparse graph: a random spanning tree (if `connected`) plus extra
    uniformly random distinct edges; small irregular test inputs."""
    rng = np.random.default_rng(seed)
    edges = set()
    if connected and n > 1:
        perm = rng.permutation(n)
        for i in range(1, n):
            j = perm[rng.integers(0, i)]
            u, v = int(perm[i]), int(j)
            edges.add((min(u, v), max(u, v)))
    target = min(n_edges, n * (n - 1) // 2)
    while len(edges) < target:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v:
            edges.add((min(u, v), max(u, v)))
    e = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
    gv = _draw(rng, g, e.shape[0])
    exc = _ground(rng, n, ground_frac, min_ground, excess)
    return assemble(n, e[:, 0], e[:, 1], gv, exc)


def rhs(n: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """Right-hand side(s) b ~ N(0, 1), from a stream independent of the matrix."""
    rng = np.random.default_rng([int(seed), 0x5EED])
    b = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    return b


# --- the named workloads (sizes and distributions of the method's test matrices) ---

def config_grid2d_32(seed: int = 0) -> CSR:
    """2D 5-point 32x32 resistor grid, g ~ U[0.5, 1.5], 5% grounded (>= 1) with
    excess ~ U[0.1, 1.0]; n = 1024."""
    return grid((32, 32), g=("uniform", 0.5, 1.5), ground_frac=0.05,
                excess=("uniform", 0.1, 1.0), seed=seed)


def config_grid3d(m: int = 128, seed: int = 0) -> CSR:
    """3D 7-point m^3 resistor grid, g log-uniform on [1e-2, 1e2] per edge, 1%
    grounded with excess ~ U[0.01, 1]; m = 128 gives n = 2,097,152."""
    return grid((m, m, m), g=("loguniform", 1e-2, 1e2), ground_frac=0.01,
                excess=("uniform", 0.01, 1.0), seed=seed)


def config_grid3d_asym(m: int = 128, seed: int = 0) -> CSR:
    """3D 7-point m^3 grid with asymmetric couplings: g log-uniform on [1e-2, 1e2] per
    edge split (1 + t, 1 - t), t ~ U[-0.5, 0.5]; 1% grounded with excess ~ U[0.01, 1]."""
    return grid_asym((m, m, m), g=("loguniform", 1e-2, 1e2), skew=0.5, ground_frac=0.01,
                     excess=("uniform", 0.01, 1.0), seed=seed)


def rgg_connect_probability(r: float) -> float:
    """Probability that two independent uniform points of the unit cube lie within
    distance r <= 1: the integral of prod_i (1 - |d_i|) over the ball |d| <= r,
    (4 pi/3) r^3 - (3 pi/2) r^4 + (8/5) r^5 - r^6 / 6 (boundary effects included)."""
    r = float(r)
    return 4.0 * np.pi / 3.0 * r ** 3 - 1.5 * np.pi * r ** 4 + 1.6 * r ** 5 - r ** 6 / 6.0


def _rgg_pairs(pts: np.ndarray, r: float):
    """All pairs u < v of points closer than r, by a cell list with cell side >= r:
    each cell meets itself and 13 of its 26 neighbour cells (one of each opposite
    pair).  Returns (u, v, dist)."""
    n = pts.shape[0]
    m = max(1, int(np.floor(1.0 / r)))
    cell = np.minimum((pts * m).astype(np.int64), m - 1)
    cid = cell[:, 0] + m * (cell[:, 1] + m * cell[:, 2])
    order = np.argsort(cid, kind="stable")
    cs = cid[order]
    start = np.searchsorted(cs, np.arange(m ** 3 + 1))
    cnt = np.diff(start)
    offs = [(0, 0, 0)] + [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                          if (dz, dy, dx) > (0, 0, 0)]
    us, vs, ds = [], [], []
    r2 = r * r
    pc = cell[order]
    for dx, dy, dz in offs:
        nc = pc + np.array([dx, dy, dz])
        ok = np.all((nc >= 0) & (nc < m), axis=1)
        src = np.nonzero(ok)[0]  # positions in sorted order
        ncid = nc[src, 0] + m * (nc[src, 1] + m * nc[src, 2])
        k = cnt[ncid]
        if (dx, dy, dz) == (0, 0, 0):
            # same cell: partners after the point itself
            k = start[ncid + 1] - (src + 1)
            base = src + 1
        else:
            base = start[ncid]
        tot = int(k.sum())
        if tot == 0:
            continue
        a = np.repeat(src, k)
        first = np.repeat(base - np.concatenate(([0], np.cumsum(k)[:-1])), k)
        b = first + np.arange(tot)
        pa, pb = order[a], order[b]
        d2 = np.sum((pts[pa] - pts[pb]) ** 2, axis=1)
        keep = d2 < r2
        pa, pb, d = pa[keep], pb[keep], np.sqrt(d2[keep])
        lo, hi = np.minimum(pa, pb), np.maximum(pa, pb)
        us.append(lo)
        vs.append(hi)
        ds.append(d)
    if not us:
        z = np.zeros(0, dtype=np.int64)
        return z, z, np.zeros(0)
    return np.concatenate(us), np.concatenate(vs), np.concatenate(ds)


def rgg(n: int, mean_degree: float = 24.0, *, ground_frac=0.005, excess=("uniform", 0.1, 10.0),
        w_clip=(1.0, 1e3), seed=0, tol=0.1, return_info=False):
    """Random geometric graph resistor network: n points uniform in [0,1]^3, an edge
    between points closer than r with conductance clip(1/dist, w_clip).  r starts at
    the value whose expected mean degree (boundary effects included) is mean_degree
    and is bisected on the realised mean degree until it is within tol.
    round(ground_frac*n) (>= 1) nodes are grounded with excess drawn from `excess`;
    then every connected component without a grounded node gets one (its smallest
    node id, excess from the same distribution); their count is reported in info."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    target = float(mean_degree)

    def expected_r():
        lo, hi = 0.0, 1.0
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            if (n - 1) * rgg_connect_probability(mid) < target:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    r = expected_r()
    u, v, d = _rgg_pairs(pts, r)
    deg = 2.0 * u.size / n
    if abs(deg - target) > tol:
        lo, hi = (r, 2.0 * r) if deg < target else (0.5 * r, r)
        for _ in range(60):
            r = 0.5 * (lo + hi)
            u, v, d = _rgg_pairs(pts, r)
            deg = 2.0 * u.size / n
            if abs(deg - target) <= tol:
                break
            if deg < target:
                lo = r
            else:
                hi = r
    order = np.lexsort((v, u))
    u, v, d = u[order], v[order], d[order]
    g = np.clip(1.0 / d, w_clip[0], w_clip[1])
    exc = _ground(rng, n, ground_frac, 1, excess)
    ncomp, label = connected_components(
        coo_matrix((np.ones(u.size), (u, v)), shape=(n, n)), directed=False)
    grounded_comp = np.zeros(ncomp, dtype=bool)
    grounded_comp[label[exc > 0]] = True
    first = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(first, label, np.arange(n))
    add = first[~grounded_comp]
    if add.size:
        exc[add] = _draw(rng, excess, add.size)
    A = assemble(n, u, v, g, exc)
    if return_info:
        return A, {"radius": r, "mean_degree": deg, "components": int(ncomp),
                   "grounds_added": int(add.size)}
    return A


def config_rgg(n: int = 2_000_000, seed: int = 0, return_info=False):
    """3D random geometric graph, n = 2,000,000 points, mean degree 24,
    w = clip(1/dist, 1, 1e3), 0.5% grounded with excess ~ U[0.1, 10]."""
    return rgg(n, 24.0, ground_frac=0.005, excess=("uniform", 0.1, 10.0), w_clip=(1.0, 1e3),
               seed=seed, return_info=return_info)


def pruned_grid(n_target: int, *, drop_frac=0.10, g=("uniform", 0.1, 10.0), ground_frac=0.02,
                excess=("uniform", 0.1, 10.0), seed=0) -> CSR:
    """2D grid of about n_target nodes (nx = round(sqrt(n)), ny = round(n / nx)) with
    round(drop_frac * edges) edges removed uniformly among those outside a random
    spanning tree (minimum spanning tree of i.i.d. uniform edge keys), so the graph
    stays connected; conductances, grounded nodes and excess drawn as in `grid`."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree

    rng = np.random.default_rng(seed)
    nx = max(1, int(round(np.sqrt(n_target))))
    ny = max(1, int(round(n_target / nx)))
    n = nx * ny
    eu, ev = grid_edges((nx, ny))
    key = rng.random(eu.size) + 1.0  # positive keys: every edge is stored
    T = minimum_spanning_tree(coo_matrix((key, (eu, ev)), shape=(n, n))).tocoo()
    tree = np.minimum(T.row, T.col).astype(np.int64) * n + np.maximum(T.row, T.col)
    in_tree = np.isin(eu * n + ev, tree)
    cand = np.flatnonzero(~in_tree)
    n_drop = min(int(round(drop_frac * eu.size)), cand.size)
    drop = rng.choice(cand, size=n_drop, replace=False)
    keep = np.ones(eu.size, dtype=bool)
    keep[drop] = False
    eu, ev = eu[keep], ev[keep]
    gv = _draw(rng, g, eu.size)
    exc = _ground(rng, n, ground_frac, 1, excess)
    return assemble(n, eu, ev, gv, exc)


def config_batch(count: int = 256, lo: float = 1e3, hi: float = 2e5, seed: int = 0):
    """`count` pruned grids with sizes log-uniform on [lo, hi] (matrix i from seed
    seed + i; the sizes from seed)."""
    rng = np.random.default_rng([seed, 0xBA7C])
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), count))
    return [pruned_grid(int(round(s)), seed=seed + i) for i, s in enumerate(sizes)]
