"""CPU oracle of the random-walk incomplete LDL^T preconditioner (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use this package; the product path never imports it.  It shares
no code with the GPU library: the arithmetic lives in ``srw_oracle.c`` (plain FP64 C,
one row and one walk at a time) and in ``dense.py`` (numpy closed forms used as pins).

``build_factor`` and ``pcg`` follow Algorithm 1 of the paper: random ordering
(Section 5.4), walks with rank homes and the exact one-step treatment (Sections 2.2.1
and 5.2), tallies (Section 3.1), factor entries by eqs. newy / newz / d, the optional
drop (Section 4), then PCG (Section 6).  With ``reuse=True`` the walks also feed the
walks Algorithm "reuse" extracts from them into the tallies (Section 5.3).
``build_factor_ldu``, ``apply_ldu`` and ``bicgstab`` are the asymmetric case of Section
7.1: the games of A and of A^T with one ordering give the LDU of rev(A), used as the
preconditioner of BiCGSTAB (Barrett et al., Templates).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srw_oracle.c")
_LIB = os.path.join(_HERE, "libsrw_oracle.so")

OK, NOT_CONVERGED, E_ARG, E_NOT_RMATRIX, E_SINGULAR, E_NOMEM = 0, 1, -1, -2, -3, -5


def build() -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-ffp-contract=off", _SRC, "-o", _LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        L.srwo_philox4x64_10.argtypes = [P, P, P]
        L.srwo_draw.argtypes = [u64, i64, i64, u64]
        L.srwo_draw.restype = ctypes.c_uint32
        L.srwo_rank.argtypes = [i64, u64, P]
        L.srwo_validate.argtypes = [i64, P, P, P]
        L.srwo_table.argtypes = [i64, P, P, P, P, P, P, P, P, P, P]
        L.srwo_walk_rows.argtypes = [i64, P, P, P, P, P, P, P, u64, i64, P, P, P, P, P, P]
        L.srwo_tally_rows.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.srwo_reuse_sequence.argtypes = [i64, P, P, i64, P, P, P, P]
        L.srwo_reuse_sequence.restype = i64
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.srwo_walk_rows_reuse.argtypes = [i64, P, P, P, P, P, P, P, u64, i64, P, P, PP, PP, PP, PP]
        L.srwo_walk_rows_reuse.restype = i64
        L.srwo_free.argtypes = [P]
        L.srwo_validate_asym.argtypes = [i64, P, P, P]
        L.srwo_apply_ldu.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P]
        L.srwo_bicgstab.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P, dbl, i32, P, P, P]
        L.srwo_factor.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, dbl, P, P, P, P]
        L.srwo_apply.argtypes = [i64, P, P, P, P, P, P, P, P]
        L.srwo_pcg.argtypes = [i64, P, P, P, P, P, P, P, P, P, dbl, i32, P, P, P]
        L.srwo_ic0.argtypes = [i64, P, P, P, P, P, P, P, P, P]
        L.srwo_walk_rows_plain.argtypes = [i64, P, P, P, P, P, u64, i64, P, P, P, P, P, P]
        L.srwo_factor_plain.argtypes = [i64, P, P, P, P, P, P, P, P, P, dbl, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------------------- RNG
def philox4x64_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint64)
    k = _c(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().srwo_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def draw(seed: int, k: int, w: int, t: int) -> int:
    return int(lib().srwo_draw(seed, k, w, t))


def rank(n: int, seed: int) -> np.ndarray:
    r = np.zeros(max(n, 1), np.int32)
    st = lib().srwo_rank(n, seed, _p(r))
    assert st == OK
    return r[:n]


def validate(A) -> int:
    return int(lib().srwo_validate(A.n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)),
                                   _p(_c(A.val, np.float64))))


# --------------------------------------------------------------------------- table
@dataclass
class Table:
    nbr: np.ndarray       # int32[nnz - n]
    thr: np.ndarray       # uint32[nnz - n]
    mthr: np.ndarray      # uint32[nnz - n]
    tau: np.ndarray       # float64[n]
    grounded: np.ndarray  # uint8[n]
    diag: np.ndarray      # float64[n]


def table(A, rk: np.ndarray) -> Table:
    m = max(A.nnz - A.n, 1)
    n1 = max(A.n, 1)
    t = Table(np.zeros(m, np.int32), np.zeros(m, np.uint32), np.zeros(m, np.uint32),
              np.zeros(n1), np.zeros(n1, np.uint8), np.zeros(n1))
    lib().srwo_table(A.n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)),
                     _p(_c(A.val, np.float64)), _p(_c(rk, np.int32)), _p(t.nbr), _p(t.thr),
                     _p(t.mthr), _p(t.tau), _p(t.grounded), _p(t.diag))
    return Table(t.nbr[: A.nnz - A.n], t.thr[: A.nnz - A.n], t.mthr[: A.nnz - A.n],
                 t.tau[: A.n], t.grounded[: A.n], t.diag[: A.n])


# --------------------------------------------------------------------------- walks
@dataclass
class Walks:
    rows: np.ndarray      # int64[r]   rows simulated (list order)
    budget: np.ndarray    # int32[r]   walks simulated per listed row (0 if tau = 0)
    rec_off: np.ndarray   # int64[r+1] record offsets
    end: np.ndarray       # int32      end node, -1 = ground
    visits: np.ndarray    # uint32     stays at the start node, start included
    length: np.ndarray    # uint32     steps


def _at(a: np.ndarray, i: int):
    """Pointer to element i of a contiguous array."""
    return ctypes.c_void_p(a.ctypes.data + i * a.itemsize)


def _over_rows(nrows: int, threads: int, fn, chunk: int = 1024) -> None:
    """Calls fn(a, b) for consecutive slices [a, b) of a row list.  With threads > 1 the
    slices are taken in order by that many host threads; ctypes releases the GIL for
    the duration of each C call, and every slice writes disjoint outputs, so the result
    is the one a single call over all rows gives."""
    if threads <= 1 or nrows <= chunk:
        fn(0, nrows)
        return
    import threading

    starts = iter(range(0, nrows, chunk))
    lock = threading.Lock()
    errors = []

    def work():
        while True:
            with lock:
                a = next(starts, None)
            if a is None or errors:
                return
            try:
                fn(a, min(a + chunk, nrows))
            except BaseException as e:  # noqa: BLE001 - re-raised in the caller
                errors.append(e)
                return

    pool = [threading.Thread(target=work) for _ in range(threads)]
    for t in pool:
        t.start()
    for t in pool:
        t.join()
    if errors:
        raise errors[0]


def walk_rows(A, rk, tb: Table, seed: int, rows, budget, threads: int = 1) -> Walks:
    """The walks of the listed rows (records in list order).  threads > 1 splits the
    list over host threads (same records)."""
    rows = _c(rows, np.int64)
    budget = np.broadcast_to(np.asarray(budget, np.int32), rows.shape).copy()
    budget[tb.tau[rows] <= 0.0] = 0
    rec_off = np.zeros(rows.size + 1, np.int64)
    np.cumsum(budget, out=rec_off[1:])
    tot = max(int(rec_off[-1]), 1)
    end = np.zeros(tot, np.int32)
    vis = np.zeros(tot, np.uint32)
    ln = np.zeros(tot, np.uint32)
    rowptr = _c(A.rowptr, np.int64)
    rkc = _c(rk, np.int32)

    def run(a, b):
        st = lib().srwo_walk_rows(A.n, _p(rowptr), _p(tb.nbr), _p(tb.thr), _p(tb.mthr),
                                  _p(tb.tau), _p(tb.grounded), _p(rkc), seed, b - a,
                                  _at(rows, a), _at(budget, a), _at(rec_off, a), _p(end),
                                  _p(vis), _p(ln))
        assert st == OK

    _over_rows(rows.size, threads, run)
    n = int(rec_off[-1])
    return Walks(rows, budget, rec_off, end[:n], vis[:n], ln[:n])


# ------------------------------------------------------------------ walk reuse
@dataclass
class Records:
    """Walks counted in the tallies when walks are reused (Section 5.3): start node
    (row), end node (-1 = ground), stays at the start (start included), steps."""
    row: np.ndarray       # int32
    end: np.ndarray       # int32
    visits: np.ndarray    # uint32
    length: np.ndarray    # uint32


def reuse_sequence(keys, nodes) -> Records:
    """Algorithm "reuse" of Section 5.3 on one legal sequence: position l = 1..len holds
    nodes[l-1] with ordering key keys[l-1] (ground: key -1, node -1).  Returns every
    walk the algorithm counts (the sequence itself included), in counting order."""
    k = _c(keys, np.int64)
    nd = _c(nodes, np.int32)
    cap = max(k.size, 1)
    out = [np.zeros(cap, np.int32), np.zeros(cap, np.int32), np.zeros(cap, np.uint32),
           np.zeros(cap, np.uint32)]
    m = lib().srwo_reuse_sequence(k.size, _p(k), _p(nd), cap, *(_p(a) for a in out))
    assert m >= 0, m
    return Records(*(a[:m] for a in out))


def walk_rows_reuse(A, rk, tb: Table, seed: int, rows, budget) -> Records:
    """The walks of `rows` (as walk_rows, same draws) with walk reuse: every simulated
    walk and every walk extracted from it, as records."""
    rows = _c(rows, np.int64)
    budget = np.broadcast_to(np.asarray(budget, np.int32), rows.shape).copy()
    ptrs = [ctypes.c_void_p() for _ in range(4)]
    m = lib().srwo_walk_rows_reuse(A.n, _p(_c(A.rowptr, np.int64)), _p(tb.nbr), _p(tb.thr),
                                   _p(tb.mthr), _p(tb.tau), _p(tb.grounded),
                                   _p(_c(rk, np.int32)), seed, rows.size, _p(rows), _p(budget),
                                   *(ctypes.byref(q) for q in ptrs))
    assert m >= 0, m
    out = []
    for q, dt in zip(ptrs, (np.int32, np.int32, np.uint32, np.uint32)):
        a = np.ctypeslib.as_array(ctypes.cast(q, ctypes.POINTER(np.ctypeslib.as_ctypes_type(dt))),
                                  shape=(max(m, 1),))
        out.append(a[:m].copy())
        lib().srwo_free(q)
    return Records(*out)


def records_to_walks(n: int, rec: Records) -> Walks:
    """Groups records by their start node (stable) into the per-row layout of Walks
    over all nodes, for `tally`."""
    order = np.argsort(rec.row, kind="stable")
    count = np.bincount(rec.row, minlength=n).astype(np.int32)[:n] if rec.row.size else \
        np.zeros(n, np.int32)
    rec_off = np.zeros(n + 1, np.int64)
    np.cumsum(count, out=rec_off[1:])
    return Walks(np.arange(n, dtype=np.int64), count, rec_off, rec.end[order].astype(np.int32),
                 rec.visits[order].astype(np.uint32), rec.length[order].astype(np.uint32))


@dataclass
class Tallies:
    walks: np.ndarray     # uint32[r] M'
    J: np.ndarray         # uint64[r] sum of visits
    G: np.ndarray         # uint32[r] walks ended at ground
    steps: np.ndarray     # uint64[r]
    visits_sq: np.ndarray  # uint64[r]
    hlen: np.ndarray      # int32[r]  distinct end nodes
    h_off: np.ndarray     # int64[r]  start of each row's H list (= record offset)
    h_end: np.ndarray     # int32     end node ids, ascending per row
    h_cnt: np.ndarray     # uint32    H'_{k,i}


def tally(wk: Walks, threads: int = 1) -> Tallies:
    """Per-row tallies of the walks (threads > 1 splits the rows over host threads)."""
    r = wk.rows.size
    count = wk.budget.astype(np.int32)
    rr = max(r, 1)
    tot = max(int(wk.rec_off[-1]), 1)
    t = Tallies(np.zeros(rr, np.uint32), np.zeros(rr, np.uint64), np.zeros(rr, np.uint32),
                np.zeros(rr, np.uint64), np.zeros(rr, np.uint64), np.zeros(rr, np.int32),
                wk.rec_off[:-1].copy(), np.zeros(tot, np.int32), np.zeros(tot, np.uint32))
    end = wk.end if wk.end.size else np.zeros(1, np.int32)
    vis = wk.visits if wk.visits.size else np.zeros(1, np.uint32)
    ln = wk.length if wk.length.size else np.zeros(1, np.uint32)
    rec_off = _c(wk.rec_off, np.int64)

    def run(a, b):
        st = lib().srwo_tally_rows(b - a, _at(count, a), _at(rec_off, a), _p(end), _p(vis),
                                   _p(ln), _at(t.walks, a), _at(t.J, a), _at(t.G, a),
                                   _at(t.steps, a), _at(t.visits_sq, a), _at(t.hlen, a),
                                   _p(t.h_end), _p(t.h_cnt))
        assert st == OK

    _over_rows(r, threads, run)
    return Tallies(t.walks[:r], t.J[:r], t.G[:r], t.steps[:r], t.visits_sq[:r], t.hlen[:r],
                   t.h_off[:r], t.h_end, t.h_cnt)


# -------------------------------------------------------------------------- factor
@dataclass
class Factor:
    n: int
    rank: np.ndarray      # int32[n]
    yptr: np.ndarray      # int64[n+1]  rows of Y (node order), strictly lower in rank
    ycol: np.ndarray      # int32
    yval: np.ndarray      # float64
    d: np.ndarray         # float64[n]
    table: Table | None = None
    walks: Walks | None = None
    tallies: Tallies | None = None

    @property
    def by_rank(self) -> np.ndarray:
        br = np.empty(self.n, np.int32)
        br[self.rank] = np.arange(self.n, dtype=np.int32)
        return br

    def dense_y(self) -> np.ndarray:
        Y = np.eye(self.n)
        for k in range(self.n):
            for q in range(self.yptr[k], self.yptr[k + 1]):
                Y[k, self.ycol[q]] = self.yval[q]
        return Y


def walk_stats(wk: Walks):
    """Per listed row: the sample variance of the stays at the start over the row's walks
    (NaN below two walks) and the mean walk length (NaN without walks), straight from
    the walk records."""
    var = np.full(wk.rows.size, np.nan)
    mean = np.full(wk.rows.size, np.nan)
    for r in range(wk.rows.size):
        s = slice(wk.rec_off[r], wk.rec_off[r + 1])
        v = wk.visits[s].astype(np.float64)
        if v.size >= 2:
            var[r] = np.var(v, ddof=1)
        if v.size >= 1:
            mean[r] = wk.length[s].astype(np.float64).mean()
    return var, mean


def assemble(A, rk, tb: Table, tl: Tallies, rows: np.ndarray, drop_tol: float) -> Factor:
    """Factor rows from tallies of the listed rows (all rows when rows = arange(n))."""
    n = A.n
    walks = np.zeros(max(n, 1), np.uint32)
    J = np.zeros(max(n, 1), np.uint64)
    hlen = np.zeros(max(n, 1), np.int32)
    h_off = np.zeros(max(n, 1), np.int64)
    walks[rows] = tl.walks
    J[rows] = tl.J
    hlen[rows] = tl.hlen
    h_off[rows] = tl.h_off
    yptr = np.zeros(n + 1, np.int64)
    args = [n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)), _p(_c(A.val, np.float64)),
            _p(_c(rk, np.int32)), _p(_c(tb.tau if n else np.zeros(1), np.float64)), _p(walks),
            _p(J), _p(h_off), _p(hlen), _p(tl.h_end), _p(tl.h_cnt), float(drop_tol), _p(yptr)]
    lib().srwo_factor(*args, None, None, None)
    nnz = int(yptr[-1])
    ycol = np.zeros(max(nnz, 1), np.int32)
    yval = np.zeros(max(nnz, 1))
    d = np.zeros(max(n, 1))
    lib().srwo_factor(*args, _p(ycol), _p(yval), _p(d))
    return Factor(n, np.asarray(rk, np.int32), yptr, ycol[:nnz], yval[:nnz], d[:n], tb)


def walk_rows_plain(A, rk, tb: Table, seed: int, rows, budget, threads: int = 1) -> Walks:
    """Walks of the plain estimator (eq. yzdetail, no one-step treatment): every listed
    row runs its budget, each walk stepping by the full game from its first step."""
    rows = _c(rows, np.int64)
    budget = np.broadcast_to(np.asarray(budget, np.int32), rows.shape).copy()
    rec_off = np.zeros(rows.size + 1, np.int64)
    np.cumsum(budget, out=rec_off[1:])
    tot = max(int(rec_off[-1]), 1)
    end = np.zeros(tot, np.int32)
    vis = np.zeros(tot, np.uint32)
    ln = np.zeros(tot, np.uint32)
    rowptr = _c(A.rowptr, np.int64)
    rkc = _c(rk, np.int32)

    def run(a, b):
        st = lib().srwo_walk_rows_plain(A.n, _p(rowptr), _p(tb.nbr), _p(tb.thr), _p(tb.grounded),
                                        _p(rkc), seed, b - a, _at(rows, a), _at(budget, a),
                                        _at(rec_off, a), _p(end), _p(vis), _p(ln))
        assert st == OK

    _over_rows(rows.size, threads, run)
    n = int(rec_off[-1])
    return Walks(rows, budget, rec_off, end[:n], vis[:n], ln[:n])


def assemble_plain(A, tl: Tallies, drop_tol: float, rk) -> Factor:
    """Factor of the plain estimator from tallies over all rows (eqs. yzdetail, d)."""
    n = A.n
    yptr = np.zeros(n + 1, np.int64)
    args = [n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)), _p(_c(A.val, np.float64)),
            _p(tl.walks), _p(tl.J), _p(tl.h_off), _p(tl.hlen), _p(tl.h_end), _p(tl.h_cnt),
            float(drop_tol), _p(yptr)]
    assert lib().srwo_factor_plain(*args, None, None, None) == OK
    nnz = int(yptr[-1])
    ycol = np.zeros(max(nnz, 1), np.int32)
    yval = np.zeros(max(nnz, 1))
    d = np.zeros(max(n, 1))
    assert lib().srwo_factor_plain(*args, _p(ycol), _p(yval), _p(d)) == OK
    return Factor(n, np.asarray(rk, np.int32), yptr, ycol[:nnz], yval[:nnz], d[:n])


def build_factor(A, walks_per_row, drop_tol: float, seed: int, rk=None,
                 reuse: bool = False, threads: int = 1, one_step_exact: bool = True) -> Factor:
    """The whole preconditioning phase of Algorithm 1 on the CPU (one_step_exact=False:
    the plain estimator of eqs. yzdetail and d, every step random).  `walks_per_row` is
    an int (uniform) or an int array over nodes (per-row budgets, each >= 1).  With
    reuse, every walk also contributes the walks Algorithm "reuse" extracts from it
    (Section 5.3) to the tallies of their start nodes.  threads > 1 runs the rows'
    walks and tallies on that many host threads (rows are independent); the factor is
    the same."""
    rk = rank(A.n, seed) if rk is None else np.asarray(rk, np.int32)
    tb = table(A, rk)
    rows = np.arange(A.n, dtype=np.int64)
    if not one_step_exact:  # the plain estimator of eqs. yzdetail and d
        assert not reuse
        wk = walk_rows_plain(A, rk, tb, seed, rows, walks_per_row, threads=threads)
        tl = tally(wk, threads=threads)
        F = assemble_plain(A, tl, drop_tol, rk)
        F.table, F.walks, F.tallies = tb, wk, tl
        return F
    if reuse:
        wk = records_to_walks(A.n, walk_rows_reuse(A, rk, tb, seed, rows, walks_per_row))
    else:
        wk = walk_rows(A, rk, tb, seed, rows, walks_per_row, threads=threads)
    tl = tally(wk, threads=threads)
    F = assemble(A, rk, tb, tl, rows, drop_tol)
    F.walks, F.tallies = wk, tl
    return F


def ic0(A, rk=None) -> Factor:
    """Zero fill-in incomplete Cholesky (the ICCG preconditioner of the paper's
    comparisons, Section 6, Tables 1-2) in the factor's form A ~ Y^T D Y, eliminating
    in decreasing rank (natural ordering when rk is None: rank = node id).  The
    result plugs into apply / pcg like a random-walk factor."""
    n = A.n
    rk = np.arange(n, dtype=np.int32) if rk is None else _c(rk, np.int32)
    by_rank = np.empty(max(n, 1), np.int32)
    by_rank[rk] = np.arange(n, dtype=np.int32)
    yptr = np.zeros(n + 1, np.int64)
    args = [n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)), _p(_c(A.val, np.float64)),
            _p(rk), _p(by_rank)]
    st = lib().srwo_ic0(*args, _p(yptr), None, None, None)
    assert st == OK
    nnz = int(yptr[-1])
    ycol = np.zeros(max(nnz, 1), np.int32)
    yval = np.zeros(max(nnz, 1))
    d = np.zeros(max(n, 1))
    st = lib().srwo_ic0(*args, _p(yptr), _p(ycol), _p(yval), _p(d))
    if st != OK:
        raise ValueError("IC(0) breakdown: a pivot is not positive")
    return Factor(n, rk, yptr, ycol[:nnz], yval[:nnz], d[:n])


def apply(F: Factor, r: np.ndarray) -> np.ndarray:
    z = np.zeros(max(F.n, 1))
    work = np.zeros(max(F.n, 1))
    rr = _c(r, np.float64)
    lib().srwo_apply(F.n, _p(F.yptr), _p(F.ycol if F.ycol.size else np.zeros(1, np.int32)),
                     _p(F.yval if F.yval.size else np.zeros(1)), _p(F.d), _p(F.by_rank),
                     _p(rr), _p(z), _p(work))
    return z[: F.n]


def pcg(A, F: Factor | None, b: np.ndarray, tol: float, max_iter: int = 10000):
    """Returns (status, x, iters, rel_res); F = None runs plain CG."""
    n = A.n
    x = np.zeros(max(n, 1))
    iters = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    bb = _c(b, np.float64)
    if F is None:
        y = (None, None, None, None, None)
    else:
        y = (_p(F.yptr), _p(F.ycol if F.ycol.size else np.zeros(1, np.int32)),
             _p(F.yval if F.yval.size else np.zeros(1)), _p(F.d), _p(F.by_rank))
    st = lib().srwo_pcg(n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)),
                        _p(_c(A.val, np.float64)), *y, _p(bb), float(tol), int(max_iter),
                        _p(x), ctypes.byref(iters), ctypes.byref(rel))
    return int(st), x[:n], int(iters.value), float(rel.value)


# ---------------------------------------------------------- Section 5.1 stopping rule
def length_criterion(S1: int, S2: int, M: int, delta: float, z: float) -> bool:
    """Section 5.1: the relative error of the mean walk length is below delta with
    confidence alpha, tested as delta * mean * sqrt(M) / sigma > z with z the standard
    normal quantile Q^{-1}((1 - alpha) / 2).  S1, S2: sums of the first M lengths and
    of their squares; sigma the sample standard deviation (a zero sigma passes)."""
    mean = float(S1) / M
    var = (float(S2) - M * mean * mean) / (M - 1)
    if not var > 0.0:
        return True
    return delta * mean * math.sqrt(M) / math.sqrt(var) > z


def adaptive_budgets(A, rk, tb: Table, seed: int, delta: float, z: float, min_walks: int = 20,
                     max_walks: int = 8192) -> np.ndarray:
    """Walks per row by the Section 5.1 rule: walks run from row k one after another
    (walk w keyed as always by (row, w, step)) until the first M >= min_walks whose
    lengths satisfy `length_criterion`, or max_walks.  Rows with tau = 0 run none.
    The lengths come from walk_rows, which reruns walks 0 .. target-1 with a doubling
    target, so the first satisfying prefix is found exactly."""
    out = np.zeros(A.n, np.int32)
    for k in range(A.n):
        if tb.tau[k] <= 0.0:
            continue
        target = min_walks
        while True:
            wk = walk_rows(A, rk, tb, seed, np.array([k]), target)
            L = wk.length.astype(np.int64)
            S1 = S2 = 0
            found = 0
            for M in range(1, target + 1):
                S1 += int(L[M - 1])
                S2 += int(L[M - 1]) ** 2
                if M >= min_walks and length_criterion(S1, S2, M, delta, z):
                    found = M
                    break
            if found:
                out[k] = found
                break
            if target >= max_walks:
                out[k] = max_walks
                break
            target = min(2 * target, max_walks)
    return out


# ------------------------------------------------------- asymmetric A (Section 7.1)
@dataclass
class Csr:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.col.size)


def transpose(A) -> Csr:
    """A^T in CSR with sorted columns (scipy's transpose)."""
    import scipy.sparse as sp

    T = sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).T.tocsr()
    T.sort_indices()
    return Csr(A.n, T.indptr.astype(np.int64), T.indices.astype(np.int32), T.data.astype(np.float64))


def validate_asym(A) -> int:
    return int(lib().srwo_validate_asym(A.n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)),
                                        _p(_c(A.val, np.float64))))


@dataclass
class LduFactor:
    """Preconditioner of an asymmetric A from two games with one ordering: `a` from the
    game of A (Y_A, D: eqs. y2 and d), `t` from the game of A^T (Y_T: eq. y3).  In rank
    order A ~ Y_T^T D Y_A, the reversed LDU of rev(A)."""
    a: Factor
    t: Factor

    @property
    def n(self) -> int:
        return self.a.n


def build_factor_ldu(A, walks_per_row, drop_tol: float, seed: int, rk=None,
                     reuse: bool = False, threads: int = 1) -> LduFactor:
    """Both games of Section 7.1 with the ordering of `seed` (or `rk`) and the same walk
    draws (so for a symmetric A the two factors coincide)."""
    rk = rank(A.n, seed) if rk is None else np.asarray(rk, np.int32)
    Fa = build_factor(A, walks_per_row, drop_tol, seed, rk=rk, reuse=reuse, threads=threads)
    Ft = build_factor(transpose(A), walks_per_row, drop_tol, seed, rk=rk, reuse=reuse,
                      threads=threads)
    return LduFactor(Fa, Ft)


def _ldu_ptrs(F: LduFactor):
    def nz(a, dt):
        return a if a.size else np.zeros(1, dt)
    return (_p(F.a.yptr), _p(nz(F.a.ycol, np.int32)), _p(nz(F.a.yval, np.float64)), _p(F.a.d),
            _p(F.t.yptr), _p(nz(F.t.ycol, np.int32)), _p(nz(F.t.yval, np.float64)),
            _p(F.a.by_rank))


def apply_ldu(F: LduFactor, r: np.ndarray) -> np.ndarray:
    z = np.zeros(max(F.n, 1))
    work = np.zeros(max(F.n, 1))
    lib().srwo_apply_ldu(F.n, *_ldu_ptrs(F), _p(_c(r, np.float64)), _p(z), _p(work))
    return z[: F.n]


def bicgstab(A, F: LduFactor | None, b: np.ndarray, tol: float, max_iter: int = 10000):
    """Preconditioned BiCGSTAB; returns (status, x, iters, rel_res); F = None runs it
    unpreconditioned."""
    n = A.n
    x = np.zeros(max(n, 1))
    iters = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    y = (None,) * 8 if F is None else _ldu_ptrs(F)
    st = lib().srwo_bicgstab(n, _p(_c(A.rowptr, np.int64)), _p(_c(A.col, np.int32)),
                             _p(_c(A.val, np.float64)), *y, _p(_c(b, np.float64)), float(tol),
                             int(max_iter), _p(x), ctypes.byref(iters), ctypes.byref(rel))
    return int(st), x[:n], int(iters.value), float(rel.value)
