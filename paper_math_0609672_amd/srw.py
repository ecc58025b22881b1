"""ctypes binding of libsrw.so (the C ABI of include/srw.h).

Argument marshalling only: every step of the method runs in the HIP library.  PyTorch
supplies device memory (tensors) and the current stream.  Importing this module
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrw.so")

OK, NOT_CONVERGED = 0, 1
E_ARG, E_NOT_RMATRIX, E_SINGULAR, E_WALK_LIMIT, E_NOMEM, E_HIP = -1, -2, -3, -4, -5, -6
ORDER_RANDOM, ORDER_GIVEN, ORDER_NATURAL = 0, 1, 2
FP64, FP32 = 0, 1


class SrwError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        self.detail = detail
        msg = f"{what}: {status_string(status)} ({status})"
        super().__init__(msg + (f" [{detail}]" if detail else ""))


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("ordering", ctypes.c_int32), ("rank", ctypes.c_void_p), ("walks", ctypes.c_void_p),
                ("factor_precision", ctypes.c_int32), ("max_steps", ctypes.c_uint64),
                ("keep", ctypes.c_int32), ("refill_period", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("solve_order", ctypes.c_int32), ("reuse", ctypes.c_int32),
                ("walk_waves", ctypes.c_int32), ("one_step_exact", ctypes.c_int32),
                ("head_rows", ctypes.c_int32)]


NUM_PHASES = 8
PHASES = ("validate", "rank", "table", "schedule", "walk", "tally", "factor", "plan")


class _Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz_a", ctypes.c_int64), ("nnz_y", ctypes.c_int64),
                ("walks", ctypes.c_int64), ("walk_steps", ctypes.c_int64),
                ("walk_deg_sum", ctypes.c_int64), ("levels_fwd", ctypes.c_int32),
                ("levels_bwd", ctypes.c_int32), ("precision", ctypes.c_int32), ("keep", ctypes.c_int32),
                ("phase_ms", ctypes.c_double * NUM_PHASES), ("tallied_walks", ctypes.c_int64),
                ("reuse", ctypes.c_int32), ("two_game", ctypes.c_int32),
                ("walk_waves", ctypes.c_int32), ("head_rows", ctypes.c_int64),
                ("walk_lds", ctypes.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsrw.so is not built ({LIB_PATH}); run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)
_P, _I64, _I32, _U64, _D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
_lib.srw_default_options.argtypes = [ctypes.POINTER(_Options)]
_lib.srw_build_factor.argtypes = [ctypes.POINTER(_Csr), _I32, _D, _U64, ctypes.POINTER(_Options),
                                  ctypes.POINTER(_P), _P]
_lib.srw_factor_free.argtypes = [_P]
_lib.srw_build_ic0.argtypes = [ctypes.POINTER(_Csr), _U64, ctypes.POINTER(_Options), ctypes.POINTER(_P), _P]
_lib.srw_factor_info.argtypes = [_P] + [_P] * 8
_lib.srw_factor_stats.argtypes = [_P, ctypes.POINTER(_Stats)]
_lib.srw_factor_depth.argtypes = [_P, ctypes.POINTER(_I32), _P]
_lib.srw_factor_export.argtypes = [_P, _P, _P, _P, _P, _P, _P]
_lib.srw_table_export.argtypes = [_P, _P, _P, _P, _P, _P, _P]
_lib.srw_tally_export.argtypes = [_P] + [_P] * 9 + [_P]
_lib.srw_walk_export.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.srw_pcg_solve.argtypes = [ctypes.POINTER(_Csr), _P, _P, _D, _I32, _P, ctypes.POINTER(_I32),
                               ctypes.POINTER(_D), _P]
_lib.srw_apply.argtypes = [_P, _P, _P, _P]
_lib.srw_apply_noalloc.argtypes = [_P, _P, _P, _P]
_lib.srw_ordering.argtypes = [_I64, _U64, _P, _P]
_lib.srw_adaptive_budgets.argtypes = [ctypes.POINTER(_Csr), _U64, ctypes.POINTER(_Options), _D, _D,
                                      _I32, _I32, _P, _P]
_lib.srw_row_features.argtypes = [ctypes.POINTER(_Csr), _P, _P, _P]
_lib.srw_budget_labels.argtypes = [_P, _I32, _P, _P]
_lib.srw_walk_stats.argtypes = [_P, _P, _P, _P]
_lib.srw_mlp_forward.argtypes = [_P, _P, _P, _I64, _P, _P]
_lib.srw_mlp_train_step.argtypes = [_P, _P, _P, _I32, ctypes.c_float, _P, _P, _P, _I64, _P, _P, _P]
_lib.srw_mlp_train_step_rows.argtypes = [_P, _P, _P, _I32, ctypes.c_float, _P, _P, _P, _I64, _P,
                                         _I64, _P, _P, _P]
_lib.srw_budget_targets.argtypes = [_P, _P, _I64, _I32, _P, _P, ctypes.POINTER(_I64), _P]
_lib.srw_mlp_standardize.argtypes = [_P, _P, _I64, _P, _P, _P]
_lib.srw_mlp_budgets.argtypes = [_P, _I64, _D, _I32, _I32, _P, _P]
_lib.srw_build_factor_batched.argtypes = [_I32, _P, _I32, _D, _P, ctypes.POINTER(_Options),
                                          ctypes.POINTER(_P), _P]
_lib.srw_batch_info.argtypes = [_P, ctypes.POINTER(_I32), _P]
_lib.srw_pcg_solve_batched.argtypes = [_P, _I32, _P, _D, _I32, _P, _P, _P, _I32, _P]
_lib.srw_apply_batched.argtypes = [_P, _I32, _P, _P, _I32, _P]
_lib.srw_build_factor_ldu.argtypes = [ctypes.POINTER(_Csr), _I32, _D, _U64, ctypes.POINTER(_Options),
                                      ctypes.POINTER(_P), _P]
_lib.srw_factor_transpose_game.argtypes = [_P, ctypes.POINTER(_P)]
_lib.srw_bicgstab_solve.argtypes = [ctypes.POINTER(_Csr), _P, _P, _D, _I32, _P, ctypes.POINTER(_I32),
                                    ctypes.POINTER(_D), _P]
_lib.srw_last_error.argtypes = []
_lib.srw_last_error.restype = ctypes.c_char_p
_lib.srw_status_string.argtypes = [ctypes.c_int]
_lib.srw_status_string.restype = ctypes.c_char_p

EXPORTED = ["srw_default_options", "srw_build_factor", "srw_build_ic0", "srw_factor_free", "srw_factor_info",
            "srw_factor_stats", "srw_factor_depth",
            "srw_factor_export", "srw_table_export", "srw_tally_export", "srw_walk_export",
            "srw_pcg_solve", "srw_apply", "srw_apply_noalloc", "srw_walk_stats", "srw_adaptive_budgets", "srw_ordering", "srw_row_features", "srw_budget_labels",
            "srw_mlp_forward", "srw_mlp_train_step", "srw_mlp_train_step_rows", "srw_budget_targets",
            "srw_mlp_standardize", "srw_mlp_budgets", "srw_build_factor_batched",
            "srw_batch_info", "srw_pcg_solve_batched", "srw_apply_batched", "srw_last_error",
            "srw_status_string"]

NOALLOC_MAX_N = 1 << 21  # SRW_NOALLOC_MAX_N
MLP_PARAMS = 4801
NUM_FEATURES = 8


def status_string(status: int) -> str:
    return _lib.srw_status_string(int(status)).decode()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


@dataclass
class Matrix:
    """Device-resident CSR (int64 rowptr, int32 col, float64 val); see srw_csr."""

    n: int
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @classmethod
    def from_host(cls, A, device="cuda"):
        return cls(A.n, torch.as_tensor(A.rowptr, dtype=torch.int64).to(device),
                   torch.as_tensor(A.col, dtype=torch.int32).to(device),
                   torch.as_tensor(A.val, dtype=torch.float64).to(device))

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def c(self) -> _Csr:
        return _Csr(self.n, self.nnz, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val))


class Factor:
    """Handle of a library-owned srw_factor."""

    def __init__(self, handle: int, device, owner=None):
        self._h = ctypes.c_void_p(handle)
        self.device = device
        self._owner = owner  # a factor inside another handle is freed with it

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None) and self._h.value:
            if self._owner is None:
                _lib.srw_factor_free(self._h)
            self._h = ctypes.c_void_p(0)

    def transpose_game(self) -> "Factor":
        """srw_factor_transpose_game: the factor of the game of A^T of a two-game factor."""
        g = _P(0)
        _check(_lib.srw_factor_transpose_game(self._h, ctypes.byref(g)), "srw_factor_transpose_game")
        return Factor(g.value, self.device, owner=self)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n, nnz_y, walks, steps = (ctypes.c_int64() for _ in range(4))
        lf, lb, prec, keep = (ctypes.c_int32() for _ in range(4))
        st = _lib.srw_factor_info(self._h, *(ctypes.byref(v) for v in (n, nnz_y, walks, steps, lf, lb, prec, keep)))
        _check(st, "srw_factor_info")
        return dict(n=n.value, nnz_y=nnz_y.value, walks=walks.value, walk_steps=steps.value,
                    levels_fwd=lf.value, levels_bwd=lb.value,
                    precision="fp32" if prec.value == FP32 else "fp64", keep=keep.value)

    def stats(self) -> dict:
        st = _Stats()
        _check(_lib.srw_factor_stats(self._h, ctypes.byref(st)), "srw_factor_stats")
        d = {f: getattr(st, f) for f, _ in _Stats._fields_ if f != "phase_ms"}
        d["phase_ms"] = {name: st.phase_ms[i] for i, name in enumerate(PHASES)}
        return d

    def depth(self, stream=None) -> int:
        """srw_factor_depth: longest dependency chain of the triangular solves."""
        d = _I32(0)
        _check(_lib.srw_factor_depth(self._h, ctypes.byref(d), _stream(stream)), "srw_factor_depth")
        return d.value

    def export(self, stream=None) -> dict:
        i = self.info()
        n, m = i["n"], i["nnz_y"]
        vt = torch.float32 if i["precision"] == "fp32" else torch.float64
        kw = dict(device=self.device)
        out = dict(yptr=torch.empty(n + 1, dtype=torch.int64, **kw),
                   ycol=torch.empty(m, dtype=torch.int32, **kw),
                   yval=torch.empty(m, dtype=vt, **kw), d=torch.empty(n, dtype=vt, **kw),
                   rank=torch.empty(n, dtype=torch.int32, **kw))
        st = _lib.srw_factor_export(self._h, _ptr(out["yptr"]), _ptr(out["ycol"]), _ptr(out["yval"]),
                                    _ptr(out["d"]), _ptr(out["rank"]), _stream(stream))
        _check(st, "srw_factor_export")
        return out

    def table(self, nnz_a: int, stream=None) -> dict:
        n = self.info()["n"]
        m = nnz_a - n
        kw = dict(device=self.device)
        out = dict(nbr=torch.empty(m, dtype=torch.int32, **kw),
                   thr=torch.empty(m, dtype=torch.int32, **kw),
                   mthr=torch.empty(m, dtype=torch.int32, **kw),
                   tau=torch.empty(n, dtype=torch.float64, **kw),
                   grounded=torch.empty(n, dtype=torch.uint8, **kw))
        st = _lib.srw_table_export(self._h, _ptr(out["nbr"]), _ptr(out["thr"]), _ptr(out["mthr"]),
                                   _ptr(out["tau"]), _ptr(out["grounded"]), _stream(stream))
        _check(st, "srw_table_export")
        return out

    def tallies(self, stream=None) -> dict:
        n, W = self.info()["n"], self.stats()["tallied_walks"]
        kw = dict(device=self.device)
        out = dict(walks=torch.empty(n, dtype=torch.int32, **kw), J=torch.empty(n, dtype=torch.int64, **kw),
                   G=torch.empty(n, dtype=torch.int32, **kw), steps=torch.empty(n, dtype=torch.int64, **kw),
                   visits_sq=torch.empty(n, dtype=torch.int64, **kw),
                   h_off=torch.empty(n, dtype=torch.int64, **kw), hlen=torch.empty(n, dtype=torch.int32, **kw),
                   h_end=torch.empty(W, dtype=torch.int32, **kw), h_cnt=torch.empty(W, dtype=torch.int32, **kw))
        st = _lib.srw_tally_export(self._h, *(_ptr(out[k]) for k in
                                              ("walks", "J", "G", "steps", "visits_sq", "h_off", "hlen",
                                               "h_end", "h_cnt")), _stream(stream))
        _check(st, "srw_tally_export")
        return out

    def records(self, stream=None) -> dict:
        i = self.info()
        n, W = i["n"], i["walks"]
        kw = dict(device=self.device)
        out = dict(rec_off=torch.empty(n, dtype=torch.int64, **kw), end=torch.empty(W, dtype=torch.int32, **kw),
                   visits=torch.empty(W, dtype=torch.int32, **kw), length=torch.empty(W, dtype=torch.int32, **kw))
        st = _lib.srw_walk_export(self._h, _ptr(out["rec_off"]), _ptr(out["end"]), _ptr(out["visits"]),
                                  _ptr(out["length"]), _stream(stream))
        _check(st, "srw_walk_export")
        return out


def last_error() -> str:
    """srw_last_error: the calling thread's last recorded failure."""
    return _lib.srw_last_error().decode()


def _check(st: int, what: str):
    if st < 0:
        raise SrwError(st, what, last_error() if st in (-5, -6) else "")


def build_factor(A: Matrix, walks_per_row: int, drop_tol: float, seed: int, *, rank=None, walks=None,
                 precision: str = "fp64", max_steps: int = 0, keep: int = 0, refill_period: int = 0,
                 profile: bool = False, schedule: int = 1, solve_order: int = 2,
                 reuse: bool = False, walk_waves: int = 0, one_step_exact: bool = True,
                 head_rows: int = 0, stream=None) -> Factor:
    """srw_build_factor: the random-walk incomplete LDL^T factor of A (with reuse, the
    walks extracted by Algorithm "reuse" of Section 5.3 join the tallies; with
    one_step_exact=False, the plain estimator of eqs. yzdetail and d).  head_rows: the
    solves' dense head (0 automatic, -1 none)."""
    opt = _options(rank, walks, precision, max_steps, keep, refill_period, profile, schedule,
                   solve_order, reuse, walk_waves, one_step_exact, head_rows)
    h = ctypes.c_void_p(0)
    csr = A.c()
    st = _lib.srw_build_factor(ctypes.byref(csr), int(walks_per_row), float(drop_tol), int(seed) & (2**64 - 1),
                               ctypes.byref(opt), ctypes.byref(h), _stream(stream))
    _check(st, "srw_build_factor")
    return Factor(h.value, A.rowptr.device)


def build_ic0(A: Matrix, seed: int = 0, *, rank="natural", solve_order: int = 2,
              head_rows: int = 0, stream=None) -> Factor:
    """srw_build_ic0: zero fill-in incomplete Cholesky in the factor's form (the ICCG
    comparison of Section 6); natural ordering unless `rank` is a device tensor of
    ranks or None (the random ordering of `seed`)."""
    opt = _options(rank, None, "fp64", 0, 0, 0, False, 1, solve_order, False, head_rows=head_rows)
    h = ctypes.c_void_p(0)
    csr = A.c()
    st = _lib.srw_build_ic0(ctypes.byref(csr), int(seed) & (2**64 - 1), ctypes.byref(opt),
                            ctypes.byref(h), _stream(stream))
    _check(st, "srw_build_ic0")
    return Factor(h.value, A.rowptr.device)


def build_factor_ldu(A: Matrix, walks_per_row: int, drop_tol: float, seed: int, *, rank=None,
                     walks=None, precision: str = "fp64", max_steps: int = 0, keep: int = 0,
                     refill_period: int = 0, profile: bool = False, schedule: int = 1,
                     solve_order: int = 2, reuse: bool = False, walk_waves: int = 0,
                     stream=None) -> Factor:
    """srw_build_factor_ldu: the two-game preconditioner of an asymmetric A (Section 7.1)."""
    opt = _options(rank, walks, precision, max_steps, keep, refill_period, profile, schedule,
                   solve_order, reuse, walk_waves)
    h = ctypes.c_void_p(0)
    csr = A.c()
    st = _lib.srw_build_factor_ldu(ctypes.byref(csr), int(walks_per_row), float(drop_tol),
                                   int(seed) & (2**64 - 1), ctypes.byref(opt), ctypes.byref(h),
                                   _stream(stream))
    _check(st, "srw_build_factor_ldu")
    return Factor(h.value, A.rowptr.device)


def bicgstab_solve(A: Matrix, F, b: torch.Tensor, tol: float, max_iter: int = 10000, x=None,
                   stream=None):
    """srw_bicgstab_solve (F None: no preconditioner).  Returns (status, x, iters,
    rel_residual); errors raise SrwError."""
    if x is None:
        x = torch.empty_like(b)
    it = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    csr = A.c()
    st = _lib.srw_bicgstab_solve(ctypes.byref(csr), F.handle if F is not None else None, _ptr(b),
                                 float(tol), int(max_iter), _ptr(x), ctypes.byref(it),
                                 ctypes.byref(rel), _stream(stream))
    _check(st, "srw_bicgstab_solve")
    return st, x, it.value, rel.value


def _options(rank, walks, precision, max_steps, keep, refill_period, profile, schedule,
             solve_order, reuse, walk_waves=0, one_step_exact=True, head_rows=0) -> _Options:
    opt = _Options()
    _lib.srw_default_options(ctypes.byref(opt))
    if isinstance(rank, str):
        if rank != "natural":
            raise ValueError("rank: a device tensor of ranks, or 'natural'")
        opt.ordering = ORDER_NATURAL
    elif rank is not None:
        opt.ordering = ORDER_GIVEN
        opt.rank = _ptr(rank).value
    if walks is not None:
        opt.walks = _ptr(walks).value
    opt.factor_precision = FP32 if precision == "fp32" else FP64
    opt.max_steps = int(max_steps)
    opt.keep = int(keep)
    opt.refill_period = int(refill_period)
    opt.profile = 1 if profile else 0
    opt.schedule = int(schedule)
    opt.solve_order = int(solve_order)
    opt.reuse = 1 if reuse else 0
    opt.walk_waves = int(walk_waves)
    opt.one_step_exact = 1 if one_step_exact else 0
    opt.head_rows = int(head_rows)
    return opt


def pcg_solve(A: Matrix, F: Factor, b: torch.Tensor, tol: float, max_iter: int = 10000, x=None,
              stream=None):
    """srw_pcg_solve.  Returns (status, x, iters, rel_residual); status is OK or
    NOT_CONVERGED, errors raise SrwError."""
    if x is None:
        x = torch.empty_like(b)
    it = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    csr = A.c()
    st = _lib.srw_pcg_solve(ctypes.byref(csr), F.handle, _ptr(b), float(tol), int(max_iter), _ptr(x),
                            ctypes.byref(it), ctypes.byref(rel), _stream(stream))
    _check(st, "srw_pcg_solve")
    return st, x, it.value, rel.value


def apply(F: Factor, r: torch.Tensor, stream=None) -> torch.Tensor:
    """srw_apply: z = (Y^T D Y)^{-1} r."""
    z = torch.empty_like(r)
    st = _lib.srw_apply(F.handle, _ptr(r), _ptr(z), _stream(stream))
    _check(st, "srw_apply")
    return z


def apply_noalloc(F: Factor, r: torch.Tensor, z=None, stream=None) -> torch.Tensor:
    """srw_apply_noalloc: z = (Y^T D Y)^{-1} r with the library's static scratch (no
    device allocation by the library; z is allocated here unless given)."""
    if z is None:
        z = torch.empty_like(r)
    st = _lib.srw_apply_noalloc(F.handle, _ptr(r), _ptr(z), _stream(stream))
    _check(st, "srw_apply_noalloc")
    return z


def adaptive_budgets(A: Matrix, seed: int, delta: float, alpha: float = 0.99, min_walks: int = 20,
                     max_walks: int = 8192, rank=None, max_steps: int = 0,
                     stream=None) -> torch.Tensor:
    """srw_adaptive_budgets: walks per row by the Section 5.1 stopping rule (int32[n]),
    z = Q^{-1}((1 - alpha) / 2) from the standard normal distribution."""
    import statistics

    z = statistics.NormalDist().inv_cdf(1.0 - (1.0 - alpha) / 2.0)
    opt = _Options()
    _lib.srw_default_options(ctypes.byref(opt))
    if rank is not None:
        opt.ordering = ORDER_GIVEN
        opt.rank = _ptr(rank).value
    opt.max_steps = int(max_steps)
    walks = torch.empty(A.n, dtype=torch.int32, device=A.rowptr.device)
    csr = A.c()
    _check(_lib.srw_adaptive_budgets(ctypes.byref(csr), int(seed) & (2**64 - 1), ctypes.byref(opt),
                                     float(delta), float(z), int(min_walks), int(max_walks),
                                     _ptr(walks), _stream(stream)), "srw_adaptive_budgets")
    return walks


# ------------------------------------------------------------ learned walk budgets
def ordering(n: int, seed: int, device="cuda", stream=None) -> torch.Tensor:
    """srw_ordering: the random ordering's rank of every node (int32[n])."""
    rank = torch.empty(n, dtype=torch.int32, device=device)
    _check(_lib.srw_ordering(int(n), int(seed) & (2**64 - 1), _ptr(rank), _stream(stream)),
           "srw_ordering")
    return rank


def row_features(A: Matrix, rank: torch.Tensor, stream=None) -> torch.Tensor:
    """srw_row_features: float32 [n, 8] per-row features."""
    f = torch.empty((A.n, NUM_FEATURES), dtype=torch.float32, device=A.rowptr.device)
    csr = A.c()
    _check(_lib.srw_row_features(ctypes.byref(csr), _ptr(rank), _ptr(f), _stream(stream)),
           "srw_row_features")
    return f


def walk_stats(F: Factor, stream=None):
    """srw_walk_stats: (visit variance, mean walk length) per row, float64 device
    tensors (the factor must be built with keep >= 1)."""
    n = F.info()["n"]
    var = torch.empty(n, dtype=torch.float64, device=F.device)
    mean = torch.empty(n, dtype=torch.float64, device=F.device)
    _check(_lib.srw_walk_stats(F.handle, _ptr(var), _ptr(mean), _stream(stream)), "srw_walk_stats")
    return var, mean


def budget_labels(F: Factor, per_step: bool = False, stream=None) -> torch.Tensor:
    """srw_budget_labels: per-walk variance of each row (float64[n], NaN = no walks),
    divided by the mean walk length with per_step; F must have been built with
    keep >= 1."""
    n = F.info()["n"]
    out = torch.empty(n, dtype=torch.float64, device=F.device)
    _check(_lib.srw_budget_labels(F.handle, 1 if per_step else 0, _ptr(out), _stream(stream)),
           "srw_budget_labels")
    return out


def mlp_forward(params: torch.Tensor, mu_sd: torch.Tensor, features: torch.Tensor,
                stream=None) -> torch.Tensor:
    """srw_mlp_forward: predicted log label of every row (float32[n])."""
    n = features.shape[0]
    out = torch.empty(n, dtype=torch.float32, device=features.device)
    _check(_lib.srw_mlp_forward(_ptr(params), _ptr(mu_sd), _ptr(features), int(n), _ptr(out),
                                _stream(stream)), "srw_mlp_forward")
    return out


def mlp_train_step(params: torch.Tensor, mu_sd: torch.Tensor, features: torch.Tensor,
                   target: torch.Tensor, *, adam_m=None, adam_v=None, step: int = 1,
                   lr: float = 1e-3, grad=None, loss=None, stream=None) -> None:
    """srw_mlp_train_step: gradient of the mean squared error on these rows into
    `grad` / `loss` (if given) and, with adam_m / adam_v, one Adam update of params."""
    n = features.shape[0]
    _check(_lib.srw_mlp_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
                                   _ptr(mu_sd), _ptr(features), _ptr(target), int(n), _ptr(grad),
                                   _ptr(loss), _stream(stream)), "srw_mlp_train_step")


def mlp_train_step_rows(params: torch.Tensor, mu_sd: torch.Tensor, features: torch.Tensor,
                        target: torch.Tensor, rows: torch.Tensor, *, adam_m=None, adam_v=None,
                        step: int = 1, lr: float = 1e-3, grad=None, loss=None,
                        stream=None) -> None:
    """srw_mlp_train_step_rows: srw_mlp_train_step on the listed rows (int32) of
    features / target, gathered inside the kernel."""
    _check(_lib.srw_mlp_train_step_rows(_ptr(params), _ptr(adam_m), _ptr(adam_v), int(step),
                                        float(lr), _ptr(mu_sd), _ptr(features), _ptr(target),
                                        int(features.shape[0]), _ptr(rows), int(rows.shape[0]),
                                        _ptr(grad), _ptr(loss), _stream(stream)),
           "srw_mlp_train_step_rows")


def budget_targets(label: torch.Tensor, features: torch.Tensor, half: bool, stream=None):
    """srw_budget_targets: (features, targets) of the rows with a finite positive
    label, in row order; targets log(label), halved with half."""
    n = label.shape[0]
    x = torch.empty((n, NUM_FEATURES), dtype=torch.float32, device=label.device)
    y = torch.empty(n, dtype=torch.float32, device=label.device)
    cnt = _I64(0)
    _check(_lib.srw_budget_targets(_ptr(label), _ptr(features), int(n), 1 if half else 0,
                                   _ptr(x), _ptr(y), ctypes.byref(cnt), _stream(stream)),
           "srw_budget_targets")
    return x[:cnt.value], y[:cnt.value]


def mlp_standardize(features: torch.Tensor, target: torch.Tensor | None = None, stream=None):
    """srw_mlp_standardize: float32[16] per-feature mean, then sample standard
    deviation (at least 1e-6); with a target, also its mean (float32[1]):
    returns mu_sd, or (mu_sd, target_mean)."""
    dev = features.device
    mu_sd = torch.empty(2 * NUM_FEATURES, dtype=torch.float32, device=dev)
    tm = torch.empty(1, dtype=torch.float32, device=dev) if target is not None else None
    _check(_lib.srw_mlp_standardize(_ptr(features), _ptr(target), int(features.shape[0]),
                                    _ptr(mu_sd), _ptr(tm), _stream(stream)), "srw_mlp_standardize")
    return mu_sd if target is None else (mu_sd, tm)


def mlp_budgets(pred: torch.Tensor, eps: float, lo: int, hi: int, stream=None) -> torch.Tensor:
    """srw_mlp_budgets: walks per row = clamp(ceil(exp(pred) / eps), lo, hi)."""
    walks = torch.empty(pred.shape[0], dtype=torch.int32, device=pred.device)
    _check(_lib.srw_mlp_budgets(_ptr(pred), int(pred.shape[0]), float(eps), int(lo), int(hi),
                                _ptr(walks), _stream(stream)), "srw_mlp_budgets")
    return walks


# ---------------------------------------------------------------- batched solves
def build_factor_batched(mats, walks_per_row: int, drop_tol: float, seeds, *, walks=None,
                         precision: str = "fp64", keep: int = 0, profile: bool = False,
                         solve_order: int = 2, stream=None) -> Factor:
    """srw_build_factor_batched: one factor for a list of Matrix objects stacked
    block-diagonally (matrix i ordered and walked with seeds[i])."""
    import numpy as np

    arr = (_Csr * len(mats))(*[m.c() for m in mats])
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    opt = _Options()
    _lib.srw_default_options(ctypes.byref(opt))
    if walks is not None:
        opt.walks = _ptr(walks).value
    opt.factor_precision = FP32 if precision == "fp32" else FP64
    opt.keep = int(keep)
    opt.profile = 1 if profile else 0
    opt.solve_order = int(solve_order)
    h = ctypes.c_void_p(0)
    st = _lib.srw_build_factor_batched(len(mats), arr, int(walks_per_row), float(drop_tol),
                                       sd.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opt),
                                       ctypes.byref(h), _stream(stream))
    _check(st, "srw_build_factor_batched")
    return Factor(h.value, mats[0].rowptr.device)


def batch_info(F: Factor):
    """srw_batch_info: (nmat, row offsets as a list of nmat + 1 ints)."""
    import numpy as np

    nm = ctypes.c_int32(0)
    _check(_lib.srw_batch_info(F.handle, ctypes.byref(nm), None), "srw_batch_info")
    off = np.zeros(nm.value + 1, dtype=np.int64)
    _check(_lib.srw_batch_info(F.handle, ctypes.byref(nm), off.ctypes.data_as(ctypes.c_void_p)),
           "srw_batch_info")
    return nm.value, off.tolist()


def apply_batched(F: Factor, R: torch.Tensor, Z=None, schedule: int = 0, stream=None):
    """srw_apply_batched: Z = M^{-1} R for every system of a batched factor, R [N, nrhs]."""
    if R.dim() != 2 or R.dtype != torch.float64 or not R.is_contiguous():
        raise ValueError("R must be a contiguous float64 [N, nrhs] tensor")
    if Z is None:
        Z = torch.empty_like(R)
    elif Z.shape != R.shape or Z.dtype != torch.float64 or not Z.is_contiguous():
        raise ValueError("Z must be a contiguous float64 tensor shaped like R")
    st = _lib.srw_apply_batched(F.handle, int(R.shape[1]), _ptr(R), _ptr(Z), int(schedule),
                                _stream(stream))
    _check(st, "srw_apply_batched")
    return Z


def pcg_solve_batched(F: Factor, B: torch.Tensor, tol: float, max_iter: int = 10000, X=None,
                      use_graph: bool = True, stream=None):
    """srw_pcg_solve_batched over B [N, nrhs].  Returns (status, X, iters [nmat, nrhs],
    rel_residual [nmat, nrhs]) with numpy arrays for the host outputs."""
    import numpy as np

    nmat, _ = batch_info(F)
    nrhs = B.shape[1]
    if X is None:
        X = torch.empty_like(B)
    it = np.zeros(nmat * nrhs, dtype=np.int32)
    rel = np.zeros(nmat * nrhs, dtype=np.float64)
    st = _lib.srw_pcg_solve_batched(F.handle, int(nrhs), _ptr(B), float(tol), int(max_iter),
                                    _ptr(X), it.ctypes.data_as(ctypes.c_void_p),
                                    rel.ctypes.data_as(ctypes.c_void_p), 1 if use_graph else 0,
                                    _stream(stream))
    _check(st, "srw_pcg_solve_batched")
    return st, X, it.reshape(nmat, nrhs), rel.reshape(nmat, nrhs)
