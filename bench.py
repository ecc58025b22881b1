#!/usr/bin/env python3
"""Benchmark of the hybrid solver on one MI355X.

One step = the whole hot path on one synthetic input already resident in HBM:
srw_build_factor (validation, random ordering, transition table, walks, tallies,
factor, transpose, level schedules) followed by srw_pcg_solve to the target
relative residual, then srw_factor_free.

Default workload: 3D 7-point resistor grid 128^3 (n = 2,097,152), conductances
log-uniform on [1e-2, 1e2], 1% of nodes grounded with excess U[0.01, 1]; 256 walks
per row, drop tolerance 1e-4, FP64 factor, one right-hand side N(0, 1), PCG to
||b - Ax|| <= 1e-8 ||b||; seed 0.

Prints one JSON line (rank 0).  `roofline` is for the walk kernel, the dominant
kernel: algorithmic bytes = 12 B per step + 8 B per entry of the row the step
leaves (counted exactly by the kernel) over the kernel's HIP-event duration on the
build stream.  `cpu_baseline` times the CPU oracle on the whole workload (build and
solve), its rows' walks and tallies split over the host threads.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "build+PCG seconds to rel. residual 1e-8 vs plain GPU method; walk steps/sec"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (generator, generator args, walks_per_row, drop_tol, tol); right-hand side
    # N(0, 1) unless listed in ONES_RHS
    "grid3d_128": ("config_grid3d", dict(m=128), 256, 1e-4, 1e-8),
    "grid3d_64": ("config_grid3d", dict(m=64), 256, 1e-4, 1e-8),
    "grid2d_32": ("config_grid2d_32", dict(), 64, 1e-3, 1e-8),
    # 3D random geometric graph, n = 2,000,000, mean degree 24 (generation ~1 min on a host core)
    "rgg_2m": ("config_rgg", dict(), 512, 1e-4, 1e-10),
}
# the 3D Dirichlet Laplacians of the paper's Table 1 (m1-m6), right-hand side all ones,
# tolerance 1e-6; 24 walks per row give the table's factor size
for _m in (50, 60, 70, 80, 90, 100):
    WORKLOADS[f"laplace3d_{_m}"] = ("laplace3d_dirichlet", dict(m=_m), 24, 0.0, 1e-6)
ONES_RHS = {k for k in WORKLOADS if k.startswith("laplace3d_")}
# asymmetric 3D grids (Section 7.1): two walk games, BiCGSTAB instead of PCG
for _m in (64, 128):
    WORKLOADS[f"grid3d_asym_{_m}"] = ("config_grid3d_asym", dict(m=_m), 256, 1e-4, 1e-8)
ASYM = {k for k in WORKLOADS if k.startswith("grid3d_asym_")}
# 256 independent pruned 2D grids, n log-uniform on [1e3, 2e5], 8 right-hand sides each:
# one batched build (one walk launch) and one batched PCG (graph-replayed iterations)
BATCH = {"batch_256": (256, 64, 1e-3, 1e-8, 8)}  # matrices, walks/row, drop, tol, nrhs
WORKLOADS.update({k: ("config_batch", dict(count=v[0]), v[1], v[2], v[3]) for k, v in BATCH.items()})


# workloads on which the walk kernel's unlocked refill periods (1, 2, 4) may be timed
SMALL_REFILL_OK = {"grid2d_32", "grid3d_64"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid3d_128", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=1)
    ap.add_argument("--solve-order", type=int, default=2,
                    help="0 rank order, 1 level order, 2 the library's automatic choice")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU baseline (the oracle on the whole workload)")
    ap.add_argument("--adaptive", type=float, default=0.0, metavar="DELTA",
                    help="walks per row by the Section 5.1 stopping rule with relative margin "
                         "DELTA at 99%% confidence (at least 20 walks), decided inside each "
                         "timed step, instead of the workload's uniform budget")
    ap.add_argument("--compare-precision", action="store_true",
                    help="after the timed steps, run one step with the other factor precision "
                         "(fp32 <-> fp64) and report it under ext_precision")
    ap.add_argument("--walks", type=int, default=0,
                    help="walks per row instead of the workload's (0 keeps the workload's)")
    ap.add_argument("--head-rows", type=int, default=0,
                    help="rows of the triangular solves' dense head (0 = the library default, "
                         "-1 = none)")
    ap.add_argument("--walk-waves", type=int, default=0,
                    help="waves per CU of the persistent walk kernel (0 = the library default)")
    ap.add_argument("--reuse", action="store_true",
                    help="walk reuse (Section 5.3): the walks extracted from every walk join "
                         "the tallies of their start rows")
    ap.add_argument("--ic0", action="store_true",
                    help="time IC(0)-PCG (natural ordering) against the random-walk factor on "
                         "the workload and report the paper's Table 1 figures (C, M1, I, M2, R1)")
    ap.add_argument("--rule", default="sqrt", choices=["equal", "sqrt", "neyman"],
                    help="learned_128: the budget rule the network learns (equal: every row "
                         "variance eps; sqrt: walks in proportion to the root of the per-walk "
                         "variance, the least summed variance per walk; neyman: least summed "
                         "variance per walk step)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the steps, copy a buffer of this many MiB three times with an "
                         "elementwise kernel (known traffic, for scaling hardware byte counters)")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Oracle threads: the host's CPU share for one GPU (16) at most."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(A, walks, drop, seed, tol, b, two_games=False, reuse=False):
    """The whole workload on the CPU oracle, as it stands: ordering and table on one
    thread, every row's walks and tallies split over the host threads, the factor and
    the solve (PCG, or BiCGSTAB for two games) on one thread.  Timed end to end."""
    import oracle as O

    threads = host_threads()
    t0 = time.perf_counter()
    if two_games:
        F = O.build_factor_ldu(A, walks, drop, seed, reuse=reuse, threads=threads)
        steps = int(F.a.walks.length.sum()) + int(F.t.walks.length.sum())
    else:
        F = O.build_factor(A, walks, drop, seed, reuse=reuse, threads=threads)
        steps = int(F.tallies.steps.sum())
    t1 = time.perf_counter()
    if two_games:
        st, x, it, rel = O.bicgstab(A, F, b, tol)
    else:
        st, x, it, rel = O.pcg(A, F, b, tol)
    t2 = time.perf_counter()
    return {
        "value": round(t2 - t0, 3),
        "unit": "s (oracle build + " + ("BiCGSTAB" if two_games else "PCG") + " to the same tolerance)",
        "cores": threads,
        "kind": "oracle",
        "sample": f"the whole workload: all {A.n} rows, {walks} walks each "
                  + ("(games of A and A^T) " if two_games else "")
                  + f"on {threads} host threads (walks and tallies), factor and solve on one",
        "cpu_model": cpu_model(),
        "build_s": round(t1 - t0, 3),
        "solve_s": round(t2 - t1, 3),
        "iters": it,
        "rel_residual": rel,
        "converged": st == 0,
        "walk_steps_per_s": round(steps / max(t1 - t0, 1e-9), 1),
    }


def cpu_baseline_batch(mats, seeds, walks, drop, tol, Bh, off):
    """The batch on the CPU oracle, as it stands: every matrix's build, then every
    (matrix, right-hand side) PCG, matrices spread over the host threads (each C call
    releases the GIL).  Timed end to end."""
    import threading

    import oracle as O

    threads = host_threads()
    order = sorted(range(len(mats)), key=lambda i: -mats[i].n)  # largest first
    facs = [None] * len(mats)
    res = {}
    lock = threading.Lock()
    it = iter(order)

    def build_worker():
        while True:
            with lock:
                i = next(it, None)
            if i is None:
                return
            facs[i] = O.build_factor(mats[i], walks, drop, seeds[i])

    t0 = time.perf_counter()
    pool = [threading.Thread(target=build_worker) for _ in range(threads)]
    [t.start() for t in pool]
    [t.join() for t in pool]
    t1 = time.perf_counter()
    jobs = iter([(i, j) for i in order for j in range(Bh.shape[1])])

    def solve_worker():
        while True:
            with lock:
                job = next(jobs, None)
            if job is None:
                return
            i, j = job
            st, x, iters, rel = O.pcg(mats[i], facs[i], Bh[off[i]:off[i + 1], j], tol)
            res[job] = (st, iters, rel)

    pool = [threading.Thread(target=solve_worker) for _ in range(threads)]
    [t.start() for t in pool]
    [t.join() for t in pool]
    t2 = time.perf_counter()
    return {
        "value": round(t2 - t0, 3),
        "unit": "s (oracle builds + PCG of every system to the same tolerance)",
        "cores": threads,
        "kind": "oracle",
        "sample": f"the whole batch: {len(mats)} matrices ({off[-1]} rows), {walks} walks per row, "
                  f"{Bh.shape[1]} right-hand sides each; matrices and systems spread over "
                  f"{threads} host threads",
        "cpu_model": cpu_model(),
        "build_s": round(t1 - t0, 3),
        "solve_s": round(t2 - t1, 3),
        "max_iters": max(v[1] for v in res.values()),
        "converged": all(v[0] == 0 for v in res.values()),
    }


def run_batch(args):
    """Config: 256 pruned 2D grids, 8 right-hand sides each.  One step = batched build +
    batched PCG of all 2,048 systems to 1e-8 + free."""
    import numpy as np
    import torch

    from paper_math_0609672_amd import metrics, srw, workloads

    count, walks, drop, tol, nrhs = BATCH[args.workload]
    if args.walks > 0:
        walks = args.walks

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    mats = workloads.config_batch(count, seed=args.seed)
    log(f"workload {args.workload}: {count} matrices generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    Ms = [srw.Matrix.from_host(A, dev) for A in mats]
    seeds = [args.seed + i for i in range(count)]
    off = np.concatenate([[0], np.cumsum([A.n for A in mats])])
    N = int(off[-1])
    Bh = workloads.rhs(N, nrhs=nrhs, seed=args.seed)
    B = torch.as_tensor(Bh, device=dev)
    X = torch.empty_like(B)
    torch.cuda.synchronize()

    def step():
        t0 = time.perf_counter()
        F = srw.build_factor_batched(Ms, walks, drop, seeds, precision=args.precision, profile=True)
        t1 = time.perf_counter()
        st, _, it, rel = srw.pcg_solve_batched(F, B, tol, 1000, X=X)
        t2 = time.perf_counter()
        s = F.stats()
        F.free()
        return dict(build_s=t1 - t0, pcg_s=t2 - t1, iters=it, rel=rel, status=st, stats=s)

    for i in range(args.warmup):
        r = step()
        log(f"warmup {i}: build {r['build_s']:.3f} s, pcg {r['pcg_s']:.3f} s, iters <= {int(r['iters'].max())}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(step())
        log(f"step {i}: build {runs[-1]['build_s']:.3f} s, pcg {runs[-1]['pcg_s']:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    K = args.steps
    s0 = runs[-1]["stats"]
    walk_ms = sum(r["stats"]["phase_ms"]["walk"] for r in runs) / K
    walk_bytes = 12.0 * s0["walk_steps"] + 8.0 * s0["walk_deg_sum"]
    achieved = walk_bytes / (walk_ms * 1e-3) / 1e9
    E = int(sum(A.nnz for A in mats))
    C = metrics.factor_size(s0["nnz_y"], N)
    it = runs[-1]["iters"]
    out = {
        "metric": METRIC,
        "value": round(elapsed / K, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / K, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (fp32 factor)",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {count} pruned 2D grids (n log-uniform on [1e3, 2e5], "
                        f"10% of edges removed, g U[0.1, 10], 2% grounded), N={N}, nnz={E}, "
                        f"{nrhs} right-hand sides each, {walks} walks/row, drop {drop}, tol {tol}, "
                        f"seed {args.seed}",
            "global_batch": count * nrhs,
            "parallelism": "single GPU",
        },
        "walk_steps_per_s": round(s0["walk_steps"] / (walk_ms * 1e-3), 1),
        "walk_steps": s0["walk_steps"],
        "build_s": round(sum(r["build_s"] for r in runs) / K, 4),
        "pcg_s": round(sum(r["pcg_s"] for r in runs) / K, 4),
        "solver": "batched pcg (graph-replayed iterations)",
        "systems": int(it.size),
        "pcg_iters_max": int(it.max()),
        "pcg_iters_mean": round(float(it.mean()), 2),
        "rel_residual_max": float(runs[-1]["rel"].max()),
        "converged": all(r["status"] == srw.OK for r in runs),
        "factor_C": C,
        "C_over_N": round(C / N, 3),
        "phase_ms": {k: round(sum(r["stats"]["phase_ms"][k] for r in runs) / K, 3) for k in srw.PHASES},
        "roofline": {
            "kernel": "k_walk",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, args.precision, s0["walk_waves"]),
            "alg_bytes_per_launch": walk_bytes,
            "avg_launch_ms": round(walk_ms, 3),
        },
    }
    if out["roofline"]["traffic"]:
        hbm = out["roofline"]["traffic"] / (walk_ms * 1e-3) / 1e9
        out["roofline"]["hbm_measured_gbs"] = round(hbm, 1)
        out["roofline"]["hbm_measured_frac"] = round(hbm / HBM_PEAK_GBS, 4)
    if not args.no_cpu:
        log(f"cpu baseline (oracle, whole batch, {host_threads()} threads)")
        out["cpu_baseline"] = cpu_baseline_batch(mats, seeds, walks, drop, tol, Bh, off)
        log(f"cpu baseline: {out['cpu_baseline']['value']} s")
    print(json.dumps(out), flush=True)


def run_ic0(args):
    """The paper's Table 1 comparison on one workload: IC(0)-PCG (natural ordering, the
    ICCG of Section 6) against the random-walk factor, both timed end to end (build +
    PCG + free), with C, M1 = 2C + E + 4N (eq. m1), iterations and M2 = M1 * I for
    each, and R1 = M2(IC(0)) / M2(random walks) -- the ratio the paper reports against
    ICCG-ILU(0)."""
    import numpy as np
    import torch

    from paper_math_0609672_amd import metrics, srw, workloads

    gen, gkw, walks, drop, tol = WORKLOADS[args.workload]
    if args.walks > 0:
        walks = args.walks
    A = workloads.laplace3d_dirichlet(**gkw) if gen == "laplace3d_dirichlet" else \
        getattr(workloads, gen)(seed=args.seed, **gkw)
    b_host = np.ones(A.n) if args.workload in ONES_RHS else workloads.rhs(A.n, seed=args.seed)
    dev = torch.device("cuda:0")
    M = srw.Matrix.from_host(A, dev)
    b = torch.as_tensor(b_host, device=dev)
    x = torch.empty_like(b)
    E, N = A.nnz, A.n

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def timed(make):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = make()
        t1 = time.perf_counter()
        st, _, it, rel = srw.pcg_solve(M, F, b, tol, 10000, x=x)
        t2 = time.perf_counter()
        nnz_y = F.info()["nnz_y"]
        F.free()
        torch.cuda.synchronize()
        return dict(s=time.perf_counter() - t0, build_s=t1 - t0, pcg_s=t2 - t1, iters=it, rel=rel,
                    status=st, nnz_y=nnz_y)

    ic0 = lambda: srw.build_ic0(M)  # noqa: E731
    rw = lambda: srw.build_factor(M, walks, drop, args.seed)  # noqa: E731
    for _ in range(args.warmup):
        timed(ic0)
        timed(rw)
    runs_ic, runs_rw = [], []
    for i in range(args.steps):
        runs_ic.append(timed(ic0))
        runs_rw.append(timed(rw))
        log(f"step {i}: IC(0) {runs_ic[-1]['s']:.4f} s ({runs_ic[-1]['iters']} iterations), "
            f"random walks {runs_rw[-1]['s']:.4f} s ({runs_rw[-1]['iters']} iterations)")

    def summary(runs):
        C = metrics.factor_size(runs[-1]["nnz_y"], N)
        it = runs[-1]["iters"]
        return {"seconds": round(float(np.median([r["s"] for r in runs])), 5),
                "build_s": round(float(np.median([r["build_s"] for r in runs])), 5),
                "pcg_s": round(float(np.median([r["pcg_s"] for r in runs])), 5),
                "iters": it, "rel_residual": runs[-1]["rel"],
                "converged": all(r["status"] == srw.OK for r in runs),
                "C": C, "C_over_N": round(C / N, 3), "M1": metrics.m1(C, E, N),
                "M2": metrics.m2(C, E, N, it)}

    si, sr = summary(runs_ic), summary(runs_rw)
    pcg_bytes = metrics.pcg_iter_bytes(E, N, runs_ic[-1]["nnz_y"]) * si["iters"]
    out = {
        "metric": METRIC,
        "value": si["seconds"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * si["seconds"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload} with IC(0)-PCG (natural ordering) against the random-walk "
                        f"factor ({walks} walks/row, drop {drop}, seed {args.seed}): {gen}{gkw or ''}, "
                        f"n={N}, nnz={E}, tol {tol}"
                        + (", right-hand side all ones" if args.workload in ONES_RHS else ""),
            "global_batch": 1,
            "parallelism": "single GPU",
        },
        "ic0": si,
        "random_walks": sr,
        "R1": round(si["M2"] / sr["M2"], 4),
        "roofline": {
            "kernel": "IC(0)-PCG (whole solve: SpMV, two triangular solves, vector passes)",
            "bound": "hbm",
            "achieved": round(pcg_bytes / si["pcg_s"] / 1e9, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(pcg_bytes / si["pcg_s"] / 1e9 / HBM_PEAK_GBS, 5),
            "traffic": None,
            "alg_bytes_per_launch": pcg_bytes,
            "avg_launch_ms": round(1e3 * si["pcg_s"], 3),
        },
    }
    print(json.dumps(out), flush=True)


LEARNED = {"learned_128": (128, 64, 20, 256, 1e-4, 1e-8)}  # eval m, train m, train mats, uniform walks, drop, tol
WORKLOADS.update({k: ("config_grid3d", dict(m=v[0]), v[3], v[4], v[5]) for k, v in LEARNED.items()})


def run_learned(args):
    """Learned walk budgets against the plain method on the 3D grid family: the network
    is trained on pilot factors of 20 matrices at 64^3 (library kernels: features,
    labels, bf16 MFMA forward/backward, Adam), then serves budgets for the 128^3 matrix.
    eps (the per-row variance target) is bisected until the learned build's PCG takes at
    most the uniform-256 build's iterations; both are then timed end to end (features,
    network, budgets, build, PCG, free for the learned one).  The uniform budget is the
    fallback: the reported step is the learned pipeline only if it is faster at equal
    iterations, and the line says which ran."""
    import numpy as np
    import torch

    from paper_math_0609672_amd import budget as LB
    from paper_math_0609672_amd import metrics, srw, workloads

    m_eval, m_train, n_train, uni, drop, tol = LEARNED[args.workload]
    dev = torch.device("cuda:0")

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # training
    t0 = time.perf_counter()
    Xs, ys = [], []
    for seed in range(1, n_train + 1):
        At = workloads.config_grid3d(m_train, seed)
        X, y = LB.pilot_rows(srw.Matrix.from_host(At, dev), seed, uni, drop, rule=args.rule)
        Xs.append(X)
        ys.append(y)
    X, y = torch.cat(Xs), torch.cat(ys)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    model = LB.fit(X, y, epochs=4, batch=65536, lr=2e-3, seed=0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    var_y = float(y.var())
    loss = model.history[-1][1]
    log(f"training: {X.shape[0]} rows from {n_train} pilot factors in {t1 - t0:.1f} s, "
        f"fit {t2 - t1:.2f} s, loss {loss:.4f} (target variance {var_y:.4f})")
    del X, y, Xs, ys

    A = workloads.config_grid3d(m_eval, args.seed)
    M = srw.Matrix.from_host(A, dev)
    b = torch.as_tensor(workloads.rhs(A.n, seed=args.seed), device=dev)
    x = torch.empty_like(b)

    def run(eps=None):
        """One end-to-end step: uniform budgets (eps None) or learned ones."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        walks = None if eps is None else LB.budgets(model, M, args.seed, eps, lo=8, hi=8192)
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        F = srw.build_factor(M, uni, drop, args.seed, walks=walks, profile=True,
                             head_rows=args.head_rows)
        st, _, it, rel = srw.pcg_solve(M, F, b, tol, 10000, x=x)
        s = F.stats()
        F.free()
        torch.cuda.synchronize()
        return dict(s=time.perf_counter() - t0, budget_s=t_b - t0, iters=it, rel=rel, status=st,
                    stats=s)

    run()  # warm
    ref = run()
    log(f"uniform {uni}: {ref['iters']} iterations, {ref['s']:.3f} s, {ref['stats']['walk_steps']:.3e} steps")
    # bisection on log eps: the largest eps (fewest walks) whose iterations <= uniform's
    lo, hi = np.log(1e-4), np.log(1.0)
    best = None
    for _ in range(10):
        mid = 0.5 * (lo + hi)
        r = run(float(np.exp(mid)))
        ok = r["status"] == srw.OK and r["iters"] <= ref["iters"]
        log(f"eps {np.exp(mid):.3e}: {r['iters']} iterations, {r['s']:.3f} s, "
            f"{r['stats']['walk_steps']:.3e} steps{' (ok)' if ok else ''}")
        if ok:
            best = (float(np.exp(mid)), r)
            lo = mid
        else:
            hi = mid
    eps = best[0] if best else None
    # timed steps: both methods, alternating
    K = args.steps
    learned, uniform = [], []
    for i in range(args.warmup):
        run(eps)
        run()
    for i in range(K):
        if eps is not None:
            learned.append(run(eps))
        uniform.append(run())
    t_u = float(np.median([r["s"] for r in uniform]))
    t_l = float(np.median([r["s"] for r in learned])) if learned else float("inf")
    use_learned = t_l < t_u
    main = learned if use_learned else uniform
    s0 = main[-1]["stats"]
    walk_ms = sum(r["stats"]["phase_ms"]["walk"] for r in main) / K
    walk_bytes = 12.0 * s0["walk_steps"] + 8.0 * s0["walk_deg_sum"]
    achieved = walk_bytes / (walk_ms * 1e-3) / 1e9
    C = metrics.factor_size(s0["nnz_y"], A.n)
    out = {
        "metric": METRIC,
        "value": round(min(t_l, t_u), 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * min(t_l, t_u), 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (network bf16, fp32 accumulation)",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: network 8-64-64-1 trained on {n_train} matrices of the 3D grid "
                        f"family at {m_train}^3 ({args.rule} rule), evaluated at {m_eval}^3 (n={A.n}) "
                        f"against uniform {uni} walks/row at equal PCG iterations; drop {drop}, "
                        f"tol {tol}, seed {args.seed}",
            "global_batch": 1,
            "parallelism": "single GPU",
        },
        "ran": "learned budgets" if use_learned else "uniform budgets (fallback: the learned "
                                                       "budgets were not faster at equal iterations)",
        "learned_s": round(t_l, 4) if learned else None,
        "uniform_s": round(t_u, 4),
        "speedup_vs_plain": round(t_u / t_l, 4) if learned else None,
        "eps": eps,
        "pcg_iters_learned": learned[-1]["iters"] if learned else None,
        "pcg_iters_uniform": uniform[-1]["iters"],
        "rel_residual_learned": learned[-1]["rel"] if learned else None,
        "rel_residual_uniform": uniform[-1]["rel"],
        "walk_steps_learned": learned[-1]["stats"]["walk_steps"] if learned else None,
        "walk_steps_uniform": uniform[-1]["stats"]["walk_steps"],
        "factor_C": C,
        "budget_s_learned": round(float(np.median([r["budget_s"] for r in learned])), 4)
        if learned else None,
        "phase_ms_learned": {k: round(v, 2) for k, v in learned[-1]["stats"]["phase_ms"].items()}
        if learned else None,
        "phase_ms_uniform": {k: round(v, 2) for k, v in uniform[-1]["stats"]["phase_ms"].items()},
        "train": {"pilot_s": round(t1 - t0, 3),
                  "fit_s": round(t2 - t1, 3), "loss": loss, "target_var": var_y},
        "roofline": {
            "kernel": "k_walk",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "alg_bytes_per_launch": walk_bytes,
            "avg_launch_ms": round(walk_ms, 3),
        },
    }
    print(json.dumps(out), flush=True)


WALK_SOURCES = ("paper_math_0609672_amd/csrc/walk.hpp", "paper_math_0609672_amd/csrc/common.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_walk_traffic.json")


def walk_source_sha():
    import hashlib

    h = hashlib.sha256()
    for rel in WALK_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, precision, walk_waves):
    """HBM bytes per walk launch from the committed counter summaries (one record per
    workload), if one was taken on this workload with the walk kernel's current source
    and grid; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            records = json.load(f).get("records", [])
    except (OSError, ValueError, AttributeError):
        return None
    sha = walk_source_sha()
    for t in records:
        if (t.get("source_sha256") == sha and t.get("workload") == workload
                and t.get("precision") == precision and t.get("walk_waves_per_cu") == walk_waves):
            return t.get("traffic_bytes")
    return None


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the walk build and PCG of this library run on a "
              "single MI355X; it has no multi-GPU mode.", file=sys.stderr)
        sys.exit(2)

    if args.refill in (1, 2, 4) and args.workload not in SMALL_REFILL_OK:
        print(f"bench.py: refill periods below 8 run only on {sorted(SMALL_REFILL_OK)}: a "
              "full-size run with refill period 1 once printed nothing for 180 s and its "
              "cause is not established.", file=sys.stderr)
        sys.exit(2)
    if args.workload in BATCH:
        run_batch(args)
        return
    if args.workload in LEARNED:
        run_learned(args)
        return
    if args.ic0:
        run_ic0(args)
        return

    import numpy as np
    import torch

    from paper_math_0609672_amd import metrics, srw, workloads

    gen, gkw, walks, drop, tol = WORKLOADS[args.workload]
    if args.walks > 0:
        walks = args.walks
    if gen == "laplace3d_dirichlet":
        A = workloads.laplace3d_dirichlet(**gkw)
    else:
        A = getattr(workloads, gen)(seed=args.seed, **gkw)
    b_host = np.ones(A.n) if args.workload in ONES_RHS else workloads.rhs(A.n, seed=args.seed)
    dev = torch.device("cuda:0")
    M = srw.Matrix.from_host(A, dev)
    b = torch.as_tensor(b_host, device=dev)
    x = torch.empty_like(b)
    torch.cuda.synchronize()

    asym = args.workload in ASYM
    build = srw.build_factor_ldu if asym else srw.build_factor
    solve = srw.bicgstab_solve if asym else srw.pcg_solve
    head = {} if asym else {"head_rows": args.head_rows}  # two-game builds take no head

    def step():
        t0 = time.perf_counter()
        budgets = None
        if args.adaptive > 0:
            budgets = srw.adaptive_budgets(M, args.seed, args.adaptive, alpha=0.99)
        F = build(M, walks, drop, args.seed, precision=args.precision,
                  refill_period=args.refill, schedule=args.schedule,
                  solve_order=args.solve_order, profile=True, walks=budgets,
                  reuse=args.reuse, walk_waves=args.walk_waves, **head)
        t1 = time.perf_counter()
        st, _, it, rel = solve(M, F, b, tol, 10000, x=x)
        t2 = time.perf_counter()
        s = F.stats()
        s2 = F.transpose_game().stats() if asym else None
        F.free()
        return dict(build_s=t1 - t0, pcg_s=t2 - t1, iters=it, rel=rel, status=st, stats=s, tstats=s2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"workload {args.workload}: n={A.n} nnz={A.nnz}")
    for i in range(args.warmup):
        r = step()
        log(f"warmup {i}: build {r['build_s']:.3f} s, pcg {r['pcg_s']:.3f} s, iters {r['iters']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(step())
        log(f"step {i}: build {runs[-1]['build_s']:.3f} s, pcg {runs[-1]['pcg_s']:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    K = args.steps
    s0 = runs[-1]["stats"]
    F = build(M, walks, drop, args.seed, precision=args.precision,
              refill_period=args.refill, schedule=args.schedule,
              solve_order=args.solve_order, reuse=args.reuse, walk_waves=args.walk_waves, **head)
    depth = F.depth()  # reported only; outside the timed steps
    F.free()
    walk_ms = sum(r["stats"]["phase_ms"]["walk"] for r in runs) / K
    steps_per_build = s0["walk_steps"]
    walk_bytes = 12.0 * steps_per_build + 8.0 * s0["walk_deg_sum"]
    if args.reuse:  # plus one 16-byte record per counted walk
        walk_bytes += 16.0 * s0["tallied_walks"]
    t0s = runs[-1]["tstats"]
    if asym:  # one walk launch per game: the average over both
        walk_ms_t = sum(r["tstats"]["phase_ms"]["walk"] for r in runs) / K
        bytes_t = 12.0 * t0s["walk_steps"] + 8.0 * t0s["walk_deg_sum"]
        if args.reuse:
            bytes_t += 16.0 * t0s["tallied_walks"]
        achieved_pair = (walk_bytes + bytes_t) / ((walk_ms + walk_ms_t) * 1e-3) / 1e9
    achieved = walk_bytes / (walk_ms * 1e-3) / 1e9
    if asym:
        achieved = achieved_pair
        steps_per_build += t0s["walk_steps"]
        walk_bytes = (walk_bytes + bytes_t) / 2
        walk_ms = (walk_ms + walk_ms_t) / 2
    build_s = sum(r["build_s"] for r in runs) / K
    pcg_s = sum(r["pcg_s"] for r in runs) / K
    iters = runs[-1]["iters"]
    E, N = A.nnz, A.n
    C = metrics.factor_size(s0["nnz_y"], N)
    phases = {k: round(sum(r["stats"]["phase_ms"][k] for r in runs) / K, 3) for k in srw.PHASES}

    out = {
        "metric": METRIC,
        "value": round(elapsed / K, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / K, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 (fp32 factor)",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {gen}{gkw or ''}, n={N}, nnz={E}, "
                        + (f"Section 5.1 walks (delta {args.adaptive}, alpha 0.99)" if args.adaptive > 0
                           else f"{walks} walks/row")
                        + (", walk reuse (Section 5.3)" if args.reuse else "")
                        + (", two games (A, A^T; Section 7.1), BiCGSTAB" if asym else "")
                        + f", drop {drop}, tol {tol}, seed {args.seed}",
            "global_batch": 1,
            "parallelism": "single GPU",
        },
        "walk_steps_per_s": round(steps_per_build / (walk_ms * 1e-3 * (2 if asym else 1)), 1),
        "walk_steps": steps_per_build,
        "walks": s0["walks"],
        "tallied_walks": s0["tallied_walks"],
        "walk_waves_per_cu": s0["walk_waves"],
        "build_s": round(build_s, 4),
        "pcg_s": round(pcg_s, 4),
        "solver": "bicgstab" if asym else "pcg",
        "pcg_iters": iters,
        "rel_residual": runs[-1]["rel"],
        "converged": all(r["status"] == srw.OK for r in runs),
        "factor_C": C,
        "C_over_N": round(C / N, 3),
        "M1": metrics.m1(C, E, N),
        "M2": metrics.m1(C, E, N) * iters,
        "solve_depth": depth,
        "solve_head_rows": s0.get("head_rows", 0),
        "phase_ms": phases,
        "roofline": {
            "kernel": "k_walk_reuse" if args.reuse else "k_walk",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "alg_bytes_per_launch": walk_bytes,
            "avg_launch_ms": round(walk_ms, 3),
        },
    }
    if args.compare_precision:
        other = "fp32" if args.precision == "fp64" else "fp64"
        x_main = x.clone()
        F2 = build(M, walks, drop, args.seed, precision=other, refill_period=args.refill,
                   schedule=args.schedule, solve_order=args.solve_order, **head)
        F2.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F2 = build(M, walks, drop, args.seed, precision=other, refill_period=args.refill,
                   schedule=args.schedule, solve_order=args.solve_order, **head)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st2, x2, it2, rel2 = solve(M, F2, b, tol, 10000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        F2.free()
        x64, x32 = (x_main, x2) if args.precision == "fp64" else (x2, x_main)
        out["ext_precision"] = {
            "factor_precision": other,
            "seconds": round(t2 - t0, 4), "build_s": round(t1 - t0, 4), "pcg_s": round(t2 - t1, 4),
            "pcg_iters": it2, "rel_residual": rel2, "converged": st2 == srw.OK,
            "x_rel_diff_fp32_vs_fp64": float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)),
        }
        log(f"{other} factor: build {t1 - t0:.3f} s, pcg {t2 - t1:.3f} s, iters {it2}")
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # an elementwise kernel: reads and writes nel doubles
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.copy_calibration} MiB read + written by one kernel")
        del src, dst
    # counters were taken on the workload's own walk budget
    default_walks = not (args.reuse or args.walks or args.adaptive > 0 or asym)
    out["roofline"]["traffic"] = (measured_traffic(args.workload, args.precision, s0["walk_waves"])
                                  if default_walks else None)
    # `achieved` is effective bandwidth: the method's algorithmic bytes over the kernel
    # time.  The caches serve part of them; the measured HBM traffic (hardware counters,
    # copy-calibrated) over the same time is the achieved HBM bandwidth.
    out["roofline"]["achieved_is"] = "effective (algorithmic bytes / kernel time)"
    if out["roofline"]["traffic"]:
        hbm = out["roofline"]["traffic"] / (out["roofline"]["avg_launch_ms"] * 1e-3) / 1e9
        out["roofline"]["hbm_measured_gbs"] = round(hbm, 1)
        out["roofline"]["hbm_measured_frac"] = round(hbm / HBM_PEAK_GBS, 4)
    if not args.no_cpu and args.adaptive <= 0:
        log(f"cpu baseline (oracle, whole workload, {host_threads()} threads)")
        out["cpu_baseline"] = cpu_baseline(A, walks, drop, args.seed, tol, b_host, two_games=asym,
                                           reuse=args.reuse)
        log(f"cpu baseline: {out['cpu_baseline']['value']} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
