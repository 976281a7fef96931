"""Benchmark: NNLS solves/s on one MI355X, mixed precision against the plain FP64 GPU path.

One step = one complete solve (validation, Gram matrix and A^T b, the whole pivot loop)
of a seeded synthetic instance whose inputs are already resident in device memory.
Default workload: sparse m = 400000, n = 50000, 20 N(0,1) entries per column at random
rows plus a block band (rows [8j, 8j+64) N(0,1), A[8j, j] += sqrt(84)), 25% of variables
active with margin 1e-3 (seed 1005), solved by the mixed path (float32 factor whose
updates run on bfloat16 MFMA, float64 refinement, float64 y_G and sign tests), by the
float32-factor mixed path and by the plain float64 path in the same process.

Prints one JSON line: the bfloat16-update path's solves/s and p50/p99 latency, the other
paths beside it, accuracy against the planted solution and between the paths, the
roofline of the dominant kernel (the tiled Cholesky, timed with HIP events on the solver's
stream during the timed steps), the 60000 x 12000 instance's legs, and the CPU oracle
timed on a bounded sample of the same workload.  Other workloads: --workload (see --help).
"""
from __future__ import annotations

import argparse
import contextlib
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix) peak
PEAK_FP32_TFLOPS = 157.3     # MI355X dense FP32 (matrix) peak
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 (matrix) peak
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E peak
CHOL_SOURCES = ("paper_cs_0408029_amd/csrc/k_chol.hip", "paper_cs_0408029_amd/csrc/tile_ops.h")
BATCH_SOURCES = ("paper_cs_0408029_amd/csrc/k_batched.hip", "paper_cs_0408029_amd/csrc/tile_ops.h")
# committed counter summaries (HBM bytes per launch of the factor) by (workload, precision)
TRAFFIC_SUMMARY = {("sparse_large", "fp64"): "profiles/k_chol_tiles_sparse_large_m60000_n12000.md",
                   ("sparse_xl", "fp32ir"): "profiles/k_chol_tiles_float_sparse_xl_m400000_n50000.md",
                   ("sparse_xl", "bf16ir"): "profiles/k_chol_tiles_bf16_sparse_xl_m400000_n50000.md",
                   ("dense_batch", "fp64"): "profiles/k_batched_dense_batch_4096.md"}
METRIC = "NNLS solves/s + p50/p99 latency vs plain FP64 GPU path at ≤1e-8 rel err"


@contextlib.contextmanager
def no_gc():
    """Timed regions run with Python's cyclic garbage collector paused (collected first):
    a full collection over this process's objects takes tens of ms and lands inside a
    step's wall-clock latency, not in the library."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def make_instance(name: str):
    import workloads as W
    if name == "sparse_large":
        return W.sparse_large(1002), ("sparse m=60000 n=12000, 25 N(0,1)/col + band(5,2.5,1.25), "
                                      "30% active, margin 1e-3, seed 1002")
    if name == "sparse_xl":
        return W.sparse_blockband(1005), ("sparse m=400000 n=50000, 20 N(0,1)/col + block band (rows "
                                          "[8j, 8j+64) N(0,1), A[8j,j] += sqrt(84)), 25% active, margin "
                                          "1e-3, seed 1005")
    if name == "sparse_small":
        return W.sparse_small(1001), ("sparse m=2000 n=400, Bernoulli(0.02) N(0,1) + diag, "
                                      "50% active, margin 0.1, seed 1001")
    raise SystemExit(f"unknown workload {name}")


def profiled_traffic(kernel_srcs, summary: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None when the
    kernel's sources have changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, summary)).read()
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in kernel_srcs)
    except OSError:
        return None
    fields = dict(l.strip().split(": ", 1) for l in text.splitlines() if ": " in l and l.startswith("    "))
    if fields.get("source_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    return float(fields["traffic_bytes_per_launch"])


CPU_THREADS = 0   # --cpu-threads: BLAS threads of the oracle timing (0: as the host sets them)


def cpu_baseline(inst, budget_s: float, max_solves: int = 5, what: str = "whole solve(s) of the benchmark instance"):
    """The oracle as it stands, on this host, over whole solves of the same instance until
    budget_s of CPU work has been spent (at least one solve, at most max_solves); with
    --cpu-threads K its BLAS runs on K threads (1: the serial baseline)."""
    import contextlib
    from oracle import bpp_solve
    limit = contextlib.nullcontext()
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        if CPU_THREADS > 0:
            limit = threadpool_limits(limits=CPU_THREADS)
            threads = CPU_THREADS
        else:
            threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    count = 0
    with limit:
        while True:
            res = bpp_solve(inst.A, inst.b)
            count += 1
            el = time.perf_counter() - t0
            if el >= budget_s or count >= max_solves:
                break
    return {"value": count / el, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{count} {what}, {el:.1f} s", "status": res.status,
            "free_set_match": bool(np.array_equal(res.free, inst.active))}


def bench_batch(args):
    """Batched dense workload: `--batch` problems (default 4096), n ~ U{16..256},
    m ~ U{2n..4n}, A = N(0,1)/sqrt(m), 40% active (seed 1003).  One step = one batched
    launch over all problems.  Beside it: the plain float64 path (one nnls_solve_dense call
    per problem) on the first --plain-sample problems."""
    import torch
    import paper_cs_0408029_amd as N
    import workloads as W
    t0 = time.perf_counter()
    insts = W.dense_batch(1003, count=args.batch)
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    As = [torch.from_numpy(np.ascontiguousarray(i.A.T)).to(dev).t() for i in insts]
    bs = [torch.from_numpy(i.b).to(dev) for i in insts]
    xs = [torch.empty(i.n, dtype=torch.float64, device=dev) for i in insts]
    ys = [torch.empty(i.n, dtype=torch.float64, device=dev) for i in insts]
    h = N.Handle(0)
    prec = N.NNLS_FP64 if args.precision == "fp64" else N.NNLS_FP32_IR
    gflag = N.NNLS_FLAG_GRAM_DUAL if args.gram_dual else 0
    opts = N.default_options(precision=prec, flags=gflag)
    popts = N.default_options(precision=prec, flags=N.NNLS_FLAG_PROFILE | gflag)

    packed = N.BatchedArgs(As, bs, xs, ys)   # descriptors marshalled once, outside the timing

    def step(o):
        st, infos = N.nnls_solve_dense_batched(h, opts=o, packed=packed)
        if st != N.NNLS_OK:
            raise RuntimeError(f"batched solve failed: {N.status_string(st)}")
        return infos

    for _ in range(args.warmup):
        step(opts)
    N.nnls_reset_profile(h)
    torch.cuda.synchronize()
    lat = []
    with no_gc():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            infos = step(popts)
            lat.append((time.perf_counter() - s0) * 1e3)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
    profs = N.nnls_get_profile(h)
    prof, gprof = profs["batched"], profs["batched_gram"]
    # accuracy against the planted solutions and the free sets
    errs, match = [], 0
    for inst, x in zip(insts, xs):
        xh = x.cpu().numpy()
        errs.append(float(np.linalg.norm(xh - inst.x_star) / np.linalg.norm(inst.x_star)))
        match += int(np.array_equal(xh > 0, inst.active))
    # the same batch prepared once and replayed from its captured graph
    pc0 = time.perf_counter()
    plan = N.BatchPlan(h, As, bs, xs, ys, opts)
    plan_s = time.perf_counter() - pc0
    shapes = plan.tile_shapes()
    for _ in range(args.warmup):
        plan.execute()
    glat = []
    with no_gc():
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            st, _ = plan.execute()
            glat.append((time.perf_counter() - s0) * 1e3)
            if st != N.NNLS_OK:
                raise RuntimeError(f"graph replay failed: {N.status_string(st)}")
        gtotal = time.perf_counter() - g0
    plan.close()
    # plain float64 path, one problem per call
    k = min(args.plain_sample, len(insts))
    o64 = N.default_options()
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for i in range(k):
        st, _ = N.nnls_solve_dense(h, As[i], bs[i], xs[i], ys[i], o64)
        if st != N.NNLS_OK:
            raise RuntimeError(f"plain solve failed: {N.status_string(st)}")
    torch.cuda.synchronize()
    plain = k / (time.perf_counter() - p0)
    h.close()
    gram_flops = sum(i.n * i.n * i.m for i in insts)
    gram_ms = gprof["ms"] / gprof["launches"] if gprof["launches"] else None
    piv_ms = prof["ms"] / prof["launches"] if prof["launches"] else None
    achieved = gram_flops / (gram_ms * 1e-3) / 1e12 if gram_ms else None
    peak = PEAK_FP64_TFLOPS if prec == N.NNLS_FP64 else PEAK_FP32_TFLOPS
    summary = TRAFFIC_SUMMARY.get(("dense_batch", args.precision))
    out = {
        "metric": METRIC,
        "value": round(args.steps * len(insts) / total, 2),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == N.NNLS_FP64 else "f32-factor+f64-refinement",
        "data": "synthetic",
        "config": {"workload": f"{len(insts)} dense problems, n~U{{16..256}}, m~U{{2n..4n}}, "
                               "N(0,1)/sqrt(m), 40% active, seed 1003",
                   "path": "batched, one launch" + (", y_G from the Gram matrix (Eq. 3)" if args.gram_dual else "")},
        "max_rel_err_vs_planted": max(errs), "free_set_matches": f"{match}/{len(insts)}",
        "graph_replay": {"solves_per_s": round(args.steps * len(insts) / gtotal, 2),
                         "ms_per_step": round(gtotal / args.steps * 1e3, 3),
                         "p50_ms": round(float(np.percentile(glat, 50)), 3),
                         "p99_ms": round(float(np.percentile(glat, 99)), 3),
                         "plan_create_s": round(plan_s, 3),
                         "autotuned_rects_per_wave": {f"n<={32 * k}": v for k, v in shapes.items()}},
        "plain_fp64_solves_per_s": round(plain, 2), "plain_sample": k,
        "roofline": {"bound": "mfma", "kernel": "k_batched_gram" + ("<double>" if prec == N.NNLS_FP64 else "<float>"),
                     "achieved": round(achieved, 4) if achieved else None,
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 5) if achieved else None,
                     "traffic": profiled_traffic(BATCH_SOURCES, summary) if summary else None,
                     "avg_launch_ms": round(gram_ms, 4) if gram_ms else None,
                     "work_per_launch": "sum over the batch of n^2 m flops (the lower half of each Gram "
                                        "matrix, 2 flops per product)"},
        "kernels_ms_per_launch": {"k_batched_gram": round(gram_ms, 4) if gram_ms else None,
                                  "k_batched (pivot loops)": round(piv_ms, 4) if piv_ms else None},
        "generation_s": round(gen_s, 1),
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        from oracle import bpp_solve
        try:
            from threadpoolctl import threadpool_info
            threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count() or 1
        c0 = time.perf_counter()
        cnt = 0
        while cnt < len(insts) and time.perf_counter() - c0 < args.cpu_budget:
            bpp_solve(insts[cnt].A, insts[cnt].b)
            cnt += 1
        el = time.perf_counter() - c0
        out["cpu_baseline"] = {"value": round(cnt / el, 2), "unit": "solves/s", "cores": int(threads),
                               "kind": "oracle", "sample": f"first {cnt} problems of the batch, {el:.1f} s"}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Serving workload: Poisson arrivals at --rate requests/s (seed 1004) of mixed sparse
    problems, n log-uniform in [64, 8192], m = 3n, 20 N(0,1) entries per column plus a band
    of sqrt(20) * (1, 1/2, 1/4), 30-60% active, margin 1e-3.  Requests cycle through a pool
    of --pool seeded problems.  --warmup-s seconds of arrivals are served before the
    statistics are reset; the next --duration seconds of arrivals are the timed window
    (latency: submit to x, y in host memory).  Beside it: a saturation run (the whole pool
    submitted at once) and the plain float64 path, one nnls_solve_csc call per problem."""
    import threading
    import torch
    import paper_cs_0408029_amd as N
    import workloads as W
    t0 = time.perf_counter()
    _, pool = W.serving_stream(1004, count=args.pool)
    gen_s = time.perf_counter() - t0
    arrs = [W.csc_arrays(p.A) + (np.ascontiguousarray(p.b),) for p in pool]
    prec = N.NNLS_FP64 if args.precision == "fp64" else N.NNLS_FP32_IR
    opts = N.default_options(precision=prec, max_workgroups=args.max_workgroups)
    srv = N.Server(0, opts=opts, workers=args.workers, batch_lanes=args.batch_lanes,
                   batch_max_n=args.batch_max_n, batch_step_iters=args.batch_step_iters)

    def submit(i):
        p = pool[i % len(pool)]
        cp, ri, va, b = arrs[i % len(pool)]
        st, tk = N.nnls_server_submit_csc(srv, p.m, p.n, cp, ri, va, b)
        if st != N.NNLS_OK:
            raise RuntimeError(f"submit failed: {N.status_string(st)}")
        return tk

    first = {}
    errors = []

    def collect(tickets, done_evt):
        for i, tk in tickets:
            p = pool[i % len(pool)]
            st, x, y, info = N.nnls_server_wait(srv, tk, p.n, timeout_ms=-1)
            if st != N.NNLS_OK:
                errors.append((i, N.status_string(st)))
            elif (i % len(pool)) not in first:
                first[i % len(pool)] = x
        done_evt.set()

    # open loop: submit at the arrival times
    def open_loop(rate, warm_s, dur_s, seed):
        rng = np.random.default_rng(seed)
        total_s = warm_s + dur_s
        gaps = rng.exponential(1.0 / rate, size=int(rate * total_s * 1.5) + 16)
        arrivals = np.cumsum(gaps)
        arrivals = arrivals[arrivals < total_s]
        n_warm = int(np.searchsorted(arrivals, warm_s))
        import queue as Q
        tq = Q.Queue()
        lag = []

        def collector():
            while True:
                item = tq.get()
                if item is None:
                    return
                i, tk = item
                p = pool[i % len(pool)]
                st, x, y, info = N.nnls_server_wait(srv, tk, p.n, timeout_ms=-1)
                if st != N.NNLS_OK:
                    errors.append((i, N.status_string(st)))
                elif (i % len(pool)) not in first:
                    first[i % len(pool)] = x

        col = threading.Thread(target=collector)
        col.start()
        start = time.perf_counter()
        timed_start = None
        for i, ta in enumerate(arrivals):
            if i == n_warm:
                # warm-up arrivals are all submitted; their completions still count until reset
                N.nnls_server_reset_stats(srv)
                timed_start = time.perf_counter()
            now = time.perf_counter() - start
            if ta > now:
                time.sleep(ta - now)
            lag.append(time.perf_counter() - start - ta)
            tq.put((i, submit(i)))
        tq.put(None)
        col.join()
        stats = N.nnls_server_stats(srv)
        wall = time.perf_counter() - (timed_start or start)
        return stats, wall, len(arrivals) - n_warm, n_warm, lag

    gc.collect()
    gc.disable()   # as in no_gc(): a collection pause would land in request latencies
    stats, wall, timed, n_warm, lag = open_loop(args.rate, args.warmup_s, args.duration, 1004)

    # saturation: the whole pool at once, twice
    N.nnls_server_reset_stats(srv)
    s0 = time.perf_counter()
    sat_tickets = [(i, submit(i)) for i in range(2 * len(pool))]
    ev = threading.Event()
    collect(sat_tickets, ev)
    sat_wall = time.perf_counter() - s0
    sat = N.nnls_server_stats(srv)
    sat_rate = 2 * len(pool) / sat_wall
    # when the offered rate exceeds what the engine completes, the queue grows without
    # bound and the latencies above measure the backlog: take them again at 80% of the
    # saturation rate, which the engine sustains
    sustained = None
    if stats["completed"] / wall < 0.95 * args.rate:
        N.nnls_server_reset_stats(srv)
        st2, wall2, timed2, _, _ = open_loop(0.8 * sat_rate, args.warmup_s, args.duration, 1005)
        sustained = {"offered_rate": round(0.8 * sat_rate, 1),
                     "solves_per_s": round(st2["completed"] / wall2, 2) if wall2 > 0 else None,
                     "p50_ms": round(st2["p50_ms"], 3), "p99_ms": round(st2["p99_ms"], 3),
                     "max_ms": round(st2["max_ms"], 3), "requests": timed2}
    gc.enable()
    srv.close()

    # plain float64 path: one problem per call on one stream
    dev = torch.device("cuda:0")
    h = N.Handle(0)
    o64 = N.default_options()
    plain_n = min(args.plain_sample, len(pool))
    dev_in = []
    for p, (cp, ri, va, b) in zip(pool[:plain_n], arrs[:plain_n]):
        dev_in.append(tuple(torch.from_numpy(a).to(dev) for a in (cp, ri, va, b)) +
                      (torch.empty(p.n, dtype=torch.float64, device=dev),
                       torch.empty(p.n, dtype=torch.float64, device=dev)))
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for p, (cp, ri, va, b, x, y) in zip(pool[:plain_n], dev_in):
        st, _ = N.nnls_solve_csc(h, p.m, p.n, cp, ri, va, b, x, y, o64)
        if st != N.NNLS_OK:
            raise RuntimeError(f"plain solve failed: {N.status_string(st)}")
    torch.cuda.synchronize()
    plain = plain_n / (time.perf_counter() - p0)
    h.close()

    errs, match = [], 0
    for k, x in first.items():
        p = pool[k]
        errs.append(float(np.linalg.norm(x - p.x_star) / np.linalg.norm(p.x_star)))
        match += int(np.array_equal(x > 0, p.active))
    ns = np.array([p.n for p in pool])
    out = {
        "metric": METRIC,
        "value": round(stats["completed"] / wall, 2) if wall > 0 else None,
        "unit": "solves/s",
        "n_gpus": 1, "steps": timed, "warmup": n_warm,
        "ms_per_step": round(stats["mean_ms"], 3),
        "p50_ms": round(stats["p50_ms"], 3), "p99_ms": round(stats["p99_ms"], 3),
        "max_ms": round(stats["max_ms"], 3),
        "offered_rate": args.rate, "completed_in_window": stats["completed"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == N.NNLS_FP64 else "f32-factor+f64-refinement",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson {args.rate:g} req/s for {args.duration:g} s after "
                               f"{args.warmup_s:g} s warm-up; sparse n log-uniform [64,8192], m=3n, "
                               f"20 N(0,1)/col + band, 30-60% active, margin 1e-3; pool of {len(pool)} "
                               "problems, seed 1004",
                   "workers": args.workers, "batch_lanes": args.batch_lanes,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "batch_max_n": args.batch_max_n, "batch_step_iters": args.batch_step_iters,
                   "max_workgroups": args.max_workgroups,
                   "pool_n_mean": float(ns.mean()), "pool_n_max": int(ns.max())},
        "saturation_solves_per_s": round(sat_rate, 2),
        "sustained": sustained,
        "saturation_p50_ms": round(sat["p50_ms"], 3), "saturation_p99_ms": round(sat["p99_ms"], 3),
        "max_running": max(stats["max_running"], sat["max_running"]),
        "batched_launches": stats["batches"] + sat["batches"],
        "peak_committed_gb": round(max(stats["peak_committed_bytes"], sat["peak_committed_bytes"]) / 1e9, 3),
        "plain_fp64_solves_per_s": round(plain, 2), "plain_sample": plain_n,
        "max_rel_err_vs_planted": max(errs) if errs else None,
        "free_set_matches": f"{match}/{len(first)}", "errors": errors[:5],
        "submit_lag_p99_ms": round(float(np.percentile(lag, 99)) * 1e3, 3) if lag else None,
        "generation_s": round(gen_s, 1),
        "roofline": None,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        from oracle import bpp_solve
        try:
            from threadpoolctl import threadpool_info
            threads = max([q.get("num_threads", 1) for q in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count() or 1
        c0 = time.perf_counter()
        cnt = 0
        while cnt < len(pool) and time.perf_counter() - c0 < args.cpu_budget:
            bpp_solve(pool[cnt].A, pool[cnt].b)
            cnt += 1
        el = time.perf_counter() - c0
        out["cpu_baseline"] = {"value": round(cnt / el, 2), "unit": "solves/s", "cores": int(threads),
                               "kind": "oracle",
                               "sample": f"first {cnt} problems of the pool, one after another, {el:.1f} s"}
    print(json.dumps(out), flush=True)


def bench_spmv(args):
    """Residual r = A x - b (row-major copy) and dual y = A^T r (CSC) on a sparse matrix much
    larger than the 256 MB last-level cache: m = --spmv-m rows, n = --spmv-n columns, --spmv-k
    distinct uniform-random rows per column, N(0,1) values (seed 1006).  A gathered vector
    longer than 2^19 doubles (x when n is, r when m is) is swept in 2 MB slices over a
    sliced copy of A (k_sliced_gather); the copies are built in each call, outside the
    timed kernels.  Kernel durations come from HIP events on the library's stream;
    bandwidth is algorithmic bytes (each array element read or written once) over that
    time."""
    import torch
    import paper_cs_0408029_amd as N
    if args.spmv_dense:
        return bench_spmv_dense(args)
    m, n, k = args.spmv_m, args.spmv_n, args.spmv_k
    rng = np.random.default_rng(1006)
    t0 = time.perf_counter()
    keys = np.repeat(np.arange(n, dtype=np.int64), k) * m + rng.integers(0, m, size=n * k, dtype=np.int64)
    keys = np.unique(keys)
    cols, rows = np.divmod(keys, m)
    del keys
    colptr = np.searchsorted(cols, np.arange(n + 1, dtype=np.int64)).astype(np.int32)
    rowidx = rows.astype(np.int32)
    del cols, rows
    nnz = int(rowidx.size)
    val = rng.standard_normal(nnz)
    x = rng.standard_normal(n)
    b = rng.standard_normal(m)
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (colptr, rowidx, val, x, b)]
    flags = torch.zeros(n, dtype=torch.uint8, device=dev)    # every column in G: y for all
    r = torch.empty(m, dtype=torch.float64, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    h = N.Handle(0)
    for _ in range(args.warmup):
        st = N.nnls_dual_csc(h, m, n, d[0], d[1], d[2], d[4], flags, d[3], r, y)
        if st != N.NNLS_OK:
            raise RuntimeError(f"dual step failed: {N.status_string(st)}")
    N.nnls_reset_profile(h)
    N.nnls_set_profiling(h, True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        N.nnls_dual_csc(h, m, n, d[0], d[1], d[2], d[4], flags, d[3], r, y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    N.nnls_set_profiling(h, False)
    prof = N.nnls_get_profile(h)
    # check a sample of rows and columns against float64 sums on the host
    import scipy.sparse as sp
    A = sp.csc_matrix((val, rowidx, colptr), shape=(m, n))
    rh, yh = r.cpu().numpy(), y.cpu().numpy()
    ridx = rng.integers(0, m, 256)
    cidx = rng.integers(0, n, 256)
    r_ref = A[ridx, :] @ x - b[ridx]
    y_ref = A[:, cidx].T @ rh
    err = max(float(np.max(np.abs(rh[ridx] - r_ref) / (1 + np.abs(r_ref)))),
              float(np.max(np.abs(yh[cidx] - y_ref) / (1 + np.abs(y_ref)))))
    h.close()
    res, dual = prof["residual"], prof["dual"]
    gbs = lambda c: c["work"] / (c["ms"] * 1e-3) / 1e9 if c["ms"] > 0 else None
    g_res, g_dual = gbs(res), gbs(dual)
    g_all = (res["work"] + dual["work"]) / ((res["ms"] + dual["ms"]) * 1e-3) / 1e9
    out = {
        "metric": "residual + dual SpMV effective bandwidth (algorithmic bytes / kernel time)",
        "value": round(g_all, 1), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round((res["ms"] + dual["ms"]) / max(res["launches"], 1), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"spmv m={m} n={n}, {k} uniform-random rows per column, N(0,1), seed 1006",
                   "nnz": nnz, "csc_mb": round(12 * nnz / 1e6, 1)},
        "residual_gbs": round(g_res, 1) if g_res else None, "residual_ms": round(res["ms"] / max(res["launches"], 1), 4),
        "dual_gbs": round(g_dual, 1) if g_dual else None, "dual_ms": round(dual["ms"] / max(dual["launches"], 1), 4),
        "wall_ms_per_call": round(wall / args.steps * 1e3, 3),
        "max_rel_err_sampled": err,
        "roofline": {"bound": "hbm",
                     "kernel": ("k_sliced_gather<, true>" if n > (1 << 19) else "k_residual_csr") + " + " +
                               ("k_sliced_gather<, false>" if m > (1 << 19) else "k_dual_csc"),
                     "achieved": round(g_all, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(g_all / PEAK_HBM_GBS, 4), "traffic": None},
        "generation_s": round(gen_s, 1),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_spmv_dense(args):
    """Dense residual r = A x - b and dual y = A^T r on a column-major m x n matrix
    (m = --dense-m, n = --dense-n, N(0,1), seed 1007), far larger than the last-level
    cache: A streams from HBM once per kernel."""
    import torch
    import paper_cs_0408029_amd as N
    m, n = args.dense_m, args.dense_n
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(1007)
    At = torch.randn(n, m, dtype=torch.float64, device=dev, generator=g)   # rows of At = columns of A
    A = At.t()
    x = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
    b = torch.randn(m, dtype=torch.float64, device=dev, generator=g)
    flags = torch.zeros(n, dtype=torch.uint8, device=dev)
    r = torch.empty(m, dtype=torch.float64, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    h = N.Handle(0)
    for _ in range(args.warmup):
        st = N.nnls_dual_dense(h, A, b, flags, x, r, y)
        if st != N.NNLS_OK:
            raise RuntimeError(f"dense dual step failed: {N.status_string(st)}")
    N.nnls_reset_profile(h)
    N.nnls_set_profiling(h, True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        N.nnls_dual_dense(h, A, b, flags, x, r, y)
    torch.cuda.synchronize()
    N.nnls_set_profiling(h, False)
    prof = N.nnls_get_profile(h)
    # sampled check against float64 products of the same device data on the host
    rng = np.random.default_rng(5)
    ri = rng.integers(0, m, 64)
    ci = rng.integers(0, n, 64)
    Ar = A[torch.from_numpy(ri).to(dev)].cpu().numpy()
    Ac = At[torch.from_numpy(ci).to(dev)].cpu().numpy()
    xh, bh, rh, yh = x.cpu().numpy(), b.cpu().numpy(), r.cpu().numpy(), y.cpu().numpy()
    err = max(float(np.max(np.abs(rh[ri] - (Ar @ xh - bh[ri])) / (1 + np.abs(Ar @ xh - bh[ri])))),
              float(np.max(np.abs(yh[ci] - Ac @ rh) / (1 + np.abs(Ac @ rh)))))
    h.close()
    res, dual = prof["residual"], prof["dual"]
    gbs = lambda c: c["work"] / (c["ms"] * 1e-3) / 1e9
    g_all = (res["work"] + dual["work"]) / ((res["ms"] + dual["ms"]) * 1e-3) / 1e9
    out = {
        "metric": "dense residual + dual effective bandwidth (algorithmic bytes / kernel time)",
        "value": round(g_all, 1), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round((res["ms"] + dual["ms"]) / max(res["launches"], 1), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"dense m={m} n={n} column-major, N(0,1), seed 1007", "a_gb": round(8 * m * n / 1e9, 2)},
        "residual_gbs": round(gbs(res), 1), "residual_ms": round(res["ms"] / max(res["launches"], 1), 4),
        "dual_gbs": round(gbs(dual), 1), "dual_ms": round(dual["ms"] / max(dual["launches"], 1), 4),
        "max_rel_err_sampled": err,
        "roofline": {"bound": "hbm", "kernel": "k_residual_dense + k_dual_dense", "achieved": round(g_all, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(g_all / PEAK_HBM_GBS, 4), "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_kappa(args):
    """Relative error against condition number, the analog of the paper's Fig. 1: 80 x 70
    matrices U diag(s) V^T with each singular value repeated 4 times and kappa from 1e1 to
    1e8 (half decades, --kappa-seeds problems each), known all-positive solution.  All
    problems of a precision go through one batched launch; beside them the CPU oracle on the
    same problems and the law fitted to the paper's printed points."""
    import torch
    import paper_cs_0408029_amd as N
    import workloads as W
    from oracle import bpp_solve
    d = np.loadtxt(os.path.join(ROOT, "tests", "golden", "fig1_normal_equations_error.txt"))
    slope, icpt = np.polyfit(1 + (d[:, 0] - 120) * 7 / 1319, -16 + (d[:, 1] - 82) * 18 / 778, 1)
    lks = np.arange(1.0, 8.01, 0.5)
    probs, keys = [], []
    for lk in lks:
        for s in range(args.kappa_seeds):
            probs.append(W.svd_conditioned(300 + s, 10 ** lk))
            keys.append(lk)
    dev = torch.device("cuda:0")
    As = [torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).t() for A, _, _ in probs]
    bs = [torch.from_numpy(b).to(dev) for _, _, b in probs]
    h = N.Handle(0)
    rows = {}
    t0 = time.perf_counter()
    for name, prec in (("gpu_fp64", N.NNLS_FP64), ("gpu_fp32ir", N.NNLS_FP32_IR)):
        xs = [torch.empty(A.shape[1], dtype=torch.float64, device=dev) for A, _, _ in probs]
        ys = [torch.empty_like(x) for x in xs]
        st, infos = N.nnls_solve_dense_batched(h, As, bs, xs, ys, N.default_options(precision=prec))
        for (A, xt, b), x, info, lk in zip(probs, xs, infos, keys):
            e = np.linalg.norm(x.cpu().numpy() - xt) / np.linalg.norm(xt) if info.status == N.NNLS_OK else np.nan
            rows.setdefault(lk, {}).setdefault(name, []).append(e)
    gpu_s = time.perf_counter() - t0
    # the final recomputation of Sec. 3 (float64 refinement of the final x_F), single-problem path
    oref = N.default_options(flags=N.NNLS_FLAG_REFINE_FINAL)
    for A_d, b_d, (A, xt, b), lk in zip(As, bs, probs, keys):
        x = torch.empty(A.shape[1], dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        st, info = N.nnls_solve_dense(h, A_d, b_d, x, y, oref)
        e = np.linalg.norm(x.cpu().numpy() - xt) / np.linalg.norm(xt) if st == N.NNLS_OK else np.nan
        rows[lk].setdefault("gpu_fp64_final_refine", []).append(e)
    h.close()
    for (A, xt, b), lk in zip(probs, keys):
        r = bpp_solve(A, b)
        e = np.linalg.norm(r.x - xt) / np.linalg.norm(xt) if r.status == "ok" else np.nan
        rows[lk].setdefault("oracle", []).append(e)
    table = []
    for lk in lks:
        row = {"log10_kappa": float(lk), "paper_law": round(float(slope * lk + icpt), 2)}
        for k, v in rows[lk].items():
            v = np.asarray(v)
            ok = v[np.isfinite(v)]
            row[k] = round(float(np.median(np.log10(ok))), 2) if ok.size else None
            row[k + "_failed"] = int(v.size - ok.size)
        table.append(row)
    fit = [(r["log10_kappa"], r["gpu_fp64"]) for r in table if r["gpu_fp64"] is not None and 1.5 <= r["log10_kappa"] <= 6]
    gslope = float(np.polyfit([a for a, _ in fit], [b for _, b in fit], 1)[0])
    out = {
        "metric": "relative error vs condition number (normal equations, Fig. 1 analog)",
        "value": round(gslope, 3), "unit": "log10 error per log10 kappa (GPU float64, kappa 1e1.5..1e6)",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(gpu_s * 1e3, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"80x70 U diag(s) V^T, singular values repeated 4 times, kappa 1e1..1e8, "
                               f"{args.kappa_seeds} problems per half decade, seeds 300+"},
        "paper_law_slope": round(float(slope), 3), "paper_law_intercept": round(float(icpt), 2),
        "paper_ne_plus_lsqr": {"4.0": round(float(np.log10(9.3e-12)), 2), "6.0": round(float(np.log10(3.1e-8)), 2),
                               "2.0": round(float(np.log10(4.7e-15)), 2)},
        "table": table, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_fig2(args):
    """The paper's speed workload (Fig. 2): random n x (n-10) matrices, N(0,1) values at a
    random density-1.0 or density-0.01 pattern, b ~ N(0,1) (seed 1008), at the paper's sizes;
    --fig2-reps matrices per point.  GPU time per solve on the plain float64 path (inputs
    resident, one call per problem) and the CPU oracle on the same matrices; the paper's
    tsnnls times (G5, serial C, final LSQR included) are context."""
    import scipy.sparse as sp
    import torch
    import paper_cs_0408029_amd as N
    from oracle import bpp_solve
    paper = {"dense": {120: 0.031, 200: 0.063, 300: 0.23, 499: 0.93, 699: 2.42, 938: 5.72},
             "sparse": {820: 0.12, 1000: 0.24, 1200: 0.47, 1420: 0.79}}
    rng = np.random.default_rng(1008)
    dev = torch.device("cuda:0")
    h = N.Handle(0)
    o = N.default_options()
    table = []
    for kind, pts in paper.items():
        for n_rows, t_paper in pts.items():
            m, n = n_rows, n_rows - 10
            gpu_t, cpu_t, stat, iters = [], [], [], []
            for rep in range(args.fig2_reps):
                if kind == "dense":
                    A = rng.standard_normal((m, n))
                else:
                    A = sp.random(m, n, density=0.01, format="csc", random_state=rng,
                                  data_rvs=rng.standard_normal)
                    A.sort_indices()
                b = rng.standard_normal(m)
                x = torch.empty(n, dtype=torch.float64, device=dev)
                y = torch.empty_like(x)
                bd = torch.from_numpy(b).to(dev)
                if kind == "dense":
                    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).to(dev).t()
                    call = lambda: N.nnls_solve_dense(h, Ad, bd, x, y, o)
                else:
                    cp = torch.from_numpy(A.indptr.astype(np.int32)).to(dev)
                    ri = torch.from_numpy(A.indices.astype(np.int32)).to(dev)
                    va = torch.from_numpy(A.data).to(dev)
                    call = lambda: N.nnls_solve_csc(h, m, n, cp, ri, va, bd, x, y, o)
                call()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = call()
                torch.cuda.synchronize()
                gpu_t.append(time.perf_counter() - t0)
                stat.append(N.status_string(st))
                iters.append(info.iterations)
                c0 = time.perf_counter()
                r = bpp_solve(A, b)
                cpu_t.append(time.perf_counter() - c0)
                if st == N.NNLS_OK and r.status == "ok":
                    xh = x.cpu().numpy()
                    if not np.array_equal(xh > 0, r.x > 0):
                        stat[-1] = "free-set mismatch"
            table.append({"kind": kind, "m": m, "n": n, "gpu_ms": round(1e3 * float(np.mean(gpu_t)), 3),
                          "oracle_ms": round(1e3 * float(np.mean(cpu_t)), 2),
                          "paper_tsnnls_ms": round(1e3 * t_paper, 1), "iterations": float(np.mean(iters)),
                          "status": sorted(set(stat))})
    h.close()
    ok = all(r["status"] == ["NNLS_OK"] for r in table)
    out = {
        "metric": "solve time on the paper's Fig. 2 matrices (plain float64 path, one call per problem)",
        "value": round(float(np.mean([r["paper_tsnnls_ms"] / r["gpu_ms"] for r in table])), 1),
        "unit": "mean speed-up over the paper's tsnnls times (other hardware: context only)",
        "n_gpus": 1, "steps": args.fig2_reps, "warmup": 1,
        "ms_per_step": round(float(np.mean([r["gpu_ms"] for r in table])), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "random n x (n-10), density 1.0 (n 120..938) and 0.01 (n 820..1420), "
                               f"N(0,1), {args.fig2_reps} matrices per point, seed 1008"},
        "all_ok_and_free_sets_match_oracle": ok, "table": table, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="metric",
                    help="metric (default): mixed vs plain FP64 on the 400000 x 50000 instance; or "
                         "sparse_large, sparse_xl, sparse_small, dense_batch, serve, spmv, kappa, fig2")
    ap.add_argument("--no-secondary", action="store_true",
                    help="metric: skip the 60000 x 12000 pair")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="BLAS threads of the oracle timing (0: the host's default; 1: serial)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32ir", "bf16ir"], default="fp64",
                    help="fp64: the plain FP64 path (the metric's reference); fp32ir: float32 factor "
                         "with float64 refinement")
    ap.add_argument("--batch", type=int, default=4096, help="dense_batch: number of problems")
    ap.add_argument("--gram-dual", action="store_true",
                    help="dense_batch: y_G = H_GF x_F - c_G (Eq. 3) instead of the residual form (Eq. 5)")
    ap.add_argument("--plain-sample", type=int, default=256,
                    help="dense_batch: problems solved one per call on the plain float64 path")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: offered requests/s")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: timed seconds of arrivals")
    ap.add_argument("--warmup-s", type=float, default=1.0, help="serve: warm-up seconds of arrivals")
    ap.add_argument("--pool", type=int, default=128, help="serve: distinct problems cycled")
    ap.add_argument("--workers", type=int, default=16, help="serve: concurrent sparse solves")
    ap.add_argument("--hw-queues", type=int, default=24,
                    help="serve: GPU_MAX_HW_QUEUES for this process (at least workers + batch lanes)")
    ap.add_argument("--batch-lanes", type=int, default=2, help="serve: batched launches in flight")
    ap.add_argument("--batch-max-n", type=int, default=256, help="serve: largest n sent to batched launches")
    ap.add_argument("--max-workgroups", type=int, default=0,
                    help="serve: workgroups of each sparse request's factor (0: the engine's default)")
    ap.add_argument("--batch-step-iters", type=int, default=1,
                    help="serve: pivot iterations per step of the batched lanes (< 0: whole solves per launch)")
    ap.add_argument("--fig2-reps", type=int, default=3, help="fig2: matrices per point")
    ap.add_argument("--kappa-seeds", type=int, default=8, help="kappa: problems per half decade")
    ap.add_argument("--spmv-dense", action="store_true", help="spmv: dense column-major A instead")
    ap.add_argument("--dense-m", type=int, default=65536, help="spmv --spmv-dense: rows")
    ap.add_argument("--dense-n", type=int, default=4096, help="spmv --spmv-dense: columns")
    ap.add_argument("--spmv-m", type=int, default=4_000_000, help="spmv: rows")
    ap.add_argument("--spmv-n", type=int, default=1_000_000, help="spmv: columns")
    ap.add_argument("--spmv-k", type=int, default=25, help="spmv: nonzeros per column")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    global CPU_THREADS
    CPU_THREADS = args.cpu_threads
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve":
        if not 1 <= args.hw_queues <= 32:
            ap.error("--hw-queues must be in [1, 32]")
        # a hardware queue for every stream of the serving engine (HIP's default is 4),
        # set before the runtime starts; it replaces a value from the environment
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    import torch
    import paper_cs_0408029_amd as N

    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_mib, "read_bytes": n * 8, "write_bytes": n * 8}))
        return

    if not os.path.exists(N.LIB_PATH):
        from paper_cs_0408029_amd.build import build
        build()
    if args.workload == "metric":
        bench_metric(args)
        return
    if args.workload == "dense_batch":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "spmv":
        bench_spmv(args)
        return
    if args.workload == "kappa":
        bench_kappa(args)
        return
    if args.workload == "fig2":
        bench_fig2(args)
        return
    inst, desc = make_instance(args.workload)
    dev = torch.device("cuda:0")
    arrays = device_arrays(inst, dev)
    h = N.Handle(0)
    fp32 = args.precision in ("fp32ir", "bf16ir")
    prec = {"fp64": N.NNLS_FP64, "fp32ir": N.NNLS_FP32_IR, "bf16ir": N.NNLS_BF16_IR}[args.precision]
    leg = measure_single(h, inst, arrays, prec, args.steps, args.warmup, profile=not args.no_profile)
    h.close()
    traffic_src = (CHOL_SOURCES, TRAFFIC_SUMMARY.get((args.workload, args.precision)))
    roof = chol_roofline(leg, {"fp64": "fp64", "fp32ir": "fp32", "bf16ir": "bf16"}[args.precision], traffic_src)
    out = {
        "metric": METRIC,
        "value": leg["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "p50_ms": leg["p50_ms"],
        "p99_ms": leg["p99_ms"],
        "pivot_iters_per_s": leg["pivot_iters_per_s"],
        "refinement_steps_per_solve": leg["refinement_steps_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32ir": "f32-factor+f64-refinement",
                  "bf16ir": "f32-factor(bf16-input updates)+f64-refinement"}[args.precision],
        "data": "synthetic",
        "config": {"workload": desc,
                   "path": {"fp64": "plain FP64 GPU path, one problem per call",
                            "fp32ir": "float32 factor, float64 refinement, one problem per call",
                            "bf16ir": "float32 factor with bfloat16-input updates, float64 refinement, "
                                      "one problem per call"}[args.precision],
                   "m": inst.m, "n": inst.n, "nnz": int(inst.A.nnz)},
        "rel_err_vs_planted": leg["rel_err_vs_planted"],
        "free_set_match": leg["free_set_match"],
        "est_rel_err": leg["est_rel_err"],
        "kernel_ms_per_step": leg["kernel_ms_per_step"],
        "factor_launches": leg["factor_launches"],
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_budget)
    print(json.dumps(out), flush=True)


def device_arrays(inst, dev):
    import torch
    A = inst.A
    return {"colptr": torch.from_numpy(A.indptr.astype(np.int32)).to(dev),
            "rowidx": torch.from_numpy(A.indices.astype(np.int32)).to(dev),
            "val": torch.from_numpy(A.data).to(dev),
            "b": torch.from_numpy(inst.b).to(dev),
            "x": torch.empty(inst.n, dtype=torch.float64, device=dev),
            "y": torch.empty(inst.n, dtype=torch.float64, device=dev)}


def measure_single(h, inst, arr, precision, steps, warmup, profile=True):
    """Whole solves of one sparse instance whose inputs are resident on the device: warm-up,
    then `steps` timed solves (HIP-event kernel timings on the solver's stream when profile).
    Returns throughput, latency percentiles, accuracy and the factor launches of the last
    solve (|F| and the leading positions kept from the previous factor)."""
    import torch
    import paper_cs_0408029_amd as N
    opts = N.default_options(precision=precision)
    popts = N.default_options(precision=precision, flags=N.NNLS_FLAG_PROFILE)

    def step(o):
        st, info = N.nnls_solve_csc(h, inst.m, inst.n, arr["colptr"], arr["rowidx"], arr["val"], arr["b"],
                                    arr["x"], arr["y"], o)
        if st != N.NNLS_OK:
            raise RuntimeError(f"solve failed: {N.status_string(st)}")
        return info

    for _ in range(warmup):
        step(opts)
    N.nnls_reset_profile(h)
    torch.cuda.synchronize()
    lat, iters, ir_steps, est = [], 0, 0, []
    with no_gc():
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            info = step(popts if profile else opts)
            lat.append((time.perf_counter() - s0) * 1e3)
            iters += info.iterations
            ir_steps += info.ir_steps
            est.append(info.est_rel_err)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
    prof = N.nnls_get_profile(h)
    trace = N.nnls_get_trace(h, reused=True)
    xh, yh = arr["x"].cpu().numpy(), arr["y"].cpu().numpy()
    return {
        "solves_per_s": round(steps / total, 4),
        "ms_per_step": round(total / steps * 1e3, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "pivot_iters_per_s": round(iters / total, 2),
        "refinement_steps_per_solve": round(ir_steps / steps, 2),
        "rel_err_vs_planted": float(np.linalg.norm(xh - inst.x_star) / np.linalg.norm(inst.x_star)),
        "free_set_match": bool(np.array_equal(xh > 0, inst.active)),
        "est_rel_err": max(est) if precision != N.NNLS_FP64 else None,
        "kernel_ms_per_step": {k: round(v["ms"] / steps, 3) for k, v in prof.items() if v["launches"]},
        "factor_launches": [[r[4], r[5]] for r in trace],
        "_prof": prof, "_x": xh,
    }


def chol_roofline(leg, kind, traffic_src):
    """Roofline of the dominant kernel (the tiled F-block factor) from the HIP-event
    timings of the timed solves: sum over launches of (|F|^3 - p^3)/3 flops (p = kept
    leading positions) over the summed launch durations.  kind: fp64, fp32, or bf16 (the
    float32 factor whose updates -- all but a fraction of a percent of its flops -- run on
    bfloat16 MFMA, so the bfloat16 peak applies)."""
    chol = leg["_prof"]["cholesky"]
    if not (chol["launches"] > 0 and chol["ms"] > 0):
        return None
    achieved = chol["work"] / (chol["ms"] * 1e-3) / 1e12
    peak = {"fp64": PEAK_FP64_TFLOPS, "fp32": PEAK_FP32_TFLOPS, "bf16": PEAK_BF16_TFLOPS}[kind]
    name = {"fp64": "k_chol_tiles<double>", "fp32": "k_chol_tiles<float>",
            "bf16": "k_chol_tiles<float, bf16 updates>"}[kind]
    srcs, summary = traffic_src
    return {"bound": "mfma", "kernel": name,
            "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
            "traffic": profiled_traffic(srcs, summary) if summary else None,
            "launches": chol["launches"], "avg_launch_ms": round(chol["ms"] / chol["launches"], 4),
            "work_per_launch": "(nF^3 - p^3)/3 flops: the F-block factor less its kept leading p columns "
                               "(nF, p per launch of one solve in factor_launches)"}


def public(leg):
    return {k: v for k, v in leg.items() if not k.startswith("_")}


def bench_metric(args):
    """The metric on the largest single-GPU configuration: the sparse 400000 x 50000
    block-band instance solved by the plain float64 path and by the two mixed paths
    (float32 factor; float32 factor with bfloat16-input updates; both with float64
    refinement, y_G and sign tests) in one process on the same device-resident inputs.
    `value` is the bfloat16-update path's solves/s; the plain path, the float32-factor
    path, the ratios, every path's accuracy and the 60000 x 12000 instance's legs go beside
    it."""
    import torch
    import paper_cs_0408029_amd as N
    t0 = time.perf_counter()
    inst, desc = make_instance("sparse_xl")
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    arr = device_arrays(inst, dev)
    h = N.Handle(0)
    prof = not args.no_profile
    plain = measure_single(h, inst, arr, N.NNLS_FP64, args.steps, args.warmup, profile=prof)
    mixed32 = measure_single(h, inst, arr, N.NNLS_FP32_IR, args.steps, args.warmup, profile=prof)
    mixed = measure_single(h, inst, arr, N.NNLS_BF16_IR, args.steps, args.warmup, profile=prof)
    roof = chol_roofline(mixed, "bf16", (CHOL_SOURCES, TRAFFIC_SUMMARY.get(("sparse_xl", "bf16ir"))))
    roof32 = chol_roofline(mixed32, "fp32", (CHOL_SOURCES, TRAFFIC_SUMMARY.get(("sparse_xl", "fp32ir"))))
    roof64 = chol_roofline(plain, "fp64", (CHOL_SOURCES, None))
    x64 = plain["_x"]

    def vs64(leg):
        return float(np.linalg.norm(leg["_x"] - x64) / np.linalg.norm(x64))

    same_free = bool(np.array_equal(mixed["_x"] > 0, x64 > 0) and np.array_equal(mixed32["_x"] > 0, x64 > 0))
    keys = ("solves_per_s", "ms_per_step", "p50_ms", "p99_ms", "pivot_iters_per_s", "rel_err_vs_planted",
            "free_set_match", "kernel_ms_per_step")
    secondary = None
    if not args.no_secondary:
        inst2, desc2 = make_instance("sparse_large")
        arr2 = device_arrays(inst2, dev)
        k2, w2 = max(args.steps, 10), max(args.warmup, 2)
        legs = {name: measure_single(h, inst2, arr2, prec, k2, w2, profile=False)
                for name, prec in (("plain_fp64", N.NNLS_FP64), ("fp32_factor", N.NNLS_FP32_IR),
                                   ("bf16_updates", N.NNLS_BF16_IR))}
        secondary = {"workload": desc2, "steps": k2}
        for name, leg in legs.items():
            secondary[name] = {k: public(leg)[k] for k in ("solves_per_s", "p50_ms", "p99_ms", "rel_err_vs_planted",
                                                            "free_set_match", "est_rel_err",
                                                            "refinement_steps_per_solve")}
        for name in ("fp32_factor", "bf16_updates"):
            secondary[name + "_vs_plain_fp64"] = round(legs[name]["solves_per_s"] / legs["plain_fp64"]["solves_per_s"], 3)
    h.close()
    out = {
        "metric": METRIC,
        "value": mixed["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "p50_ms": mixed["p50_ms"],
        "p99_ms": mixed["p99_ms"],
        "pivot_iters_per_s": mixed["pivot_iters_per_s"],
        "refinement_steps_per_solve": mixed["refinement_steps_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "vs_plain_fp64": round(mixed["solves_per_s"] / plain["solves_per_s"], 3),
        "dtype": "f32-factor(bf16-input updates)+f64-refinement",
        "data": "synthetic",
        "config": {"workload": desc,
                   "path": "mixed: float32 F-block factor whose left-looking updates run on bfloat16 MFMA "
                           "(float32 accumulation), float64 refinement with a compensated residual, float64 "
                           "y_G and sign tests; one problem per call",
                   "baseline_path": "plain FP64 GPU path, one problem per call, same process and inputs",
                   "m": inst.m, "n": inst.n, "nnz": int(inst.A.nnz)},
        "rel_err_vs_planted": mixed["rel_err_vs_planted"],
        "rel_err_vs_plain_fp64": vs64(mixed),
        "est_rel_err": mixed["est_rel_err"],
        "free_set_match": mixed["free_set_match"] and plain["free_set_match"] and mixed32["free_set_match"]
                          and same_free,
        "plain_fp64": {k: public(plain)[k] for k in keys},
        "fp32_factor": dict({k: public(mixed32)[k] for k in keys},
                            refinement_steps_per_solve=mixed32["refinement_steps_per_solve"],
                            est_rel_err=mixed32["est_rel_err"], rel_err_vs_plain_fp64=vs64(mixed32),
                            vs_plain_fp64=round(mixed32["solves_per_s"] / plain["solves_per_s"], 3),
                            roofline=roof32),
        "plain_fp64_roofline": roof64,
        "kernel_ms_per_step": mixed["kernel_ms_per_step"],
        "factor_launches": mixed["factor_launches"],
        "roofline": roof,
        "secondary": secondary,
        "generation_s": round(gen_s, 1),
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_budget, max_solves=1,
                                           what="whole solve(s) of the 400000 x 50000 instance")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
