#!/usr/bin/env python3
"""Benchmark of the MI355X multigrid Poisson hot path (HONEI, arXiv 0904.4152).

A step is one mixed-precision solve (FP32 V(2,2) cycles inside an FP64 defect
correction) to 1e-8 relative residual of the 4097 x 4097 (L = 12) Q1 Poisson
problem on a grid jittered by +-0.2 h with a Gaussian right-hand side; the
hierarchy (bands of all levels) and b are resident in HBM before timing.
Prints one JSON line with solves/s (value), the roofline of the dominant
kernel (the finest-level fused FP32 pre-smoothing pass: two damped Jacobi
sweeps, the defect and its restriction in one sweep over the bands), the
band-SpMV GB/s, the plain FP64 solve time beside the mixed one, the L = 10
and L = 6 workloads, the batched and serving workloads, and the oracle timed
on the host CPU, whose FP64 solutions of the L = 12, 10 and 6 problems give
each GPU result's error against the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
# Algorithmic bytes per finest node of one fused FP32 smoothing pass: the nine
# stored bands, x and b read and the iterate written (12 scalars of 4 bytes);
# the coarse vector (one scalar per coarse node) is added separately.
FUSED_ALG_B = 12 * 4
# What the pass must at least move: the matrix is symmetric bit for bit, so
# it reads the diagonal and the four upper bands only (8 scalars per node).
FUSED_MIN_B = 8 * 4
# Sources the fused passes are built from: a counter record taken on other
# sources is stale.
TRAFFIC_SOURCES = ["csrc/kernels.hip", "csrc/fused_ops.h", "csrc/device_ops.h",
                   "csrc/mg_internal.h", "build.py"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=50)
    ap.add_argument("--only-kernels", action="store_true",
                    help="time the band kernels only (for profiler runs)")
    ap.add_argument("--only-step", action="store_true",
                    help="set up the L = 12 workload and run the warm-up and timed steps "
                         "only (for profiler runs of exactly the timed step)")
    ap.add_argument("--tiles", default=None,
                    help="install the L = 12 tiles from this file (written by --save-tiles) "
                         "instead of autotuning them (for profiler runs)")
    ap.add_argument("--save-tiles", default=None,
                    help="write the L = 12 tiles the autotuner picked to this file")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--only-batch", action="store_true",
                    help="set up the 256-problem batch, tune its tiles and run --warmup untimed "
                         "and --steps timed batched solves only (for profiler runs)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-count", type=int, default=20000)
    ap.add_argument("--serve-warmup", type=int, default=2000)
    ap.add_argument("--serve-slots", type=int, default=64)
    return ap.parse_args()


def _code_only(src: str) -> str:
    """C++ source without comments and with whitespace collapsed: what the
    compiler sees of it (no string literal in the hashed sources holds a
    comment marker)."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_hash() -> str:
    """Hash of the code (comments excluded) and build flags of the band
    kernels and fused passes whose HBM counters profiles/hbm_traffic.json
    records."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_0904_4152_amd")
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(pkg, name)) as f:
            h.update(name.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key: str):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary
    under profiles/ was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("kernels", {}).get(kernel_key)


def time_launches(fn, iters, torch):
    """Average duration of fn() launches, timed with HIP events recorded on
    the stream the kernels are launched on (torch's current stream)."""
    st = torch.cuda.current_stream()
    for _ in range(5):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(iters):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / iters


def bench_blas1(ctx, torch, dev, sizes=None):
    """BLAS level 1 (Sec. 6.1) over lengths from cache-resident to HBM-sized:
    axpy (asynchronous, HIP-event timed per launch; 3 streams, 2 flops per
    element) and dot / norm2 (synchronous calls, host wall time including the
    result's return; 2 / 1 streams)."""
    sizes = sizes or [1 << 16, 1 << 20, 1 << 24, 1 << 28]
    rows = []
    for n in sizes:
        rec = {"n": n}
        for name, dt, es in (("saxpy", torch.float32, 4), ("daxpy", torch.float64, 8)):
            x = torch.ones(n, dtype=dt, device=dev)
            y = torch.ones(n, dtype=dt, device=dev)
            iters = max(10, min(2000, (1 << 26) // n))
            t = time_launches(lambda: ctx.axpy(1e-3, x, y), iters, torch)
            rec[name] = {"us": t * 1e6, "GB_s": 3 * es * n / t / 1e9,
                         "MFLOP_s": 2 * n / t / 1e6}
            if name == "saxpy":
                reps = max(5, min(200, (1 << 24) // n))
                for op, fn, streams in (("sdot", lambda: ctx.dot(x, y), 2),
                                        ("snrm2", lambda: ctx.norm2(x), 1)):
                    fn()
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        fn()
                    t = (time.perf_counter() - t0) / reps
                    rec[op] = {"us": t * 1e6, "GB_s": streams * es * n / t / 1e9}
            del x, y
        rows.append(rec)
    torch.cuda.empty_cache()
    return rows


def bench_band4(ctx, torch, dev, N=4096, iters=50):
    """The shallow-water prediction step (Sec. 2.2) as one fused pass on an
    N x N grid in FP32: u_new = u + M1 v + M2 w + M3 u + M4 u + s with four
    four-band matrices (x and y second-order differences and their mixed
    stencils).  Algorithmic bytes per node: 16 band values, the distinct
    vectors v, w, u and s read once and u_new written (84 B)."""
    n = N * N
    g = torch.Generator(device=dev).manual_seed(5)
    bands = [torch.rand((4, n), generator=g, device=dev, dtype=torch.float32) for _ in range(4)]
    v, w, u, s = (torch.rand(n, generator=g, device=dev, dtype=torch.float32) for _ in range(4))
    out = torch.empty_like(u)
    offs = [(-2, -1, 1, 2), (-2 * N, -N, N, 2 * N), (-1, 1, -N, N),
            (-N - 1, -N + 1, N - 1, N + 1)]
    t = time_launches(lambda: ctx.band4_combine(bands, offs, [v, w, u, u], u, out, s=s), iters,
                      torch)
    alg = 84 * n
    res = {"N": N, "n": n, "us": t * 1e6, "alg_bytes": alg, "GB_s": alg / t / 1e9,
           "frac_hbm_peak": alg / t / 1e9 / PEAK_HBM_GBS}
    del bands, v, w, u, s, out
    torch.cuda.empty_cache()
    return res


def batch_problems(mg, ctx, synth, torch, dev, count=256):
    """The 256-problem composition: levels U{5..9} (seed 4004), jitter
    U[0, 0.25) h (seed 4005), geometry seed 4100+p, uniform RHS seed 4200+p."""
    levels = synth.batch_levels(count, 5, 9, 4004)
    amps = synth.batch_jitter(count, 0.25, 4005)
    hs, bs, xs = [], [], []
    for p in range(count):
        h = mg.Hierarchy(ctx, int(levels[p]), jitter=float(amps[p]), seed=4100 + p)
        b = torch.empty(h.n, dtype=torch.float64, device=dev)
        h.rhs_uniform(4200 + p, b)
        hs.append(h)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    return levels, hs, bs, xs


def bench_batch_only(mg, ctx, synth, torch, dev, args):
    """The batch alone: tuned tiles, then --warmup and --steps batched
    solves (each from zero initial guesses, which the library does not read)."""
    opts = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8, zero_guess=1)
    _, hs, bs, xs = batch_problems(mg, ctx, synth, torch, dev)
    mg.batch_clear_tiles()
    mg.solve_batch(hs, bs, xs, opts)
    mg.batch_autotune(hs, opts, reps=10)
    dts = []
    for i in range(args.warmup + args.steps):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = mg.solve_batch(hs, bs, xs, opts)
        torch.cuda.synchronize()
        if i >= args.warmup:
            dts.append(time.perf_counter() - t0)
    ok = all(s.status == 0 and s.rel_res <= opts.rel_tol for s in stats)
    print(json.dumps({"only_batch": True, "ms_per_batch": float(np.median(dts)) * 1e3,
                      "steps": args.steps, "warmup": args.warmup, "all_reached_tol": ok}))
    for h in hs:
        h.close()


def bench_batch(mg, ctx, synth, torch, dev, opts, count=256):
    """256 independent mixed solves advanced together (one persistent launch
    per V-cycle stage), against the same problems solved one after another."""
    levels, hs, bs, xs = batch_problems(mg, ctx, synth, torch, dev, count)
    # tile heights picked by the autotuner for this composition (no result
    # bit depends on them); the rule's choice is timed as well, for reference
    mg.batch_clear_tiles()
    mg.solve_batch(hs, bs, xs, opts)  # warm-up (graph capture)
    t_rule = []
    for _ in range(3):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mg.solve_batch(hs, bs, xs, opts)
        torch.cuda.synchronize()
        t_rule.append(time.perf_counter() - t0)
    t0 = time.perf_counter()
    tiles = mg.batch_autotune(hs, opts, reps=10)
    t_tune = time.perf_counter() - t0
    mg.solve_batch(hs, bs, xs, opts)  # warm-up with the tuned tiles
    reps = 5
    dts = []
    for _ in range(reps):
        for x in xs:  # the zero initial guesses are inputs: set outside the timed call
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = mg.solve_batch(hs, bs, xs, opts)
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t0)
    dt = float(np.median(dts))
    ok = all(s.status == 0 and s.rel_res <= opts.rel_tol for s in stats)
    alg = sum(s.alg_bytes for s in stats)
    dt_seq = 0.0
    for h, b, x in zip(hs, bs, xs):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.solve(b, x, opts)
        torch.cuda.synchronize()
        dt_seq += time.perf_counter() - t0
    rec = {"problems": count, "unknowns": int(sum(h.n for h in hs)),
           "levels": {int(L): int((levels == L).sum()) for L in range(5, 10)},
           "ms": dt * 1e3, "solves_s": count / dt, "all_reached_tol": ok,
           "alg_GB_s": alg / dt / 1e9, "sequential_ms": dt_seq * 1e3,
           "speedup_vs_sequential": dt_seq / dt,
           "mean_outer": float(np.mean([s.outer_steps for s in stats])),
           "mean_inner": float(np.mean([s.cycles for s in stats])),
           "autotune": {"seconds": t_tune, "tiles": tiles,
                        "rule_tiles_ms": float(np.median(t_rule)) * 1e3}}
    for h in hs:
        h.close()
    return rec


def serve_once(mg, ctx, synth, rate, n_warm, n_meas, slots, budget):
    import threading
    srv = mg.Server(ctx, slots=slots, budget_bytes=budget, max_level=11,
                    opts=mg.default_opts(precision=mg.MG_PREC_MIXED))
    total = n_warm + n_meas
    req = synth.serving_requests(total, rate, 5005)
    lat = {}
    failures = []

    def collect():
        got = 0
        while got < total:
            r = srv.next(timeout=30.0)
            if r is None:
                failures.append("timeout")
                return
            t, rc, st = r
            if rc != 0:
                failures.append(rc)
            lat[t] = (st.seconds, st.queue_seconds, st.cycles, st.outer_steps)
            got += 1

    th = threading.Thread(target=collect)
    th.start()
    tickets = []
    start = time.perf_counter()
    t_first_meas = None
    for r in range(total):
        due = start + req["t"][r]
        now = time.perf_counter()
        if due > now:
            time.sleep(due - now)
        if r == n_warm:
            t_first_meas = time.perf_counter()
        tickets.append(srv.submit(int(req["L"][r]), float(req["tol"][r]),
                                  float(req["jitter"][r]), int(req["geom_seed"][r]),
                                  int(req["rhs_seed"][r])))
    t_last_submit = time.perf_counter()
    th.join()
    t_end = time.perf_counter()
    info = srv.info()
    srv.close()
    meas = [lat[t] for t in tickets[n_warm:] if t in lat]
    ls = np.array([m[0] for m in meas]) * 1e3
    qs = np.array([m[1] for m in meas]) * 1e3
    dur = t_end - t_first_meas
    return {"offered_req_s": rate,
            "submitted_req_s": n_meas / max(t_last_submit - t_first_meas, 1e-9),
            "achieved_solves_s": n_meas / dur, "requests": n_meas, "warmup": n_warm,
            "slots": slots, "budget_GB": budget / 1e9,
            "p50_ms": float(np.percentile(ls, 50)), "p90_ms": float(np.percentile(ls, 90)),
            "p99_ms": float(np.percentile(ls, 99)), "mean_queue_ms": float(qs.mean()),
            "mean_service_ms": float((ls - qs).mean()),
            "hbm_high_water_GB": info.bytes_high_water / 1e9,
            "queue_high_water": int(info.queue_high_water), "failures": len(failures)}


def bench_serving(mg, ctx, synth, args):
    budget = 200 * 10 ** 9
    rec = {"headline": serve_once(mg, ctx, synth, args.serve_rate, args.serve_warmup,
                                  args.serve_count, args.serve_slots, budget)}
    sweep = []
    for rate in (250, 500, 1000):
        sweep.append(serve_once(mg, ctx, synth, rate, 100, 400, args.serve_slots, budget))
    rec["sweep"] = sweep
    return rec


def progress(msg: str) -> None:
    """One line per finished phase on stderr (stdout carries only the JSON)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def host_cpu():
    try:
        model = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                     if ln.startswith("model name"))
    except (OSError, StopIteration):
        model = "unknown"
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count()
    return {"nproc": affinity, "cpu_count": os.cpu_count(), "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def oracle_baseline(L, jit, gseed, rseed, synth):
    """The oracle's FP64 solve of the L = 12 problem on the host: once on one
    thread (the paper's one-core protocol) and once on every host core (the
    OpenMP build: element-wise loops threaded, same bits).  Assembly is
    excluded from both timings.  Returns the baseline record and the
    solution."""
    import oracle
    xy = synth.coords(L, jit, gseed)
    bh = synth.rhs_gaussian(L, rseed)
    runs = {}
    xo = ost = None
    for threaded in (False, True):
        oh = oracle.Hierarchy(L, xy, threaded=threaded)
        t0 = time.perf_counter()
        x_, st_ = oh.solve_fp64(bh, o=oracle.opts(rel_tol=1e-8))
        dt = time.perf_counter() - t0
        oh.close()
        runs[threaded] = (dt, st_.cycles, oracle.threads(threaded))
        if xo is None:
            xo, ost = x_, st_
        elif not np.array_equal(xo, x_):
            raise RuntimeError("threaded oracle differs from the one-thread oracle")
    dt1, cyc, _ = runs[False]
    dtn, _, nthr = runs[True]
    cpu = {"value": 1.0 / dtn, "unit": "solves/s", "cores": nthr, "kind": "oracle",
           "sample": "one plain FP64 V(2,2) solve to 1e-8 of the same L=12 problem "
                     "(%d cycles, assembly excluded) on %d host threads: %.2f s; "
                     "one thread: %.1f s" % (cyc, nthr, dtn, dt1),
           "seconds": dtn,
           "single_thread": {"value": 1.0 / dt1, "unit": "solves/s", "cores": 1,
                             "seconds": dt1},
           "host": host_cpu()}
    return cpu, xo, ost


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (each problem and each solve "
              "runs on a single MI355X); --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_0904_4152_amd as mg
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = mg.Context(0)
    out = {}
    if args.only_batch:
        bench_batch_only(mg, ctx, synth, torch, dev, args)
        return

    # ---------------- headline workload: L = 12, jitter 0.2 h, Gaussian RHS
    L, jit, gseed, rseed = 12, 0.2, 1003, 2003
    t = time.perf_counter()
    h = mg.Hierarchy(ctx, L, jitter=jit, seed=gseed)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    # the fused passes' tiles (rows per tile, wavefronts per row) of every
    # level, picked by the autotuner before anything is timed (no result bit
    # depends on them)
    mg.batch_clear_tiles()
    t = time.perf_counter()
    if args.tiles:
        tiles = mg.load_tiles(args.tiles)
    else:
        tiles = h.autotune(reps=10)
        if args.save_tiles:
            mg.save_tiles(tiles, args.save_tiles)
    t_tune = time.perf_counter() - t
    n = h.n
    b = torch.from_numpy(synth.rhs_gaussian(L, rseed)).to(dev)
    x = torch.zeros_like(b)
    # every solve starts from x = 0: zero_guess tells the library, which then
    # does not read x (no fill of x and no test of it for zero per solve)
    mixed = mg.default_opts(precision=mg.MG_PREC_MIXED, rel_tol=1e-8, zero_guess=1)
    fp64 = mg.default_opts(precision=mg.MG_PREC_FP64, rel_tol=1e-8, zero_guess=1)

    def solve(hh, bb, xx, o):
        if not o.zero_guess:
            xx.zero_()
        st = hh.solve(bb, xx, o)
        if st.status != 0 or st.rel_res > 1e-8:
            raise RuntimeError("solve did not reach 1e-8: status %d rel_res %g"
                               % (st.status, st.rel_res))
        return st

    def timed_step():
        for _ in range(args.warmup):
            solve(h, b, x, mixed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = [solve(h, b, x, mixed) for _ in range(args.steps)]
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, stats[-1]

    if args.only_step:
        t_mixed, st_m = timed_step()
        print(json.dumps({"only_step": True, "ms_per_step": t_mixed * 1e3,
                          "steps": args.steps, "warmup": args.warmup,
                          "outer_steps": st_m.outer_steps, "inner_cycles": st_m.cycles,
                          "rel_res": st_m.rel_res}))
        return

    # band kernels at full size (FP32 bands 604 MB: larger than the 256 MB
    # Infinity Cache, so these are HBM rates)
    rng = np.random.default_rng(0)
    x32 = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(dev)
    y32 = torch.empty_like(x32)
    b32 = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(dev)
    x64 = x32.double()
    y64 = torch.empty_like(x64)
    b64 = b32.double()
    it = args.kernel_iters
    t_spmv32 = time_launches(lambda: h.spmv(L, x32, y32), it, torch)
    t_spmv64 = time_launches(lambda: h.spmv(L, x64, y64), it, torch)
    t_jac32 = time_launches(lambda: h.jacobi(L, b32, x32, y32, 0.7), it, torch)
    # the FP64 outer defect of the mixed solve (diagonal and upper bands read)
    t_def64 = time_launches(lambda: h.defect(L, b64, x64, y64), it, torch)
    # the fused passes of the FP32 cycle on the finest level (the solve's
    # dominant kernels): pre = 2 sweeps + defect + restriction, post =
    # prolongation + 2 sweeps + residual norm
    Nc = ((1 << (L - 1)) + 1) ** 2
    bc32 = torch.zeros(Nc, dtype=torch.float32, device=dev)
    t_pre32 = time_launches(lambda: h.pre_smooth(L, b32, x32, y32, bc32), it, torch)
    t_post32 = time_launches(lambda: h.post_smooth(L, b32, x32, bc32, y32), it, torch)
    gbs = lambda by, s: by / s / 1e9

    def rec(t_, alg, minimum=None):
        r = {"us": t_ * 1e6, "alg_bytes": alg, "GB_s": gbs(alg, t_),
             "frac_hbm_peak": gbs(alg, t_) / PEAK_HBM_GBS}
        if minimum is not None:
            r["min_bytes"] = minimum
            r["GB_s_min_bytes"] = gbs(minimum, t_)
        return r

    fused_alg = FUSED_ALG_B * n + 4 * Nc
    fused_min = FUSED_MIN_B * n + 4 * Nc
    out["band_kernels"] = {
        # nine bands + x read, y written
        "spmv_fp32": rec(t_spmv32, 11 * 4 * n),
        "spmv_fp64": rec(t_spmv64, 11 * 8 * n),
        # nine bands + x + b read, x' written
        "jacobi_fp32": rec(t_jac32, 12 * 4 * n),
        # nine bands + x + b read, d written; it reads 5 bands (the lower ones
        # are the neighbours' upper ones): min_bytes
        "defect_fp64": rec(t_def64, 12 * 8 * n, 8 * 8 * n),
        # pre: 2 sweeps + defect + restriction; post: prolongation + 2 sweeps
        "fused_pre_fp32": rec(t_pre32, fused_alg, fused_min),
        "fused_post_fp32": rec(t_post32, fused_alg, fused_min),
    }
    del bc32
    del x32, y32, b32, x64, y64, b64
    if args.only_kernels:
        # saxpy at 2^28 elements (1 GiB per vector): the BLAS-1 reference rate
        out["blas1"] = bench_blas1(ctx, torch, dev, sizes=[1 << 28])
        out["swe_band4"] = bench_band4(ctx, torch, dev)
        # a plain device copy of known size (1 GiB read + 1 GiB written):
        # the calibration reference for the HBM byte counters
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        t_copy = time_launches(lambda: dst.copy_(src), 5, torch)
        out["calibration_copy"] = {"bytes_read": src.numel() * 4, "bytes_written": src.numel() * 4,
                                   "us": t_copy * 1e6,
                                   "GB_s": 2 * src.numel() * 4 / t_copy / 1e9}
        print(json.dumps(out))
        return

    progress("band kernels timed")
    t_mixed, st_m = timed_step()
    x_mixed = x.cpu().numpy()
    progress("timed step: %.3f ms per mixed solve" % (t_mixed * 1e3))

    st_f = solve(h, b, x, fp64)  # warm the FP64 graphs
    t0 = time.perf_counter()
    nf = 2
    for _ in range(nf):
        st_f = solve(h, b, x, fp64)
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t0) / nf
    x_fp64 = x.cpu().numpy()
    out["L12"] = {
        "n": n, "setup_s": t_setup,
        "autotune": {"seconds": t_tune, "tiles": tiles},
        "mixed": {"ms": t_mixed * 1e3, "outer_steps": st_m.outer_steps,
                  "inner_cycles": st_m.cycles, "rel_res": st_m.rel_res,
                  "alg_bytes": st_m.alg_bytes, "alg_GB_s": st_m.alg_bytes / t_mixed / 1e9},
        "fp64": {"ms": t_fp64 * 1e3, "cycles": st_f.cycles, "rel_res": st_f.rel_res,
                 "alg_bytes": st_f.alg_bytes, "alg_GB_s": st_f.alg_bytes / t_fp64 / 1e9},
        "mixed_speedup_vs_fp64": t_fp64 / t_mixed,
    }

    def timed(hh, o, reps=3):
        st = solve(hh, b, x, o)  # warm the graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st = solve(hh, b, x, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        return {"ms": dt * 1e3, "steps": st.cycles, "outer_steps": st.outer_steps,
                "rel_res": st.rel_res, "alg_GB_s": st.alg_bytes / dt / 1e9}

    # CG preconditioned by one cycle (FP64 cycle; FP32 cycle on r / ||r||)
    out["L12"]["pcg_fp64"] = timed(h, mg.default_opts(precision=mg.MG_PREC_FP64, rel_tol=1e-8,
                                                      krylov=1, zero_guess=1))
    out["L12"]["pcg_mixed"] = timed(h, mg.default_opts(precision=mg.MG_PREC_MIXED,
                                                       rel_tol=1e-8, krylov=1, zero_guess=1))
    h.close()
    torch.cuda.empty_cache()
    # coarse grid on level 4 (17 x 17) solved by CG, as in the paper's setup
    h4 = mg.Hierarchy(ctx, L, coarse_level=4, jitter=jit, seed=gseed)
    h4.set_coarse_solver(mg.MG_COARSE_CG, tol=1e-10, max_iter=200)
    out["L12"]["mixed_cg_coarse_L4"] = timed(h4, mixed)
    h4.close()
    del b, x
    torch.cuda.empty_cache()
    progress("L = 12 FP64, CG variants done")

    # ---------------- L = 10 (FP64 vs mixed) and L = 6 (sin sin, FP64)
    small_x = {}
    for name, (LL, a, gs, kind, reps) in {"L10": (10, 0.2, 1002, "uniform", 5),
                                          "L6": (6, 0.0, 0, "sinsin", 20)}.items():
        hh = mg.Hierarchy(ctx, LL, jitter=a, seed=gs)
        if kind == "uniform":
            bb = torch.from_numpy(synth.rhs_uniform(LL, 2002)).to(dev)
        else:
            bb = torch.empty(hh.n, dtype=torch.float64, device=dev)
            hh.rhs_sinsin(bb)
        xx = torch.zeros_like(bb)
        r_ = {}
        for pname, o in (("fp64", fp64), ("mixed", mixed)):
            solve(hh, bb, xx, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                s = solve(hh, bb, xx, o)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            r_[pname] = {"ms": dt * 1e3, "solves_s": 1.0 / dt, "cycles": s.cycles,
                         "outer_steps": s.outer_steps, "rel_res": s.rel_res}
            small_x[(name, pname)] = xx.cpu().numpy()
        out[name] = r_
        hh.close()

    progress("L = 10 and L = 6 done")
    # ---------------- BLAS level 1 at lengths from cache- to HBM-resident
    out["blas1"] = bench_blas1(ctx, torch, dev)
    # ---------------- shallow-water prediction step (four-band combination)
    out["swe_band4"] = bench_band4(ctx, torch, dev)

    # ---------------- batched: 256 problems, L ~ U{5..9}, jitter U[0, 0.25) h
    if not args.no_batch:
        out["batch256"] = bench_batch(mg, ctx, synth, torch, dev, mixed)
        torch.cuda.empty_cache()
        progress("batch done")
    # ---------------- serving: Poisson arrivals, P(L) ~ 1/L on 6..11
    if not args.no_serving:
        out["serving"] = bench_serving(mg, ctx, synth, args)
        progress("serving done")

    # ---------------- oracle on the host CPU (bounded sample)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cpu, xo, ost = oracle_baseline(L, jit, gseed, rseed, synth)
        progress("oracle timed: %.1f s one thread, %.2f s on %d threads"
                 % (cpu["single_thread"]["seconds"], cpu["seconds"], cpu["cores"]))

        # each GPU result against the oracle's FP64 solution of the same problem
        # (inputs from the host generators and the oracle's own load vector)
        def vs_oracle(xo_, ost_, xf, xm):
            xn = float(np.linalg.norm(xo_))
            return {"oracle_cycles": ost_.cycles,
                    "fp64_rel_solution_diff": float(np.linalg.norm(xf - xo_)) / xn,
                    "mixed_rel_solution_diff": float(np.linalg.norm(xm - xo_)) / xn}

        out["L12"]["vs_oracle"] = vs_oracle(xo, ost, x_fp64, x_mixed)
        for name, LL, a, gs in (("L10", 10, 0.2, 1002), ("L6", 6, 0.0, 0)):
            xy_s = synth.coords(LL, a, gs)
            Ns = (1 << LL) + 1
            b_s = (synth.rhs_uniform(LL, 2002) if name == "L10"
                   else oracle.load_vector(Ns, xy_s, fn=0))
            oh_s = oracle.Hierarchy(LL, xy_s, threaded=True)
            xo_s, ost_s = oh_s.solve_fp64(b_s, o=oracle.opts(rel_tol=1e-8))
            oh_s.close()
            out[name]["vs_oracle"] = vs_oracle(xo_s, ost_s, small_x[(name, "fp64")],
                                               small_x[(name, "mixed")])

    bk = out["band_kernels"]
    pre = bk["fused_pre_fp32"]
    traffic = traffic_from_profiles("fused_pre_fp32")
    top = next(r for r in tiles if r["level"] == L)
    roof = {"bound": "hbm", "achieved": pre["GB_s"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": pre["GB_s"] / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": "k_pre<float, false, %d> (finest-level fused FP32 pre-smoothing pass: "
                      "two damped Jacobi sweeps, defect, restriction; tiles of %d rows)"
                      % (64 * top["row_waves"], top["tile_rows"]),
            "us": pre["us"],
            "alg_bytes": fused_alg,
            "alg_bytes_model": "12 scalars per finest node (9 stored bands, x and b read, "
                               "iterate written) + 1 per coarse node (coarse rhs written)",
            "min_bytes": fused_min,
            "frac_min_bytes": pre["GB_s_min_bytes"] / PEAK_HBM_GBS,
            "min_bytes_model": "8 scalars per finest node (diagonal and 4 upper bands, x, b, "
                               "iterate) + 1 per coarse node",
            "frac_counter_traffic": (traffic / (pre["us"] * 1e-6) / 1e9 / PEAK_HBM_GBS
                                     if traffic else None)}
    line = {
        "metric": "MG solves/s & band-SpMV GB/s (mixed vs FP64 @1e-8 rel.res); serving p99",
        "value": 1.0 / t_mixed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "Q1 Poisson mixed-precision MG solve, 4097x4097 (L=12), "
                               "jitter 0.2h seed 1003, Gaussian RHS seed 2003, V(2,2) "
                               "omega 0.7, rel.res 1e-8",
                   "L": L, "unknowns": n},
        "roofline": roof,
        "cpu_baseline": cpu,
        "spmv_fp32_GB_s": bk["spmv_fp32"]["GB_s"],
        "spmv_fp32_frac": bk["spmv_fp32"]["frac_hbm_peak"],
        "spmv_fp64_GB_s": bk["spmv_fp64"]["GB_s"],
        "spmv_fp64_frac": bk["spmv_fp64"]["frac_hbm_peak"],
        "mixed_ms": t_mixed * 1e3,
        "fp64_ms": t_fp64 * 1e3,
        "mixed_speedup_vs_fp64": t_fp64 / t_mixed,
        "speedup_vs_oracle_all_cores": (cpu["seconds"] / t_mixed) if cpu else None,
    }
    if "batch256" in out:
        line["batch256_ms"] = out["batch256"]["ms"]
        line["batch256_solves_s"] = out["batch256"]["solves_s"]
    if "serving" in out:
        hd = out["serving"]["headline"]
        line["serving_solves_s"] = hd["achieved_solves_s"]
        line["serving_p50_ms"] = hd["p50_ms"]
        line["serving_p99_ms"] = hd["p99_ms"]
    line.update(out)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
