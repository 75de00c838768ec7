"""All-mode sparse MTTKRP benchmark on one MI355X.

Workload (default): 3-mode 200000 x 150000 x 100000 tensor, 20M distinct
nonzeros with Zipf(1.2) index skew per mode, values U(0,1) fp32, rank 32, fp32
factors.  One step = the MTTKRP along every mode in turn (the paper's total
execution time sums the per-mode MTTKRP times), with the mode copies and
factors resident in HBM before timing starts.  The CP-ALS sweep (MTTKRPs plus
the FP64 normal-equation updates) and the layout build are timed separately
and reported in the same JSON line, and so are the second half of the metric:
`batch` (256 small tensors: batched vs per-tensor launches, 20 CP-ALS sweeps
in a HIP graph) and `serve` (Poisson CP-ALS jobs at 0.95 and 2 x the plain
method's capacity: jobs/s and p50/p99 latency, continuous batching vs one job
at a time).

Prints one JSON line.  ``--gpus`` above 1 is refused: the library runs on one
device.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "all-mode spMTTKRP GFLOP/s & HBM % peak; batched req/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0

DEFAULT_WORKLOAD = "zipf1.2-20M-R32"
WORKLOADS = {
    "zipf1.2-20M-R32": dict(tensor="zipf1.2-20M", R=32),
    "precision-100M-4mode": dict(tensor="zipf1.1-100M-4mode", R=32),
    "uniform-100k-R16": dict(tensor="small-uniform", R=16),
    "batch256-R16": dict(tensor=None, R=16),
    "serve-poisson": dict(tensor=None, R=0),
    "paper-shapes": dict(tensor=None, R=32),
}

# Shapes and nonzero counts of the paper's evaluation tensors (its Table III),
# for synthetic stand-ins (seeded, Zipf(1.2) per mode).  The 3-mode
# 2.9M x 2.1M x 25.5M, 143.6M-nonzero one takes a few minutes to generate and
# is kept apart (--skip-large-shape leaves it out).
PAPER_SHAPES = {
    "chicago-like": ((6200, 24, 77, 32), 5_300_000),
    "enron-like": ((6100, 5700, 244_300, 1200), 54_200_000),
    "nips-like": ((2500, 2900, 14_000, 17), 3_100_000),
    "uber-like": ((183, 24, 1100, 1700), 3_300_000),
    "vast-like": ((165_400, 11_400, 2, 100, 89), 26_000_000),
}
PAPER_SHAPE_LARGE = {"nell1-like": ((2_900_000, 2_100_000, 25_500_000), 143_600_000)}


def default_shape(N, R):
    """The library's default launch shape as the shape autotuner names it:
    8 partitions per CU; for 3 modes 512 threads and 4 gathers (2 at R = 16)."""
    return (8, 512, 2 if R == 16 else 4) if N == 3 else (8, 0, 0)


def algorithmic_bytes(dims, nnz, R, factor_bytes=4, idx16_modes=0):
    """Bytes a mode's MTTKRP must move: the mode copy's indices (4 bytes each,
    2 in the copies of output modes whose bit is set in idx16_modes) and
    values, a 4-byte row pointer per output row, each input factor read once,
    the output written once."""
    N = len(dims)
    per_mode = []
    for n in range(N):
        ib = 2 if idx16_modes >> n & 1 else 4
        b = nnz * (ib * (N - 1) + 4) + 4 * (dims[n] + 1)
        b += sum(dims[m] * R * factor_bytes for m in range(N) if m != n)
        b += dims[n] * R * 4
        per_mode.append(b)
    return per_mode


def sources_digest():
    """SHA-256 over the sources that shape the per-mode MTTKRP launches (partition
    and fix-up kernels, their launch geometry and the layout; the CP-ALS and
    probe kernels are left out), sorted by name, with comments and blank
    lines removed: HBM traffic counted for one build of that code is only
    reported for that code."""
    import hashlib
    import re
    d = os.path.join(ROOT, "paper_2503_18198_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip", ".cpp")) and name != "als_kernels.hip" and not name.startswith("probe"):
            with open(os.path.join(d, name), encoding="utf-8") as f:
                text = f.read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
            code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
            h.update(name.encode())
            h.update(code.encode())
    return h.hexdigest()


def profiled_traffic(workload):
    """HBM bytes per mode of the MTTKRP (the partition kernel and its fix-up
    launches) from the committed rocprofv3 counter summary of this workload
    (FETCH_SIZE and WRITE_SIZE in KiB, scaled by the factors a plain copy of
    known size gives), or None when the summary is missing or was taken from
    other sources."""
    path = os.path.join(ROOT, "profiles", f"mttkrp_{workload}.traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != sources_digest():
        return None
    fetch = float(kv["fetch_kib_per_launch"]) * float(kv["fetch_factor"])
    write = float(kv["write_kib_per_launch"]) * float(kv["write_factor"])
    return round((fetch + write) * 1024.0), kv.get("launch_shape")


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(t, R, F, budget_s=20.0):
    """The FP64 oracle on the host, all modes, on a bounded leading sample of
    the nonzeros: median of 3 runs on every host thread, and one run on 1
    thread, each sample doubled until a run takes about budget_s/10 (the
    whole baseline then takes about budget_s)."""
    import oracle

    threads = max(1, min(os.cpu_count() or 1, 64))
    N = len(t.dims)
    F64 = [f.astype(np.float64) for f in F]
    val = t.val.astype(np.float64)

    def run(sample, nthr):
        t0 = time.perf_counter()
        for n in range(N):
            oracle.mttkrp(t.idx[:sample], val[:sample], t.dims, F64, n, threads=nthr)
        return time.perf_counter() - t0

    def sized(nthr, seconds):
        # Double the sample until one run takes `seconds`: the oracle's
        # per-thread outputs are a fixed cost that a small probe over-weights.
        sample = min(t.nnz, 1_000_000)
        while sample < t.nnz and run(sample, nthr) < seconds:
            sample = min(t.nnz, 2 * sample)
        return sample

    s_all = sized(threads, budget_s / 10)
    times = sorted(run(s_all, threads) for _ in range(3))
    dt_all = times[1]
    s_one = sized(1, budget_s / 10)
    dt_one = run(s_one, 1)
    rate_all = N * R * s_all * N / dt_all / 1e9
    rate_one = N * R * s_one * N / dt_one / 1e9
    return {"value": rate_all, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"first {s_all} of {t.nnz} nonzeros, all {N} modes, R={R}, FP64 C oracle, "
                      f"{threads} OpenMP threads, median of 3 runs ({', '.join(f'{x:.2f}' for x in times)} s)",
            "single_thread": {"value": rate_one, "unit": "GFLOP/s",
                              "sample": f"first {s_one} nonzeros, all {N} modes, 1 thread, {dt_one:.2f} s"},
            "cpu_model": cpu_model()}


def bench_batch(args, R=16, count=256):
    """Many small uneven tensors: all tensors' MTTKRP along each mode in one
    batched launch pair vs one launch pair per tensor (the plain method).
    Returns the result line as a dict."""
    import torch

    import workloads
    from paper_2503_18198_amd import capi

    t0 = time.perf_counter()
    ts = workloads.batch_tensors(count=count)
    gen_s = time.perf_counter() - t0
    total_nnz = sum(t.nnz for t in ts)
    print(f"[bench] generated {count} tensors, {total_nnz} nonzeros in {gen_s:.1f}s", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    hs = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R), stream=stream) for t in ts]
    build_s = time.perf_counter() - t0
    F = [[torch.from_numpy(f).cuda() for f in workloads.random_factors(t.dims, R, seed=i)] for i, t in enumerate(ts)]
    outs = [[torch.empty((d, R), device="cuda") for d in t.dims] for t in ts]
    # Launch shape (partitions per CU, workgroup size, gathers in flight):
    # measured by the shape autotuner unless the partition size is given.
    if args.parts_per_cu:
        capi.mttkrp_batch_autotune(hs, R, F, outs, candidates=[args.parts_per_cu], reps=1, stream=stream)
        info = capi.mttkrp_layout_info(hs[0])
        tuned = {"parts_per_cu": args.parts_per_cu, "wg_threads": info["wg_threads"],
                 "gathers_in_flight": info["gathers_in_flight"], "source": "--parts-per-cu"}
    else:
        t0 = time.perf_counter()
        best, times = capi.mttkrp_batch_autotune_shape(hs, R, F, outs, reps=3, stream=stream)
        info = capi.mttkrp_layout_info(hs[0])
        ms = sorted(times.values())
        dflt = times.get(default_shape(3, R))
        tuned = {"parts_per_cu": best[0], "wg_threads": info["wg_threads"],
                 "gathers_in_flight": info["gathers_in_flight"], "source": "mttkrp_batch_autotune_shape",
                 "candidates": len(times),
                 "spread_ms_per_pass": {"fastest": round(ms[0], 4), "median": round(ms[len(ms) // 2], 4),
                                        "slowest": round(ms[-1], 4),
                                        "default_shape": round(dflt, 4) if dflt else None},
                 "candidate_ms_per_pass": {f"{p}/{th or 'def'}/{g or 'def'}": round(v, 4)
                                           for (p, th, g), v in times.items()},
                 "tuning_s": round(time.perf_counter() - t0, 2)}
    print(f"[bench] launch shape {tuned}", file=sys.stderr, flush=True)
    b = capi.mttkrp_batch_create(hs, R)

    def batched(st=stream):
        for n in range(3):
            capi.mttkrp_batch_run(b, n, F, [o[n] for o in outs], stream=st)

    def plain(st=stream):
        for n in range(3):
            for i, h in enumerate(hs):
                capi.mttkrp_run(h, n, F[i], outs[i][n], R, stream=st)

    def timed(fn, K, W):
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(K):
            fn()
        z.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(z) / K

    def graphed(fn, K):
        fn()                              # eager first: uploads the descriptors for these pointers
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            fn(None)
        gr.replay()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(K):
            gr.replay()
        z.record(stream)
        torch.cuda.synchronize()
        del gr
        return a.elapsed_time(z) / K

    ms_b_eager = timed(batched, args.steps, args.warmup)
    ms_p_eager = timed(plain, max(3, args.steps // 4), 1)
    ms_b = graphed(batched, args.steps)
    ms_p = graphed(plain, max(3, args.steps // 4))

    # 20 CP-ALS sweeps of every tensor: batched sweeps captured once in a HIP
    # graph and replayed, against plain per-tensor sweeps launched eagerly.
    als_iters = 20
    Fa = [[f.clone() for f in fs] for fs in F]
    lam = [torch.zeros(R, dtype=torch.float64, device="cuda") for _ in ts]
    fit = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in ts]
    F0 = [[f.clone() for f in fs] for fs in F]

    def reset():
        for fs, f0 in zip(Fa, F0):
            for f, g in zip(fs, f0):
                f.copy_(g)
        for i, h in enumerate(hs):
            capi.cpd_als_init(h, Fa[i], R, stream=stream)

    reset()
    capi.cpd_als_batch_iter_async(b, Fa, lam, fit, stream=stream)   # uploads the descriptors for these pointers
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):   # captured on torch's capture stream (the current stream inside)
        for _ in range(als_iters):
            capi.cpd_als_batch_iter_async(b, Fa, lam, fit)
    reset()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    z = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    g.replay()
    z.record(stream)
    torch.cuda.synchronize()
    for h in hs:
        capi.cpd_als_status(h, stream=stream)
    ms_graph = a.elapsed_time(z)
    fits_graph = [float(f.item()) for f in fit]
    reset()
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(als_iters):
        for i, h in enumerate(hs):
            capi.cpd_als_iter_async(h, Fa[i], lam[i], R, fit[i], stream=stream)
    z.record(stream)
    torch.cuda.synchronize()
    for h in hs:
        capi.cpd_als_status(h, stream=stream)
    ms_plain_als = a.elapsed_time(z)
    same = all(float(f.item()) == fg for f, fg in zip(fit, fits_graph))
    del g

    # The same batch on copies with 32-bit coordinates (wide_indices=1) and the
    # same launch shape: what the 16-bit coordinates are worth here.
    info0 = capi.mttkrp_layout_info(hs[0])
    shape_opts = dict(max_R=R, wide_indices=1, parts_per_cu=info0["parts_per_cu"], part_threads=info0["wg_threads"],
                      part_gathers=info0["gathers_in_flight"])
    hw = [capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=shape_opts, stream=stream) for t in ts]
    bw = capi.mttkrp_batch_create(hw, R)

    def batched_wide(st=stream):
        for n in range(3):
            capi.mttkrp_batch_run(bw, n, F, [o[n] for o in outs], stream=st)

    ms_wide = graphed(batched_wide, args.steps)
    bw.free()
    for h in hw:
        h.free()
    idx16 = sum(capi.mttkrp_layout_info(h)["idx16_modes"] == 0b111 for h in hs)

    flops = sum(3 * R * t.nnz * 3 for t in ts)
    byts = sum(sum(algorithmic_bytes(t.dims, t.nnz, R, idx16_modes=capi.mttkrp_layout_info(h)["idx16_modes"]))
               for t, h in zip(ts, hs))
    res = {
        "metric": "batched all-mode spMTTKRP (tensors x all modes per second)",
        "value": round(count / (ms_b / 1e3), 1),
        "unit": "tensor-all-modes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_b, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch256-R16: {count} 3-mode tensors, dims U[100,5000], nnz log-U[1e3,1e6] "
                               f"(capped), uniform distinct, R={R}; one step = all modes of every tensor",
                   "total_nnz": total_nnz, "R": R},
        "launch_shape": tuned,
        "timing": "one step = 3 modes; both methods replayed from a HIP graph of one step",
        "plain_ms_per_step": round(ms_p, 4),
        "batched_speedup_vs_plain": round(ms_p / ms_b, 3),
        "coords_16bit": {"tensors_with_16bit_copies": idx16, "ms_per_step_with_32bit_coords": round(ms_wide, 4),
                         "speedup": round(ms_wide / ms_b, 3)},
        "eager_launch_ms_per_step": {"batched": round(ms_b_eager, 4), "plain": round(ms_p_eager, 4)},
        "gflops": round(flops / (ms_b / 1e3) / 1e9, 1),
        "hbm_pct_peak": round(100.0 * byts / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS, 2),
        "als_20_sweeps": {"batched_graph_ms": round(ms_graph, 3), "plain_eager_ms": round(ms_plain_als, 3),
                          "speedup": round(ms_plain_als / ms_graph, 3),
                          "tensor_sweeps_per_s": round(count * als_iters / (ms_graph / 1e3), 1),
                          "fits_bitwise_equal": same},
        "build_s": round(build_s, 2),
    }
    b.free()
    for h in hs:
        h.free()
    return res


def bench_precision(args):
    """FP32 factors against BF16 factor copies (FP32 products and sums) on the
    4-mode 50000 x 40000 x 30000 x 2000, 100M-nonzero Zipf(1.1) tensor with
    lognormal values: all-mode MTTKRP time at R=32 and R=64 for both factor
    types, beside the gather probe's time.  The errors of both against the
    FP64 oracle are measured in tests/test_gpu_precision.py."""
    import torch

    import workloads
    from paper_2503_18198_amd import capi

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t = workloads.named_tensor("zipf1.1-100M-4mode", progress=log)
    N = len(t.dims)
    log(f"generated {t.dims} nnz={t.nnz}")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=64, relabel=int(args.relabel)), stream=stream)
    build_s = time.perf_counter() - t0
    log(f"layout built in {build_s:.1f}s")
    K, W = args.steps, args.warmup

    def per_mode_ms(fn):
        ev = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(N)]
        tot = [0.0] * N
        for rep in range(W + K):
            for n in range(N):
                ev[n][0].record(stream)
                fn(n)
                ev[n][1].record(stream)
            torch.cuda.synchronize()
            if rep >= W:
                for n in range(N):
                    tot[n] += ev[n][0].elapsed_time(ev[n][1])
        return [x / K for x in tot]

    by = {}
    for R in (32, 64):
        F = workloads.random_factors(t.dims, R, seed=3)
        d32 = [torch.from_numpy(f).cuda() for f in F]
        d16 = [f.to(torch.bfloat16) for f in d32]
        outs = [torch.empty((d, R), device="cuda") for d in t.dims]
        for name, dF, run, fb in (("fp32", d32, capi.mttkrp_run, 4), ("bf16", d16, capi.mttkrp_run_bf16, 2)):
            ms = per_mode_ms(lambda n: run(h, n, dF, outs[n], R, stream=stream))
            probe = per_mode_ms(lambda n: capi.mttkrp_gather_probe(h, n, dF, R, 1, stream=stream))
            byts = algorithmic_bytes(t.dims, t.nnz, R, factor_bytes=fb,
                                     idx16_modes=capi.mttkrp_layout_info(h)["idx16_modes"])
            flops = N * R * t.nnz * N
            by[f"{name}_R{R}"] = {
                "ms_all_modes": round(sum(ms), 4), "per_mode_ms": [round(x, 4) for x in ms],
                "gflops": round(flops / (sum(ms) / 1e3) / 1e9, 1),
                "hbm_frac": round(sum(byts) / (sum(ms) / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "gather_probe_ms_all_modes": round(sum(probe), 4),
            }
            log(f"R={R} {name}: {sum(ms):.3f} ms all modes")
    h.free()
    main = by["fp32_R32"]
    res = {
        "metric": "all-mode spMTTKRP GFLOP/s, FP32 factors vs BF16 factor copies",
        "value": main["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": main["ms_all_modes"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "precision-100M-4mode: 4-mode 50000x40000x30000x2000, 100M distinct nonzeros "
                               "(Zipf(1.1)), lognormal(0,1) values, R in {32,64}, FP32 vs BF16 factor rows"
                               + (", indices renumbered by degree" if args.relabel else ""),
                   "nnz": t.nnz, "dims": list(t.dims)},
        "by_dtype_and_R": by,
        "build_s": round(build_s, 2),
    }
    print(json.dumps(res))
    return 0


def bench_paper_shapes(args, R=32):
    """The paper's load-balancing ablation (Sec. V-B, Fig. 4) on synthetic
    tensors with the shapes and nonzero counts of its evaluation set (Table
    III), at kappa = one partition per compute unit.  Per mode, three
    partitioners on the same kernel: the library's nonzero split with the
    deterministic carry fix-up ("nonzero_split"); scheme 2 (equal nonzero chunks, global
    atomics for rows cut by chunk boundaries); scheme 1 (whole rows dealt to
    kappa partitions by LPT).  All-mode totals for scheme 1 only, scheme 2
    only, the paper's adaptive choice (scheme 1 where I_n >= kappa, else
    scheme 2) and the nonzero split.  Returns the result line as a dict."""
    import torch

    import workloads
    from paper_2503_18198_amd import capi

    stream = torch.cuda.current_stream()
    K, W = args.steps, args.warmup
    shapes = dict(PAPER_SHAPES)
    if not args.skip_large_shape:
        shapes.update(PAPER_SHAPE_LARGE)
    if args.only_shapes:
        every = {**PAPER_SHAPES, **PAPER_SHAPE_LARGE}
        unknown = [n for n in args.only_shapes if n not in every]
        if unknown:
            raise SystemExit(f"unknown shape(s) {unknown}; known: {sorted(every)}")
        shapes = {n: every[n] for n in args.only_shapes}
    rows = {}
    for name, (dims, nnz) in shapes.items():
        t0 = time.perf_counter()
        t = workloads.random_tensor(dims, nnz, dist="zipf", s=1.2, seed=7,
                                    progress=lambda m: print(f"[bench] {name}: {m}", file=sys.stderr, flush=True))
        gen_s = time.perf_counter() - t0
        N = len(t.dims)
        # 32-bit coordinates in every column (scheme-1 copies have no 16-bit
        # form), so that only the partitioning differs.
        h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, wide_indices=1), stream=stream)
        kappa = capi.mttkrp_layout_info(h)["cu_count"]
        t1 = time.perf_counter()
        h1 = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(max_R=R, partitioner=capi.MTTKRP_PART_ROWS_LPT,
                                                                      lpt_parts=kappa), stream=stream)
        lpt_build_s = time.perf_counter() - t1
        dF = [torch.from_numpy(f).cuda() for f in workloads.random_factors(t.dims, R, seed=7)]
        # Scheme 1's balance per mode: LPT's largest partition load over the
        # mean, and the heaviest row's share of the nonzeros.
        lpt_ratio, heavy_pct = [], []
        for n in range(N):
            loads = np.bincount(t.idx[:, n].astype(np.int64), minlength=dims[n]).astype(np.uint64)
            _, pl = capi.mttkrp_lpt_partition(loads, kappa)
            lpt_ratio.append(round(float(pl.max()) / (float(pl.sum()) / kappa), 2))
            heavy_pct.append(round(100.0 * float(loads.max()) / max(t.nnz, 1), 2))
        del t
        out = {k: [torch.empty((d, R), device="cuda") for d in dims] for k in ("nnz", "s2", "s1")}

        def per_mode(run, hh, o):
            ev = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(N)]
            tot = [0.0] * N
            for rep in range(W + K):
                for n in range(N):
                    ev[n][0].record(stream)
                    run(hh, n, dF, o[n], R, stream=stream)
                    ev[n][1].record(stream)
                torch.cuda.synchronize()
                if rep >= W:
                    for n in range(N):
                        tot[n] += ev[n][0].elapsed_time(ev[n][1])
            return [x / K for x in tot]

        ms = {"nonzero_split": per_mode(capi.mttkrp_run, h, out["nnz"]),
              "scheme2_atomics": per_mode(capi.mttkrp_run_scheme2, h, out["s2"]),
              "scheme1_lpt": per_mode(capi.mttkrp_run, h1, out["s1"])}
        adaptive = [ms["scheme1_lpt"][n] if dims[n] >= kappa else ms["scheme2_atomics"][n] for n in range(N)]

        def rel(a, b):
            return max(float(torch.linalg.norm(a[n] - b[n]) / max(float(torch.linalg.norm(b[n])), 1e-30))
                       for n in range(N))

        byts = sum(algorithmic_bytes(dims, nnz, R))
        flops = N * R * nnz * N
        tot = {k: sum(v) for k, v in ms.items()}
        tot["adaptive_paper"] = sum(adaptive)
        rows[name] = {
            "dims": list(dims), "nnz": int(nnz), "gen_s": round(gen_s, 1), "lpt_build_s": round(lpt_build_s, 2),
            "ms_per_mode": {k: [round(x, 4) for x in v] for k, v in ms.items()},
            "lpt_load_max_over_mean": lpt_ratio, "heaviest_row_pct": heavy_pct,
            "adaptive_choice": ["scheme1" if dims[n] >= kappa else "scheme2" for n in range(N)],
            "ms_all_modes": {k: round(v, 4) for k, v in tot.items()},
            "speedup_vs_adaptive": {k: round(tot["adaptive_paper"] / v, 3) for k, v in tot.items()},
            "gflops_nonzero_split": round(flops / (tot["nonzero_split"] / 1e3) / 1e9, 1),
            "hbm_frac_nonzero_split": round(byts / (tot["nonzero_split"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "max_rel_diff_vs_nonzero_split": {"scheme2_atomics": rel(out["s2"], out["nnz"]),
                                           "scheme1_lpt": rel(out["s1"], out["nnz"])},
        }
        print(f"[bench] {name}: {json.dumps(rows[name])}", file=sys.stderr, flush=True)
        h.free()
        h1.free()
        del dF, out
        torch.cuda.empty_cache()

    def gm(key):
        return round(float(np.exp(np.mean([np.log(r["ms_all_modes"]["adaptive_paper"] / r["ms_all_modes"][key])
                                           for r in rows.values()]))), 3)

    res = {
        "metric": "all-mode spMTTKRP GFLOP/s on tensors shaped like the paper's evaluation set",
        "value": round(float(np.exp(np.mean([np.log(r["gflops_nonzero_split"]) for r in rows.values()]))), 1),
        "unit": "GFLOP/s (geometric mean)", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(sum(r["ms_all_modes"]["nonzero_split"] for r in rows.values()), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "paper-shapes: Zipf(1.2) stand-ins with the shapes and nnz of the paper's Table III "
                               f"tensors, R={R}, fp32, kappa = {kappa} partitions for scheme 1"},
        "tensors": rows,
        "speedup_vs_adaptive_geomean": {k: gm(k) for k in ("nonzero_split", "scheme2_atomics", "scheme1_lpt",
                                                           "adaptive_paper")},
    }
    return res


def fiber_stats(t, R, shapes=((32, 256), (8, 512)), cus=256, L=4):
    """How much factor-row reuse over fibers the mode copies offer (an
    analysis on the host; no GPU).  In the mode-n copy, sorted by i_n and then
    cyclically by the other indices, a fiber is a run of nonzeros sharing
    (i_n, i_(n+1)); every nonzero of a fiber gathers the same row of the
    next factor.  Per mode:
    * fibers, their mean length and their nonzero-weighted mean length;
    * `whole_wave_skip`: on the partition kernel's layout (each lane group
      takes a run of gsz consecutive nonzeros, 64 / lanes-per-row groups per
      wave), the fraction of wave steps at which no group starts a fiber, so
      that the wave could skip the (n+1) gather instruction; gsz follows the
      library's partition geometry for the given (partitions per CU, workgroup
      threads) shapes;
    * `split_gathers_per_nnz`: row gathers per nonzero if each fiber's
      nonzeros were dealt into segments of L sharing one (n+1) row, the
      remainder kept as single nonzeros, against N - 1 today."""
    idx = t.idx
    nnz, N = idx.shape
    lanes = max(1, R * 4 // 16)
    G = 64 // lanes
    out = {"groups_per_wave": G, "segment_nonzeros": L, "modes": []}
    for n in range(N):
        m = (n + 1) % N
        key = np.sort(idx[:, n].astype(np.int64) * int(t.dims[m]) + idx[:, m])
        start = np.ones(nnz, dtype=bool)
        start[1:] = key[1:] != key[:-1]
        lens = np.diff(np.append(np.flatnonzero(start), nnz))
        segs = int((lens // L).sum())
        gathers = (nnz - segs * L) * (N - 1) + segs * (1 + L * (N - 2))
        skip = {}
        for ppc, threads in shapes:
            groups = threads // lanes
            per = -(-nnz // (ppc * cus * groups))
            gsz = max(32, -(-per // 32) * 32)
            W = nnz // (G * gsz)       # whole waves
            frac = None
            if W:
                f = start[: W * G * gsz].reshape(W, G, gsz).copy()
                f[:, :, 0] = True
                frac = round(float(1.0 - f.any(axis=1).mean()), 4)
            skip[f"{ppc}/{threads}"] = {"gsz": gsz, "fraction": frac}
        out["modes"].append({"fibers": int(len(lens)), "mean_len": round(nnz / len(lens), 2),
                             "nnz_weighted_mean_len": round(float((lens.astype(np.float64) ** 2).sum() / nnz), 1),
                             "whole_wave_skip": skip,
                             "split_gathers_per_nnz": round(gathers / nnz, 3)})
    return out


def _serve_tensor(spec):
    t = spec.tensor()
    return t.idx, t.val, t.dims, t.nnz


def serve_jobs(args):
    """The serving workload's jobs, generated in forked worker processes; call
    before this process touches the GPU."""
    import concurrent.futures
    import multiprocessing

    import workloads
    from paper_2503_18198_amd.serve import ServeJob

    n_warm, n_timed = args.serve_warmup_jobs, args.serve_jobs
    n_jobs = n_warm + n_timed
    specs = workloads.job_stream(n_jobs, rate_per_s=1.0, nnz_range=(1e4, 1e7))
    # generated in forked workers before this process touches the GPU
    t0 = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("fork")) as pool:
        tensors = []
        for i, tt in enumerate(pool.map(_serve_tensor, specs, chunksize=1)):
            tensors.append(tt)
            if (i + 1) % 20 == 0:
                print(f"[bench] generated {i + 1} of {n_jobs} jobs ({time.perf_counter() - t0:.0f}s)",
                      file=sys.stderr, flush=True)
    base = [ServeJob(job_id=sp.job_id, arrival_s=sp.arrival_s, dims=dims, R=sp.R, idx=idx, val=val, nnz=nnz,
                     seed=sp.job_id, max_iters=50, tol=1e-4) for sp, (idx, val, dims, nnz) in zip(specs, tensors)]
    nnzs = np.array([j.nnz for j in base])
    print(f"[bench] generated {n_jobs} jobs, {nnzs.sum() / 1e6:.0f}M nonzeros, in {time.perf_counter() - t0:.1f}s "
          f"on {workers} processes", file=sys.stderr, flush=True)
    return base


def bench_serve(args, base, rhos=(0.5, 0.8, 0.95, 2.0), slot_list=None):
    """Poisson CP-ALS jobs (3-5 modes, dims log-U[1e2,1e5], nnz log-U[1e4,1e7],
    Zipf(1.2), R in {16,32,64}, fit change < 1e-4 or 50 sweeps) served with
    continuous batching, against the plain method (one job at a time, FIFO),
    at offered loads of rho x the plain method's measured capacity.  The
    first jobs of the stream are warm-up: they run but are not counted.
    Returns the result line as a dict."""
    import torch

    from paper_2503_18198_amd.serve import CpdServer, GpuExecutor, ServeJob

    n_warm, n_timed = args.serve_warmup_jobs, args.serve_jobs
    n_jobs = n_warm + n_timed
    slot_list = list(slot_list or args.serve_slots)
    nnzs = np.array([j.nnz for j in base])
    torch.cuda.set_device(0)

    def clone(js, scale):
        return [ServeJob(job_id=j.job_id, arrival_s=j.arrival_s * scale, dims=j.dims, R=j.R, idx=j.idx, val=j.val,
                         nnz=j.nnz, seed=j.seed, max_iters=j.max_iters, tol=j.tol) for j in js]

    def timed_metrics(srv, js):
        t = [j for j in js if j.job_id >= n_warm]
        span = max(j.finished_s for j in t) - min(j.arrival_s for j in t)
        m = srv.metrics(t, span)
        m["admit_s_total"] = srv.admit_s
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in m.items()}

    def progress(what):
        count = [0]

        def retired(job):
            count[0] += 1
            if count[0] % 50 == 0:
                print(f"[bench] {what}: {count[0]} jobs done", file=sys.stderr, flush=True)
        return retired

    def serve(js, batched, slots, build_threads):
        srv = CpdServer(GpuExecutor(batched=batched, wide_indices=args.wide_indices), budget, max_slots=slots, build_threads=build_threads,
                        on_retire=progress(f"{slots} slot(s)"))
        srv.run(js)
        return timed_metrics(srv, js)

    budget = int(args.serve_budget_gib * (1 << 30))
    # warm-up (allocations, first launches), then the plain method's capacity:
    # every job present at time 0, one at a time
    CpdServer(GpuExecutor(batched=True, wide_indices=args.wide_indices), budget, max_slots=64, build_threads=args.serve_build_threads).run(
        clone(base[:8], 0.0))
    t0 = time.perf_counter()
    cap_jobs = clone(base, 0.0)
    cap_srv = CpdServer(GpuExecutor(batched=False, wide_indices=args.wide_indices), budget, max_slots=1, on_retire=progress("capacity"))
    cap_srv.run(cap_jobs)
    mean_service = max(j.finished_s for j in cap_jobs) / n_jobs
    print(f"[bench] plain capacity {1.0 / mean_service:.2f} jobs/s ({time.perf_counter() - t0:.0f}s, "
          f"{cap_srv.admit_s:.1f}s of it in layout builds)", file=sys.stderr, flush=True)
    mean_gap = float(np.mean(np.diff([0.0] + [j.arrival_s for j in base])))
    loads = {}
    for rho in rhos:
        scale = mean_service / rho / mean_gap      # arrival times scaled to rho x plain capacity
        plain = serve(clone(base, scale), False, 1, 0)
        loads[str(rho)] = {"plain_fifo": plain}
        print(f"[bench] rho {rho}: plain {plain['jobs_per_s']:.2f} jobs/s p50 {plain['p50_latency_s']:.3f}s "
              f"p99 {plain['p99_latency_s']:.3f}s", file=sys.stderr, flush=True)
        for slots in slot_list:
            served = serve(clone(base, scale), True, slots, args.serve_build_threads)
            loads[str(rho)][f"continuous_batching_{slots}_slots"] = served
            print(f"[bench] rho {rho}: {slots} slots {served['jobs_per_s']:.2f} jobs/s "
                  f"p50 {served['p50_latency_s']:.3f}s p99 {served['p99_latency_s']:.3f}s",
                  file=sys.stderr, flush=True)
    top = loads[str(max(rhos))][f"continuous_batching_{slot_list[0]}_slots"]
    res = {
        "metric": "served CP-ALS jobs/s with p50/p99 latency (continuous batching vs one job at a time)",
        "value": top["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1, "steps": top["steps"],
        "warmup": n_warm, "ms_per_step": round(1e3 / top["jobs_per_s"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serve-poisson: {n_warm} warm-up + {n_timed} timed Poisson CP-ALS jobs, 3-5 modes, "
                               f"dims log-U[1e2,1e5], nnz log-U[1e4,1e7] ({nnzs.sum() / 1e6:.0f}M in all), "
                               f"Zipf(1.2), R in {{16,32,64}}, stop at |dfit|<1e-4 or 50 sweeps, offered load "
                               f"rho x plain capacity for rho in {list(rhos)}, HBM budget {args.serve_budget_gib:g} GiB, slots "
                               f"{slot_list}, {args.serve_build_threads} layout-build threads, "
                               f"{'32-bit coordinates' if args.wide_indices else '16-bit coordinates where dims fit'}; value = "
                               f"served jobs/s at the highest load with {slot_list[0]} slots; "
                               f"ms_per_step = ms per served job"},
        "by_offered_load": loads,
        "plain_capacity_jobs_per_s": round(1.0 / mean_service, 3),
    }
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-side-workloads", action="store_true",
                    help="default workload only: leave out the batch and serve sub-objects")
    ap.add_argument("--parts-per-cu", type=int, default=0)
    ap.add_argument("--shape", default="",
                    help="fixed launch shape PPC,THREADS,GATHERS of the nonzero-ordered copies (no tuning)")
    ap.add_argument("--relabel", action="store_true",
                    help="renumber each mode's indices by decreasing nonzero count before building "
                         "(the default and precision workloads' nonzero-ordered copies)")
    ap.add_argument("--wide-indices", action="store_true",
                    help="serve-poisson: build every job's copies with 32-bit coordinates")
    ap.add_argument("--no-tune-shape", action="store_true",
                    help="time the library's default launch shape instead of the autotuned one")
    ap.add_argument("--kernel", choices=("steps", "nonzero"), default="nonzero",
                    help="layout timed for the MTTKRP: nonzero-ordered copies or hot-steps copies (3- and 4-mode)")
    ap.add_argument("--no-compare-layouts", action="store_true",
                    help="time only the chosen layout (no second layout beside it)")
    ap.add_argument("--hot-rows", type=int, default=0, help="rows per input factor cached in LDS (-1: as many as fit)")
    ap.add_argument("--als-iters", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true", help="accepted for compatibility; parity lives in tests/")
    ap.add_argument("--no-gather-ceiling", action="store_true")
    ap.add_argument("--skip-large-shape", action="store_true",
                    help="paper-shapes: leave out the 143.6M-nonzero tensor")
    ap.add_argument("--only-shapes", nargs="+", default=None,
                    help="paper-shapes: run only these tensors (e.g. nell1-like)")
    ap.add_argument("--serve-slots", type=int, nargs="+", default=[8, 4],
                    help="concurrent job slots of the continuous-batching server (serve-poisson)")
    ap.add_argument("--serve-jobs", type=int, default=200, help="timed jobs of serve-poisson")
    ap.add_argument("--serve-warmup-jobs", type=int, default=20, help="warm-up jobs ahead of them")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0,
                    help="device memory the serving loop may admit jobs into (serve-poisson)")
    ap.add_argument("--serve-build-threads", type=int, default=4,
                    help="worker threads for layout builds in the continuous-batching server")
    ap.add_argument("--fiber-stats", action="store_true",
                    help="only print, for the workload's tensor, how much factor-row reuse over fibers its "
                         "mode copies offer (host analysis, no GPU)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB, 5 times (to calibrate "
                         "the HBM byte counters against a kernel of known traffic)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs on one device "
              "(the design notes describe how the path would shard).", file=sys.stderr)
        return 2

    if args.fiber_stats:
        import workloads

        wl = WORKLOADS[args.workload]
        if not wl["tensor"]:
            raise SystemExit("--fiber-stats needs a single-tensor workload")
        t = workloads.named_tensor(wl["tensor"])
        print(json.dumps({"workload": args.workload, "fiber_stats": fiber_stats(t, wl["R"])}))
        return 0

    import torch

    import workloads
    from paper_2503_18198_amd import capi

    if args.workload == "serve-poisson":
        print(json.dumps(bench_serve(args, serve_jobs(args))))   # jobs generated before the GPU is touched
        return 0
    side = args.workload == DEFAULT_WORKLOAD and not args.no_side_workloads
    jobs = serve_jobs(args) if side else None
    torch.cuda.set_device(0)
    if args.workload == "batch256-R16":
        print(json.dumps(bench_batch(args)))
        return 0
    if args.workload == "precision-100M-4mode":
        return bench_precision(args)
    if args.workload == "paper-shapes":
        print(json.dumps(bench_paper_shapes(args)))
        return 0
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * 2 ** 20 // 4
        a = torch.rand(n, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "launches": 5}))
        return 0
    wl = WORKLOADS[args.workload]
    R = wl["R"]
    t_gen = time.perf_counter()
    t = workloads.named_tensor(wl["tensor"])
    F = workloads.random_factors(t.dims, R, seed=workloads.WORKLOADS[wl["tensor"]]["seed"])
    gen_s = time.perf_counter() - t_gen
    N = len(t.dims)
    print(f"[bench] generated {t.dims} nnz={t.nnz} in {gen_s:.1f}s", file=sys.stderr, flush=True)

    # The timed layout: nonzero-ordered copies (the library default) unless
    # --kernel steps.  The other layout of a 3- or 4-mode tensor is timed
    # beside it on the same factors; the gather-ceiling probe runs on the
    # nonzero-ordered copies.
    steps = args.kernel == "steps" and N in (3, 4)
    other = N in (3, 4) and not args.no_compare_layouts
    opts0 = dict(max_R=R, hot_rows=args.hot_rows, relabel=int(args.relabel))
    if args.parts_per_cu:
        opts0["parts_per_cu"] = args.parts_per_cu
    opts1 = dict(max_R=R, hot_steps=1, parts_per_cu=args.parts_per_cu or 2)
    stream = torch.cuda.current_stream()
    t_b = time.perf_counter()
    h = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=opts1 if steps else opts0, stream=stream)
    build_s = time.perf_counter() - t_b
    print(f"[bench] layout built in {build_s:.1f}s ({capi.mttkrp_layout_bytes(h) / 2**30:.2f} GiB)",
          file=sys.stderr, flush=True)
    t_b = time.perf_counter()
    h_other = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=opts0 if steps else opts1,
                                       stream=stream) if other else None
    other_build_s = time.perf_counter() - t_b
    h0 = h_other if steps else h      # nonzero-ordered copies (None: not built)
    dF = [torch.from_numpy(f).cuda() for f in F]
    outs = [torch.empty((d, R), dtype=torch.float32, device="cuda") for d in t.dims]

    # Launch shape of the nonzero-ordered copies (partitions per CU, and for
    # 3-mode tensors the workgroup size and gathers in flight): measured by
    # the library's shape autotuner over its default candidates, unless fixed.
    launch_shape = None
    if not steps and not args.no_tune_shape:
        t_t = time.perf_counter()
        if args.shape:
            cands = [tuple(int(x) for x in args.shape.split(","))]
        elif args.parts_per_cu:
            cands = sorted({(args.parts_per_cu, th, g) for _, th, g in capi.mttkrp_batch_autotune_default_shapes(N)})
        else:
            cands = None
        best, times = capi.mttkrp_autotune_shape(h, R, dF, outs, candidates=cands, reps=3, stream=stream)
        info = capi.mttkrp_layout_info(h)
        ms = sorted(times.values())
        dflt = times.get(default_shape(N, R))
        launch_shape = {"parts_per_cu": best[0], "wg_threads": info["wg_threads"],
                        "gathers_in_flight": info["gathers_in_flight"],
                        "source": "--shape" if args.shape else "mttkrp_autotune_shape",
                        "candidates": len(times),
                        "all_mode_ms": {"chosen": round(times[best], 4), "fastest": round(ms[0], 4),
                                        "median": round(ms[len(ms) // 2], 4), "slowest": round(ms[-1], 4),
                                        "default_shape": round(dflt, 4) if dflt else None},
                        "tuning_s": round(time.perf_counter() - t_t, 2)}
        print(f"[bench] launch shape {launch_shape}", file=sys.stderr, flush=True)

    def all_modes(ev=None, hh=None):
        for n in range(N):
            if ev is not None:
                ev[n][0].record(stream)
            capi.mttkrp_run(hh or h, n, dF, outs[n], R, stream=stream)
            if ev is not None:
                ev[n][1].record(stream)

    for _ in range(args.warmup):
        all_modes()
    torch.cuda.synchronize()
    K = args.steps
    events = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(N)]
              for _ in range(K)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(K):
        all_modes(events[k])
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_step = total_ms / K
    mode_ms = [float(np.mean([events[k][n][0].elapsed_time(events[k][n][1]) for k in range(K)])) for n in range(N)]
    step_ms = [events[k][0][0].elapsed_time(events[k][N - 1][1]) for k in range(K)]

    # The other layout on the same factors, for comparison.
    mode_ms_other = None
    if other:
        for _ in range(args.warmup):
            all_modes(hh=h_other)
        ev0 = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(N)]
               for _ in range(K)]
        torch.cuda.synchronize()
        for k in range(K):
            all_modes(ev0[k], hh=h_other)
        torch.cuda.synchronize()
        mode_ms_other = [float(np.mean([ev0[k][n][0].elapsed_time(ev0[k][n][1]) for k in range(K)])) for n in range(N)]
    mode_ms0 = mode_ms_other if steps else mode_ms

    flops = N * R * t.nnz * N
    gflops = flops / (ms_step / 1e3) / 1e9
    bytes_mode = algorithmic_bytes(t.dims, t.nnz, R, idx16_modes=capi.mttkrp_layout_info(h)["idx16_modes"])
    traffic = profiled_traffic(args.workload)
    achieved = sum(bytes_mode) / (sum(mode_ms) / 1e3) / 1e9
    result = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N}-mode {'x'.join(map(str, t.dims))}, {t.nnz} distinct nonzeros "
                               f"({'Zipf(%s)' % workloads.WORKLOADS[wl['tensor']]['s'] if workloads.WORKLOADS[wl['tensor']]['dist'] == 'zipf' else 'uniform'}), "
                               f"R={R}, fp32 factors, all-mode MTTKRP per step",
                   "nnz": t.nnz, "dims": list(t.dims), "R": R},
        "hbm_pct_peak": round(100.0 * sum(bytes_mode) / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 2),
        "per_mode_ms": [round(x, 4) for x in mode_ms],
        "step_ms_median": round(float(np.median(step_ms)), 4),
        "step_ms_min": round(float(np.min(step_ms)), 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic[0] if traffic else None,
                     "traffic_launch_shape": traffic[1] if traffic else None,
                     "kernel": ("per-mode MTTKRP launches (mttkrp_step_kernel on hot-steps copies + "
                                "mttkrp_fixup_kernel)" if steps else
                                "per-mode MTTKRP launches (mttkrp_part_kernel + its mttkrp_fixup_kernel launches)") +
                               ": algorithmic bytes per mode / HIP-event time of the mode's launches, averaged over "
                               "modes",
                     "algorithmic_bytes_per_launch": round(sum(bytes_mode) / N),
                     "bytes_per_mode": bytes_mode},
        "build_s": round(build_s, 2),
        "launch": capi.mttkrp_layout_info(h),
        "launch_shape": launch_shape,
        "layout": ("hot-steps copies (rows ordered by hot/cold input rows, padded to wave steps; built on the host)"
                   if steps else "nonzero-ordered copies" + (", indices renumbered by degree" if args.relabel else "")),
    }
    if other:
        result["nonzero_order_copies" if steps else "hot_steps_copies"] = {
            "per_mode_ms": [round(x, 4) for x in mode_ms_other], "all_mode_ms": round(sum(mode_ms_other), 4),
            "build_s": round(other_build_s, 2), "launch": capi.mttkrp_layout_info(h_other),
            "what": ("the same MTTKRP on the nonzero-ordered copies (mttkrp_part_kernel)" if steps else
                     "the same MTTKRP on hot-steps copies (mttkrp_step_kernel; hot_steps=1, 2 partitions per CU): "
                     "rows ordered by hot/cold input rows and padded to wave steps, hot rows read from LDS") +
                    ", same factors and steps"}

    # On-chip ceilings of this index pattern: the same partitions' stream
    # loads alone, and with every factor-row gather, without the arithmetic.
    if not args.no_gather_ceiling and h0 is not None:
        def probe_ms(what):
            ev = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(N)]
            tot = [0.0] * N
            for rep in range(K + 1):
                for n in range(N):
                    ev[n][0].record(stream)
                    capi.mttkrp_gather_probe(h0, n, dF, R, what, stream=stream)
                    ev[n][1].record(stream)
                torch.cuda.synchronize()
                if rep:
                    for n in range(N):
                        tot[n] += ev[n][0].elapsed_time(ev[n][1])
            return [x / K for x in tot]
        stream_ms = probe_ms(0)
        gather_ms = probe_ms(1)
        one_lane_ms = probe_ms(2)
        l1_ms = probe_ms(3)
        gbytes = [t.nnz * (N - 1) * R * 4 for _ in range(N)]
        result["gather_ceiling"] = {
            "stream_only_ms_per_mode": [round(x, 4) for x in stream_ms],
            "stream_and_gathers_ms_per_mode": [round(x, 4) for x in gather_ms],
            "gathered_bytes_per_mode": gbytes[0],
            "gathered_TBps_in_probe": round(sum(gbytes) / (sum(gather_ms) / 1e3) / 1e12, 2),
            "gathered_TBps_in_mttkrp": round(sum(gbytes) / (sum(mode_ms0) / 1e3) / 1e12, 2),
            "mttkrp_time_over_probe_time": round(sum(mode_ms0) / sum(gather_ms), 3),
            "same_gathers_one_lane_per_row_ms_per_mode": [round(x, 4) for x in one_lane_ms],
            "same_gathers_l1_resident_rows_ms_per_mode": [round(x, 4) for x in l1_ms],
            "what": "mttkrp_gather_probe on the nonzero-ordered copies (default launch shape): their MTTKRP's "
                    "stream loads and factor-row gathers on the same partitions and lanes, arithmetic and stores "
                    "replaced by an XOR fold; the same gather instructions with one lane of each row's group "
                    "reading (1/L of the bytes), and with every row L1-resident (row index & 63)",
        }

    # CP-ALS sweeps (MTTKRP plus the FP64 update), timed separately.
    if args.als_iters > 0:
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
        Fa = [f.clone() for f in dF]
        capi.cpd_als_init(h, Fa, R, stream=stream)
        capi.cpd_als_iter(h, Fa, lam, R, fit, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.als_iters):
            capi.cpd_als_iter_async(h, Fa, lam, R, fit, stream=stream)
        z.record(stream)
        torch.cuda.synchronize()
        capi.cpd_als_status(h)
        result["als"] = {"ms_per_iter": round(a.elapsed_time(z) / args.als_iters, 3),
                         "iters": args.als_iters, "fit_last": float(fit.item())}


    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(t, R, F)
    h.free()
    if h_other is not None:
        h_other.free()
    del dF, outs
    if side:
        # The second half of the metric: batched requests/s and served p50/p99
        # latency, on the batching and serving workloads, as sub-objects.
        result["batch"] = _sub(bench_batch(args), ("metric", "value", "unit", "ms_per_step", "config",
                                                   "launch_shape", "plain_ms_per_step", "batched_speedup_vs_plain", "coords_16bit",
                                                   "eager_launch_ms_per_step", "gflops", "hbm_pct_peak",
                                                   "als_20_sweeps", "build_s"))
        torch.cuda.empty_cache()
        sv = bench_serve(args, jobs, rhos=(0.95, 2.0), slot_list=args.serve_slots[:1])
        result["serve"] = _sub(sv, ("metric", "value", "unit", "config", "plain_capacity_jobs_per_s",
                                    "by_offered_load"))
    print(json.dumps(result))
    return 0


def _sub(d, keys):
    return {k: d[k] for k in keys if k in d}


if __name__ == "__main__":
    sys.exit(main())
