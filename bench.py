#!/usr/bin/env python3
"""Benchmark of reproducible GroupBy-SUM (repro<T,L>) on one MI355X.

Workload (low-cardinality scan): 200M rows, int32 keys uniform over 1024
groups, a float64 and a float32 value column with exponent spread
2^U(-60,60) and exact cancellation pairs, both summed into repro<double,3>.
One step = initialise two state buffers, GroupBy-SUM of each column, and
finalise both (the whole path), with inputs resident in HBM.

Prints ONE JSON line: throughput (rows/s), the roofline of the dominant
kernel (the aggregation pass over the float64 column, timed with HIP events
on its stream), the non-reproducible FP64-atomic baseline on the same
columns, and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_agg_cols_lowcard_200M_g1024_L3.md")
# the sources that define the low-cardinality aggregation kernel, hashed in this order
KERNEL_SOURCES = ("repro_cols.hip", "repro_lds.hpp", "repro_agg.hpp", "repro_device.hpp")


def measured_traffic():
    """HBM bytes per launch of the aggregation kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the kernel sources
    changed since those counters were taken."""
    import hashlib

    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("kernel_source_sha256", "traffic_")))
    csrc = os.path.join(ROOT, "paper_1802_09883_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in KERNEL_SOURCES)).hexdigest()
    if vals.get("kernel_source_sha256") != h or "traffic_bytes_per_launch" not in vals:
        return None
    return int(vals["traffic_bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


CONFIGS = {
    # name: rows, groups, levels, key dtype, value columns, generator
    "lowcard": dict(rows=200_000_000, groups=1024, L=3, desc="lowcard scan: {n} rows, int32 keys U[0,{G}), "
                    "f64 + f32 columns 2^U(-60,60) with exact cancellation pairs, repro<double,{L}>"),
    "highcard": dict(rows=100_000_000, groups=1 << 22, L=2, desc="highcard skewed: {n} rows, int64 keys Zipf(1) "
                     "over {G} groups, f64 +-lognormal(0,4), repro<double,{L}>, partitioned"),
    "plain": dict(rows=1_000_000, groups=16, L=2, desc="plain GroupBy-SUM: {n} rows, int32 keys U[0,{G}), "
                  "f64 N(0,1)*2^U(-20,20), repro<double,{L}>"),
    "serve": dict(rows=0, groups=0, L=2, desc="served: {q} GroupBy queries (Poisson arrivals at 70% of capacity), "
                  "4 SUM aggregates over 6 decimal-like f64 columns (SUM c0, SUM c1, SUM c2*c3, SUM c4*c5), rows "
                  "log-uniform 1e4..5e7 ({n} in all), groups log-uniform 4..2^20, int32 keys, repro<double,2>, "
                  "{slots} slots, memory-admitted"),
    "float": dict(rows=200_000_000, groups=1024, L=2, desc="float accumulators: {n} rows, int32 keys U[0,{G}), "
                  "f32 column 2^U(-60,60) with exact cancellation pairs, repro<float,{L}>"),
    "sum": dict(rows=200_000_000, groups=1, L=3, desc="ungrouped sum: {n} f64 values 2^U(-60,60) with exact "
                "cancellation pairs (the lowcard f64 column), repro<double,{L}>"),
    "batched": dict(rows=0, groups=0, L=0, desc="batched: {jobs} independent GroupBy-SUM jobs in one persistent "
                    "launch (graph-replayed), rows log-uniform 1e3..1e7 ({n} in all), groups log-uniform 1..2^16, "
                    "int32 keys, f64 N(0,1)*2^U(-30,30), repro<double,L>, L in {{2,3}}, autotuned"),
}


def make_columns(workloads, name, n, G):
    if name == "lowcard":
        keys, v64, v32 = workloads.lowcard(n=n, groups=G)
        return keys, [("f64", v64), ("f32", v32)]
    if name == "highcard":
        keys, v = workloads.highcard(n=n, groups=G)
        return keys, [("f64", v)]
    if name == "float":
        keys, _, v32 = workloads.lowcard(n=n, groups=G)
        return keys, [("f32", v32)]
    keys, v = workloads.plain(n=n, groups=G)
    return keys, [("f64", v)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", choices=sorted(CONFIGS), default="lowcard")
    ap.add_argument("--rows", type=int, default=0, help="override the config's row count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-column", action="store_true",
                    help="aggregate the columns of a multi-column workload in separate calls (one key pass each)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (HBM counter calibration)")
    ap.add_argument("--stream-ceiling", action="store_true",
                    help="only measure the read-stream ceiling: a plain read kernel over the low-cardinality "
                         "workload's bytes, swept over launch shapes")
    ap.add_argument("--atomic-ceiling", action="store_true",
                    help="only measure global 64-bit atomic adds: uniform indices over the 64 MiB of level words "
                         "of the high-cardinality workload, and that workload's Zipf keys")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.stream_ceiling:
        return stream_ceiling(args)
    if args.atomic_ceiling:
        return atomic_ceiling(args)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              "(sharding over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.config == "batched":
        return bench_batched(args)
    if args.config == "serve":
        return bench_serve(args)
    if args.config == "sum":
        return bench_sum(args)

    import torch

    from paper_1802_09883_amd import api, workloads

    cfg = CONFIGS[args.config]
    n = args.rows or cfg["rows"]
    G, L = cfg["groups"], cfg["L"]
    log(f"generating {args.config} workload n={n} G={G}")
    t0 = time.time()
    keys, cols = make_columns(workloads, args.config, n, G)
    log(f"generated in {time.time() - t0:.1f}s; copying to the GPU")
    dev = torch.device("cuda:0")
    kt = torch.from_numpy(keys).to(dev)
    vts = [(name, torch.from_numpy(v).to(dev)) for name, v in cols]
    T = torch.float32 if args.config == "float" else torch.float64
    states = [api.state_init(G, L, T, dev) for _ in vts]
    outs = [torch.empty(G, dtype=T, device=dev) for _ in vts]
    wsb = max(api.workspace_bytes(n, G, kt.dtype, v.dtype, L, T) for _, v in vts)
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)

    fused = len(vts) > 1 and not args.per_column
    if fused:
        wsb = max(wsb, api.workspace_bytes_cols(n, G, kt.dtype, [v.dtype for _, v in vts], L, T))
        ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)

    def step():
        for st in states:
            api.state_reset(st, G, L, T)
        if fused:  # one key pass for every column
            api.groupby_sum_cols(kt, [v for _, v in vts], G, L, T, states=states, status=status, workspace=ws)
        else:
            for st, (_, v) in zip(states, vts):
                api.groupby_sum(kt, v, G, L, T, states=st, status=status, workspace=ws)
        for st, out in zip(states, outs):
            api.finalize(st, G, L, T, out=out)

    plains = [torch.zeros(G, dtype=torch.float64, device=dev) for _ in vts]

    def plain_step():
        for pl in plains:
            pl.zero_()
        if fused:
            api.plain_groupby_sum_cols(kt, [v for _, v in vts], G, outs=plains)
        else:
            for pl, (_, v) in zip(plains, vts):
                api.plain_groupby_sum(kt, v, G, out=pl)

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if int(status.item()) != 0:
        raise SystemExit(f"device status {int(status.item())} on a clean workload")

    log(f"timing {args.steps} steps")
    ncol = 1 if fused else len(vts)  # aggregation calls per step
    # measured launches per call: the partitioned path reports its scatter and its aggregation
    per_call = 2 if args.config == "highcard" else 1
    api.profile_arm(ncol * per_call * args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms = api.profile_read()
    ms_step = (t1 - t0) * 1000.0 / args.steps
    kcol = [kms[i::ncol * per_call] for i in range(ncol * per_call)]
    knames = (["+".join(name for name, _ in vts)] if fused else [name for name, _ in vts]) if per_call == 1 \
        else ["partition scatter", "partition aggregation"]
    log(f"step {ms_step:.3f} ms; aggregation kernel " +
        ", ".join(f"{name} {np.mean(k):.3f} ms" for name, k in zip(knames, kcol)))

    # inputs small enough to stay in the 256 MB Infinity Cache between steps,
    # and the partitioned path (whose states and partition buffers may stay in
    # it): also time single steps after streaming 1 GiB through the caches (cold)
    cold_ms = None
    in_bytes = kt.numel() * kt.element_size() + sum(v.numel() * v.element_size() for _, v in vts)
    if in_bytes < (512 << 20) or args.config == "highcard":
        flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        cold = []
        for _ in range(args.steps):
            flush.fill_(1.0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            step()
            e1.record()
            torch.cuda.synchronize()
            cold.append(e0.elapsed_time(e1))
        cold_ms = float(np.median(cold))
        del flush
        log(f"cold-cache step {cold_ms:.4f} ms (median of {args.steps})")

    for _ in range(args.warmup):
        plain_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    log(f"plain FP64 atomic step {plain_ms:.3f} ms")

    # algorithmic bytes: rows read once per column; states and outputs written once
    kb = keys.dtype.itemsize
    state_b = api.state_bytes(G, L, T)
    vsum = sum(v.element_size() for _, v in vts)
    if fused:  # the keys are read once for all columns
        alg_step = n * (kb + vsum) + len(vts) * (state_b + G * 8)
        alg_k0 = n * (kb + vsum)
    else:
        alg_step = sum(n * (kb + v.element_size()) + state_b + G * 8 for _, v in vts)
        alg_k0 = n * (kb + vts[0][1].element_size())
    k0 = float(np.mean(kcol[0]))
    ach_gbs = alg_k0 / (k0 * 1e-3) / 1e9
    kname = {"lowcard": "k_agg_lds<int32,f64,f64,L=3>", "plain": "k_agg_lds<int32,f64,f64,L=2>",
             "float": "k_agg_lds<int32,f32,f32,L=2>",
             "highcard": "k_agg_part<f64,f64,L=2> (after partitioning)"}[args.config]
    roofline = {"bound": "hbm", "achieved": round(ach_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach_gbs / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic() if fused and n == CONFIGS["lowcard"]["rows"] else None,
                "kernel": (f"k_agg_cols<int32,L={L},NC={len(vts)}> ({' + '.join(nm for nm, _ in vts)} columns, one "
                           f"key pass)") if fused else f"{kname} ({vts[0][0]} column)",
                "kernel_ms": round(k0, 4),
                "alg_bytes_per_launch": alg_k0}
    if args.config == "highcard":
        # the dominant kernel is the partition scatter: keys and values read
        # once, (local key, value) pairs written once
        vb = vts[0][1].element_size()
        sc_bytes = n * (kb + vb) + n * (2 + vb)
        sc_ms = float(np.mean(kcol[0]))
        ag_ms = float(np.mean(kcol[1]))
        sc_gbs = sc_bytes / (sc_ms * 1e-3) / 1e9
        roofline.update({"achieved": round(sc_gbs, 1), "frac": round(sc_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "k_part_scatter<int64,f64> (partition pass: key+value read, local key+value "
                                   "written)", "kernel_ms": round(sc_ms, 4), "alg_bytes_per_launch": sc_bytes,
                         "partition_aggregation": {"kernel": "k_agg_part<f64,f64,L=2>", "ms": round(ag_ms, 4),
                                                   "alg_bytes": n * (2 + vb),
                                                   "achieved": round(n * (2 + vb) / (ag_ms * 1e-3) / 1e9, 1)}})

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(keys, [v for _, v in cols], G, L, args.cpu_seconds, T64=(args.config != "float"))

    rows_per_s = n / (ms_step * 1e-3)
    rec = {
        "metric": "repro GroupBy-SUM rows/s",
        "value": rows_per_s,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.config == "float" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["desc"].format(n=n, G=G, L=L), "name": args.config, "rows": n, "groups": G,
                   "L": L, "columns": [name for name, _ in vts], "key_passes": 1 if fused else len(vts),
                   "parallelism": "single GPU"},
        "step_hbm_frac": round(alg_step / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "cold_cache_ms_per_step": round(cold_ms, 4) if cold_ms is not None else None,
        "plain_fp64_atomic": {"ms_per_step": round(plain_ms, 4), "slowdown": round(ms_step / plain_ms, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def bench_batched(args):
    """512 independent jobs per step: one graph replay of the batch launch
    (reset kernel + persistent kernel), states overwritten and finalised."""
    import torch

    from paper_1802_09883_amd import api, workloads

    rows, groups, Ls = workloads.batched_jobs()
    log(f"generating {len(rows)} jobs, {int(rows.sum())} rows")
    specs = [(*workloads.batched_job(int(r), int(g), j), int(g), int(l))
             for j, (r, g, l) in enumerate(zip(rows, groups, Ls))]
    dev = torch.device("cuda:0")
    jobs = [api.Job(torch.from_numpy(k).to(dev), torch.from_numpy(v).to(dev), G, L,
                    torch.empty(api.state_bytes(G, L), dtype=torch.uint8, device=dev),
                    torch.empty(G, dtype=torch.float64, device=dev)) for k, v, G, L in specs]
    n = int(rows.sum())
    log("autotuning")
    t0 = time.time()
    best, tuned_ms = api.batch_tune(jobs)
    log(f"tuned in {time.time() - t0:.1f}s: {best} {tuned_ms:.3f} ms")
    run = api.batch_prepare(jobs, config=best)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    api.batch_launch(run, status, stream=s)  # eager once (also warms up)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        api.batch_launch(run, status, stream=s)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    if int(status.item()) != 0:
        raise SystemExit(f"device status {int(status.item())} on a clean workload")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()  # replay() launches the graph on the current stream
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    ms_dev = e0.elapsed_time(e1) / args.steps
    log(f"step {ms_step:.3f} ms (device {ms_dev:.3f} ms)")
    # plain FP64 atomic baseline: one launch per job
    plains = [torch.zeros(j.num_groups, dtype=torch.float64, device=dev) for j in jobs]

    def plain_step():
        for pl, j in zip(plains, jobs):
            pl.zero_()
            api.plain_groupby_sum(j.keys, j.values, j.num_groups, out=pl)

    for _ in range(args.warmup):
        plain_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    log(f"plain FP64 atomic step {plain_ms:.3f} ms")
    alg = sum(len(k) * 12 + G * L * 16 + G * 8 for k, _, G, L in specs)
    ach = alg / (ms_dev * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batched(specs, args.cpu_seconds)
    rec = {
        "metric": "repro GroupBy-SUM rows/s", "value": n / (ms_step * 1e-3), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": CONFIGS["batched"]["desc"].format(jobs=len(jobs), n=n), "name": "batched",
                   "jobs": len(jobs), "rows": n, "tuned": best, "parallelism": "single GPU"},
        "step_hbm_frac": round(alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "plain_fp64_atomic": {"ms_per_step": round(plain_ms, 4), "slowdown": round(ms_step / plain_ms, 3),
                              "note": "one launch per job"},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_batch<int32,f64,f64> (persistent, with its reset kernel)",
                     "kernel_ms": round(ms_dev, 4), "alg_bytes_per_launch": alg},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def bench_sum(args):
    """Ungrouped reproducible sum: one step = reset the state, sum the column,
    finalise (the profile events bracket nothing here: HIP events on the
    stream around the whole step)."""
    import torch

    from paper_1802_09883_amd import api, workloads

    cfg = CONFIGS["sum"]
    n = args.rows or cfg["rows"]
    L = cfg["L"]
    _, v64, _ = workloads.lowcard(n=n, groups=1024, with_f32=False)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(v64).to(dev)
    st = api.state_init(1, L)
    out = torch.empty(1, dtype=torch.float64, device=dev)

    def step():
        api.state_reset(st, 1, L)
        api.sum(v, L, state=st)
        api.finalize(st, 1, L, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ms_dev = e0.elapsed_time(e1) / args.steps
    # baseline: torch's (non-reproducible) sum reduction, device time by HIP
    # events on the stream it runs on
    for _ in range(args.warmup):
        pl = torch.sum(v)
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record()
    for _ in range(args.steps):
        pl = torch.sum(v)
    p1.record()
    torch.cuda.synchronize()
    plain_ms = p0.elapsed_time(p1) / args.steps
    alg = n * 8
    ach = alg / (ms_dev * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(np.zeros(n, np.int32), [v64], 1, L, args.cpu_seconds)
    rec = {
        "metric": "repro GroupBy-SUM rows/s", "value": n / (ms * 1e-3), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["desc"].format(n=n, L=L), "name": "sum", "rows": n, "groups": 1, "L": L,
                   "parallelism": "single GPU"},
        "step_hbm_frac": round(ach / HBM_PEAK_GBS, 4),
        "plain_fp64_atomic": {"ms_per_step": round(plain_ms, 4), "slowdown": round(ms_dev / plain_ms, 3),
                              "note": "torch.sum (non-reproducible tree reduction) on the same column; both "
                                      "timed by HIP events on their stream"},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_sum<f64,f64,L=3> + k_sum_merge + state reset + finalize (whole step)",
                     "kernel_ms": round(ms_dev, 4), "alg_bytes_per_launch": alg},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def bench_serve(args):
    """A stream of GroupBy queries through the request loop: first all at
    once (capacity), then Poisson arrivals at 70% of that rate (latency)."""
    import torch

    from paper_1802_09883_amd import api, workloads

    Q = 128
    # defaults from a sweep of slots x workgroup cap x chunk rows on this
    # workload: 4 slots and 64M-row chunks gave the lowest p99 at 70% load
    slots = int(os.environ.get("REPRO_SERVE_SLOTS", "4"))
    max_bypass = int(os.environ.get("REPRO_SERVE_BYPASS", "8"))
    chunk_rows = int(os.environ.get("REPRO_SERVE_CHUNK", str(64 << 20)))
    rows, groups, gaps = workloads.served_queries(Q)
    n_all = int(rows.sum())
    log(f"generating {Q} queries, {n_all} rows")
    pool = workloads.decimal_columns(int(rows.max()), 6)
    dev = torch.device("cuda:0")
    pool_t = [torch.from_numpy(np.ascontiguousarray(c)).to(dev) for c in pool]
    rng = np.random.default_rng(7)
    offs = [int(rng.integers(0, int(rows.max()) - int(n) + 1)) for n in rows]
    specs = []
    for q, (n, G) in enumerate(zip(rows, groups)):
        gen = torch.Generator(device=dev)
        gen.manual_seed(1000 + q)
        keys = torch.randint(0, int(G), (int(n),), generator=gen, dtype=torch.int32, device=dev)
        specs.append(api.QuerySpec(keys, [c[offs[q]:offs[q] + int(n)] for c in pool_t], int(G),
                                   workloads.SERVED_AGGS, L=2))
    arena = 24 << 30

    qwg = int(os.environ.get("REPRO_QUERY_WG", "0"))  # persistent workgroups per query (0: all)

    def run(arrivals):
        srv = api.Server(arena, slots=slots, query_workgroups=qwg, max_bypass=max_bypass, chunk_rows=chunk_rows)
        try:
            t0 = srv.clock()
            arr = t0 + arrivals
            done, i = {}, 0
            while len(done) < Q:
                now = srv.clock()
                while i < Q and arr[i] <= now:
                    srv.submit(specs[i])
                    i += 1
                comp, _, _ = srv.poll()
                for t, tm in comp:
                    done[t] = tm
            torch.cuda.synchronize()
            ends = np.array([done[k] for k in range(Q)])
            return ends - arr, ends.max() - arr.min()
        finally:
            srv.close()

    def run_alone():
        """Each query on an idle server, one after another: its latency
        with nothing else on the device."""
        srv = api.Server(arena, slots=slots, query_workgroups=qwg, max_bypass=max_bypass, chunk_rows=chunk_rows)
        try:
            out = np.empty(Q)
            for i in range(Q):
                t0 = srv.clock()
                srv.submit(specs[i])
                comp = []
                while not comp:
                    comp, _, _ = srv.poll()
                out[i] = comp[0][1] - t0
            return out
        finally:
            srv.close()

    log("warm-up pass")
    run(np.zeros(Q))
    log("capacity: all queries at once")
    _, span_c = run(np.zeros(Q))
    rate = 0.7 * Q / span_c
    log(f"capacity {Q / span_c:.1f} queries/s ({n_all / span_c:.3e} rows/s); open loop at {rate:.1f} queries/s")
    lat, span_o = run(np.cumsum(gaps) / rate)
    p50, p99 = np.percentile(lat, 50) * 1e3, np.percentile(lat, 99) * 1e3
    log(f"latency p50 {p50:.3f} ms, p99 {p99:.3f} ms, span {span_o * 1e3:.2f} ms")
    alone = run_alone()
    a50, a99 = np.percentile(alone, 50) * 1e3, np.percentile(alone, 99) * 1e3
    slow = lat / alone
    log(f"alone: p50 {a50:.3f} ms, p99 {a99:.3f} ms; in-mix/alone p50 {np.percentile(slow, 50):.2f}, "
        f"p99 {np.percentile(slow, 99):.2f}")
    # plain FP64 atomic baseline: the same aggregates, one query after another
    outs = [torch.zeros(int(G), dtype=torch.float64, device=dev) for G in groups]
    prods = torch.empty(int(rows.max()), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, o in zip(specs, outs):
        n = s.keys.numel()
        for a, b in s.aggs:
            v = s.cols[a] if b is None else torch.mul(s.cols[a], s.cols[b], out=prods[:n])
            o.zero_()
            api.plain_groupby_sum(s.keys, v, s.num_groups, out=o)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    alg = int(sum(int(n) * 52 + 4 * int(G) * 8 for n, G in zip(rows, groups)))  # keys + 6 columns read, 4 outputs
    ach = alg / span_c / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_serve(pool, offs, rows, groups, args.cpu_seconds)
    rec = {
        "metric": "repro GroupBy-SUM rows/s", "value": n_all / span_c, "unit": "rows/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(span_c * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": CONFIGS["serve"]["desc"].format(q=Q, n=n_all, slots=slots), "name": "serve",
                   "queries": Q, "rows": n_all, "slots": slots, "max_bypass": max_bypass,
                   "query_workgroups": qwg, "chunk_rows": chunk_rows, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(p50, 4), "p99": round(p99, 4), "mean": round(float(np.mean(lat)) * 1e3, 4),
                       "offered_rate_qps": round(rate, 2), "open_loop_rows_per_s": n_all / span_o,
                       "alone_p50": round(a50, 4), "alone_p99": round(a99, 4),
                       "in_mix_over_alone_p50": round(float(np.percentile(slow, 50)), 3),
                       "in_mix_over_alone_p99": round(float(np.percentile(slow, 99)), 3),
                       "note": "alone: each query on an idle server, one after another; in_mix_over_alone: "
                               "per-query latency at the offered rate over its latency alone"},
        "step_hbm_frac": round(ach / HBM_PEAK_GBS, 4),
        "plain_fp64_atomic": {"ms_per_step": round(plain_s * 1e3, 4), "slowdown": round(span_c / plain_s, 3),
                              "note": "same aggregates, queries one after another"},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole request loop (capacity run): input columns read once per query",
                     "kernel_ms": round(span_c * 1e3, 4), "alg_bytes_per_launch": alg},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def cpu_baseline_serve(pool, offs, rows, groups, seconds):
    """The CPU oracle on whole queries (4 aggregates each, expression columns
    formed in numpy), in order, for about `seconds`, rows/s."""
    import torch

    from oracle import oracle
    from paper_1802_09883_amd import workloads

    cores, host = host_cpus()
    t0 = time.perf_counter()
    done, nq = 0, 0
    for q, (n, G) in enumerate(zip(rows, groups)):
        gen = torch.Generator(device="cuda:0")
        gen.manual_seed(1000 + q)
        keys = torch.randint(0, int(G), (int(n),), generator=gen, dtype=torch.int32, device="cuda:0").cpu().numpy()
        cols = [c[offs[q]:offs[q] + int(n)] for c in pool]
        for a, b in workloads.SERVED_AGGS:
            v = cols[a] if b is None else cols[a] * cols[b]
            st, _ = oracle.groupby_sum(keys, v, int(G), 2, True, threads=cores)
            oracle.finalize(st, int(G), 2)
        done += int(n)
        nq += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "rows/s", "cores": cores, "kind": "oracle", "host": host,
            "sample": f"first {nq} of {len(rows)} queries ({done} rows, 4 aggregates each), {cores} threads, "
                      f"{dt:.1f} s (key generation included)"}


def cpu_baseline_batched(specs, seconds):
    """The CPU oracle on the first jobs of the batch (whole jobs, in order)
    until about `seconds` of work, rows/s."""
    from oracle import oracle

    cores, host = host_cpus()
    t0 = time.perf_counter()
    done, njobs = 0, 0
    for k, v, G, L in specs:
        st, _ = oracle.groupby_sum(k, v, G, L, True, threads=cores)
        oracle.finalize(st, G, L)
        done += len(k)
        njobs += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "rows/s", "cores": cores, "kind": "oracle", "host": host,
            "sample": f"first {njobs} of {len(specs)} jobs ({done} rows), {cores} threads, {dt:.1f} s"}


def stream_ceiling(args):
    """Read-stream ceiling: repro_read_probe over 3.2e9 bytes (the keys and
    both value columns of the low-cardinality scan), each launch shape timed
    with HIP events over `steps` launches; prints one JSON line."""
    import ctypes

    import torch

    from paper_1802_09883_amd import _lib

    lib = _lib.load()
    nbytes = CONFIGS["lowcard"]["rows"] * 16
    dev = torch.device("cuda:0")
    buf = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    shapes = [(wg, th) for th in (256, 512, 1024) for wg in (256, 512, 1024, 2048, 4096)]
    res = []
    for wg, th in shapes:
        def launch():
            _lib.check(lib.repro_read_probe(ctypes.c_void_p(buf.data_ptr()), nbytes, wg, th,
                                            ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(stream.cuda_stream)),
                       "read_probe")
        for _ in range(args.warmup):
            launch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            launch()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res.append({"workgroups": wg, "threads": th, "ms": round(ms, 4), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1)})
        log(f"read probe {wg} x {th}: {ms:.4f} ms, {res[-1]['GB/s']} GB/s")
    best = max(res, key=lambda r: r["GB/s"])
    agg_shape = next(r for r in res if r["workgroups"] == 256 and r["threads"] == 1024)
    print(json.dumps({"metric": "read-stream ceiling", "bytes": nbytes, "steps": args.steps, "best": best,
                      "aggregation_launch_shape": agg_shape, "peak_GB/s": HBM_PEAK_GBS, "sweep": res}), flush=True)


def atomic_ceiling(args):
    """Global-atomic rate (repro_atomic_probe): 1e8 64-bit atomic adds with
    uniform indices over 2^23 words (the 64 MiB of int64 level words of
    2^22 groups at L = 2, which fit the Infinity Cache), then with the
    high-cardinality workload's Zipf(1) keys over 2^22 words.  Aggregating
    that workload's level units with global atomics needs L = 2 such adds
    per row (after a pass for the tops), so 2x the uniform time is a lower
    bound for it, to compare with the partitioned step."""
    import ctypes

    import torch

    from paper_1802_09883_amd import _lib, workloads

    lib = _lib.load()
    dev = torch.device("cuda:0")
    cfg = CONFIGS["highcard"]
    n, G = cfg["rows"], cfg["groups"]
    stream = torch.cuda.current_stream(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    uni = torch.randint(0, 2 * G, (n,), generator=gen, dtype=torch.int32, device=dev)
    keys, _ = workloads.highcard(n=n, groups=G)
    zipf = torch.from_numpy(keys.astype(np.int32)).to(dev)
    del keys
    table = torch.zeros(2 * G, dtype=torch.int64, device=dev)
    res = {}
    for name, idx, words in (("uniform_64MiB", uni, 2 * G), ("zipf_keys", zipf, G)):
        def launch():
            _lib.check(lib.repro_atomic_probe(ctypes.c_void_p(idx.data_ptr()), n, ctypes.c_void_p(table.data_ptr()),
                                              words, 4096, ctypes.c_void_p(stream.cuda_stream)), "atomic_probe")
        launch()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            launch()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"atomics": n, "ms": round(ms, 4), "G_atomics_per_s": round(n / (ms * 1e-3) / 1e9, 2)}
        log(f"{name}: {n} atomics in {ms:.3f} ms ({res[name]['G_atomics_per_s']} G/s)")
    total = int(table.sum().item())
    if total != n * (1 + reps) * 2:
        raise SystemExit(f"atomic probe lost adds: {total} != {n * (1 + reps) * 2}")
    print(json.dumps({"metric": "global-atomic ceiling", "workgroups": 4096, "threads": 256, **res,
                      "level_adds_per_row": 2,
                      "atomic_groupby_lower_bound_ms": {"uniform": round(2 * res["uniform_64MiB"]["ms"], 3),
                                                        "zipf_keys": round(2 * res["zipf_keys"]["ms"], 3)}}),
          flush=True)


def copy_calibration(nbytes):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
    calibrate the HBM-traffic counters (bytes read = bytes written = nbytes)."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 3}), flush=True)


def host_cpus():
    """Threads for the CPU baseline and a description of the host: every CPU
    this process may run on (its affinity set), capped by OMP_NUM_THREADS
    when the environment sets it (the job's share of a shared host)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = max(1, min(avail, cap) if cap > 0 else avail)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return threads, {"nproc": os.cpu_count(), "affinity": avail, "omp_num_threads": cap or None, "model": model}


def cpu_baseline(keys, cols, G, L, seconds, T64=True):
    """The CPU oracle (threaded over row chunks, then merged) on a bounded
    prefix of the same rows, every column, finalised: rows/s."""
    from oracle import oracle

    cores, host = host_cpus()

    def run(m):
        t0 = time.perf_counter()
        for v in cols:
            st, _ = oracle.groupby_sum(keys[:m], v[:m], G, L, T64, threads=cores)
            oracle.finalize(st, G, L, T64)
        return time.perf_counter() - t0

    probe = min(len(keys), 2_000_000)
    dt = run(probe)
    m = int(min(len(keys), max(probe, probe * seconds / max(dt, 1e-6))))
    # when every row takes less than `seconds`, whole passes are repeated
    reps = max(1, int(round(seconds / max(dt * m / probe, 1e-6)))) if m == len(keys) else 1
    log(f"cpu oracle probe {probe} rows in {dt:.2f}s; timing {reps} x {m} rows on {cores} threads")
    t0 = time.perf_counter()
    for _ in range(reps):
        run(m)
    dt = time.perf_counter() - t0
    rate = reps * m / dt
    # beside it, on a prefix of about a second's work: the oracle on one
    # thread, and a plain (non-reproducible) FP64 GroupBy-SUM on one thread
    # (numpy bincount with weights), both over every column
    # (at least 1e6 rows: each oracle call also initialises every group's state)
    m1 = int(min(len(keys), max(10 ** 6, rate / max(cores, 1))))
    t0 = time.perf_counter()
    for v in cols:
        st, _ = oracle.groupby_sum(keys[:m1], v[:m1], G, L, T64, threads=1)
        oracle.finalize(st, G, L, T64)
    one = m1 / (time.perf_counter() - t0)
    k1 = keys[:m1].astype(np.int64)
    t0 = time.perf_counter()
    for v in cols:
        np.bincount(k1, weights=v[:m1].astype(np.float64), minlength=G)
    plain1 = m1 / (time.perf_counter() - t0)
    log(f"cpu oracle {rate:.3e} rows/s on {cores} threads, {one:.3e} on one; plain FP64 {plain1:.3e} on one")
    return {"value": rate, "unit": "rows/s", "cores": cores, "kind": "oracle", "host": host,
            "sample": f"{reps} pass(es) over the first {m} rows (of {len(keys)}) of all {len(cols)} column(s), "
                      f"{cores} threads, {dt:.1f} s",
            "ns_per_row_per_core": round(cores * 1e9 / rate, 2),
            "one_thread": {"oracle_rows_per_s": one, "plain_fp64_rows_per_s": plain1,
                           "oracle_over_plain": round(plain1 / one, 2), "rows": m1,
                           "plain": "numpy bincount with float64 weights"}}


if __name__ == "__main__":
    main()
