#!/usr/bin/env python3
"""Benchmark of the gfx950 LSD radix sort.

Default workload: one step sorts 2^26 (32-bit key, 32-bit value) pairs
(value = input index) once on each of the six input distributions (uniform,
gaussian, zero, sorted, reverse, bucket; MT19937 seed 1), inputs resident in
HBM before timing starts, out-of-place so every step sorts the same input.
Reported: whole-job Mkeys/s, the HBM roofline of the dominant kernel (the
digit pass) measured with HIP events on the library's launch stream, and the
CPU oracle's rate on a bounded sample.  The same line carries the rest of
the metric: the whole-sort fraction without the all-zero input, the
measured copy ceiling, 2^25 64-bit keys (own roofline), and the batched
segmented sort of 20,000 segments against one sort call per segment (both
timed with HIP events, eager and replayed from graphs).

Other workloads (``--workload``): u64_keys / u64_pairs (2^25 64-bit),
u32_keys_small (2^20 32-bit keys), segmented, serving, grid, and merge (the
stable merge sort on the same inputs, ``--merge-kind``).  Prints ONE JSON
line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    # name: (n, key bits, has values, description)
    "u32_pairs": (1 << 26, 32, True, "2^26 u32 key + u32 value pairs (value = input index)"),
    "u64_keys": (1 << 25, 64, False, "2^25 u64 keys, full 64-bit range"),
    "u64_pairs": (1 << 25, 64, True, "2^25 u64 key + u64 value pairs (value = input index)"),
    "u32_keys_small": (1 << 20, 32, False, "2^20 u32 keys (latency-bound, cache-resident)"),
}
COPY_CALIB_BYTES = 1 << 30  # plain copy used to calibrate the HBM byte counters


ROOT = os.path.dirname(os.path.abspath(__file__))
# the sources the digit-pass kernel is compiled from: counter readings taken
# on other sources are stale
KERNEL_SOURCES = ("paper_1511_03404_amd/csrc/rs_kernels.h", "paper_1511_03404_amd/csrc/rs_device.h")
MERGE_SOURCES = ("paper_1511_03404_amd/csrc/rs_merge.h", "paper_1511_03404_amd/csrc/rs_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def pass_kernel_name(bits, has_v, cfg):
    """The digit-pass kernel's name as rocprofv3 prints it (without arguments)."""
    t = "unsigned int" if bits == 32 else "unsigned long"
    return (f"void rs::k_pass<{t}, {t}, {'true' if has_v else 'false'}, "
            f"rs::PassCfg<{cfg['radix_bits']}, {cfg['threads']}, {cfg['items']}> >")


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, cfg):
    """HBM bytes per launch of the workload's dominant kernel from the
    committed counter summary, or None if it is missing, was taken on a
    different kernel source or on another configuration."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if workload.startswith("merge_"):
        w = t.get("merge", {}).get(workload)
        if w is None or w.get("source_sha256_16") != kernel_source_hash(MERGE_SOURCES):
            return None
        return w.get("traffic_bytes_per_launch")
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    w = t.get("workloads", {}).get(workload)
    if w is None or w.get("config") != cfg:
        return None
    return w.get("traffic_bytes_per_launch")


def summarize_pmc(root):
    """Turn rocprofv3 --pmc runs into the per-launch traffic summary.

    Expects <root>/<workload>/{FETCH_SIZE,WRITE_SIZE}/run_counter_collection.csv
    for the workloads, and <root>/copy/{FETCH_SIZE,WRITE_SIZE}/... for the
    1 GiB plain copy (bench.py --workload copy_calib) that scales each
    counter to bytes."""
    import csv

    def mean(path, prefix):
        v = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
             if r["Kernel_Name"].startswith(prefix)]
        return (sum(v) / len(v), len(v)) if v else (None, 0)

    cf, _ = mean(os.path.join(root, "copy", "FETCH_SIZE", "run_counter_collection.csv"),
                 "__amd_rocclr_copyBuffer")
    cw, _ = mean(os.path.join(root, "copy", "WRITE_SIZE", "run_counter_collection.csv"),
                 "__amd_rocclr_copyBuffer")
    fs, ws = COPY_CALIB_BYTES / (cf * 1024), COPY_CALIB_BYTES / (cw * 1024)
    out = {"kernel_source_sha256_16": kernel_source_hash(),
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
           "calibration": f"1 GiB plain copy (torch copy_, runtime blit kernel): FETCH_SIZE "
                          f"{cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB",
           "workloads": {}}
    import paper_1511_03404_amd as rs
    ctx = rs.Context(0)  # host-side only: the built-in configuration per size class
    for w, (n, bits, has_v, _) in WORKLOADS.items():
        # the counter runs skip the tuner: the built-in configuration of this size
        cfg = rs.configs(bits, has_v)[ctx.tune_get(bits, has_v, False, rs.size_class(n))]
        k = pass_kernel_name(bits, has_v, cfg)
        fp = os.path.join(root, w, "FETCH_SIZE", "run_counter_collection.csv")
        wp = os.path.join(root, w, "WRITE_SIZE", "run_counter_collection.csv")
        if not (os.path.exists(fp) and os.path.exists(wp)):
            continue
        f, nf = mean(fp, k)
        wr, _ = mean(wp, k)
        out["workloads"][w] = {"kernel": k, "config": cfg, "fetch_kib_per_launch": round(f, 1),
                               "write_kib_per_launch": round(wr, 1),
                               "traffic_bytes_per_launch": int(f * 1024 * fs + wr * 1024 * ws),
                               "launches_sampled": nf}
    # the merge pass, per merge kind measured (bench.py --workload merge)
    for w, (_, bits, has_v, _) in WORKLOADS.items():
        t = "unsigned int" if bits == 32 else "unsigned long"
        k = (f"void rs::k_merge_pass<{t}, {t}, {'true' if has_v else 'false'}, "
             f"{'512, 4' if bits == 64 else '256, 8'}, 1>")
        fp = os.path.join(root, "merge_" + w, "FETCH_SIZE", "run_counter_collection.csv")
        wp = os.path.join(root, "merge_" + w, "WRITE_SIZE", "run_counter_collection.csv")
        if not (os.path.exists(fp) and os.path.exists(wp)):
            continue
        f, nf = mean(fp, k)
        wr, _ = mean(wp, k)
        out.setdefault("merge", {})["merge_" + w] = {
            "kernel": k, "source_sha256_16": kernel_source_hash(MERGE_SOURCES),
            "fetch_kib_per_launch": round(f, 1), "write_kib_per_launch": round(wr, 1),
            "traffic_bytes_per_launch": int(f * 1024 * fs + wr * 1024 * ws),
            "launches_sampled": nf}
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="u32_pairs",
                    choices=sorted(WORKLOADS) + ["copy_calib", "segmented", "serving", "grid",
                                                 "merge"])
    ap.add_argument("--dists", default="all",
                    help="comma list of distributions, or 'all' for the six")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: leave out the copy ceiling, the 64-bit keys and the "
                         "segmented batch that the line carries beside the headline")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner: use the default configuration (index 0)")
    ap.add_argument("--cpu-sample-log2", type=int, default=26,
                    help="cpu_baseline: log2 of the elements the oracle sorts per distribution")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="print the traffic summary of rocprofv3 --pmc runs under DIR and exit")
    ap.add_argument("--segments", type=int, default=20000,
                    help="segmented workload: number of segments")
    ap.add_argument("--seg-log2", default="4,20",
                    help="segmented workload: log2 of the smallest and largest segment size")
    ap.add_argument("--seg-dist", default="uniform", choices=["uniform", "bucket", "zero"],
                    help="segmented workload: key distribution (bucket: the same draws mapped "
                         "through a table of 64 distinct values by their top 6 bits)")
    ap.add_argument("--tiny-cap", type=int, default=-1,
                    help="segmented workload: segments of 2..cap elements go to the bitonic "
                         "network (0: to the radix block sort; -1: the library default)")
    ap.add_argument("--per-segment-steps", type=int, default=1,
                    help="segmented workload: timed steps of the one-sort-per-segment form "
                         "(0 skips it)")
    ap.add_argument("--requests", type=int, default=100000,
                    help="serving workload: number of requests per load level")
    ap.add_argument("--slots", type=int, default=4, help="serving workload: streams")
    ap.add_argument("--merge-kind", default="u32_pairs", choices=sorted(WORKLOADS),
                    help="merge workload: the kind and size of the radix workload of that name")
    ap.add_argument("--grid-max-log2", type=int, default=25,
                    help="grid workload: largest log2 size (64-bit kinds stop one lower)")
    ap.add_argument("--grid-min-log2", type=int, default=15,
                    help="grid workload: smallest log2 size")
    ap.add_argument("--grid-tune", action="store_true",
                    help="grid workload: autotune each kind and size class before timing it")
    ap.add_argument("--grid-graph", action="store_true",
                    help="grid workload: also time each point replayed from a captured HIP graph")
    ap.add_argument("--grid-oracle-max-log2", type=int, default=22,
                    help="grid workload: time the oracle up to this log2 size (speedup column)")
    return ap.parse_args()


def bench_serving(args, torch, rs, datagen, dev):
    """Serving loop: Poisson arrivals of sort requests (sizes log-uniform in
    [2^10, 2^24], half 32-bit and half 64-bit keys, half with values), device
    buffers capped at 64 GB, continuous batching on several streams.  The
    saturation rate R_max comes from a closed-loop run (all requests queued
    at once); open-loop runs at 0.5 and 0.9 R_max report p50/p99 latency."""
    from paper_1511_03404_amd.serving import HipBackend, Request, Scheduler, serve, summarize
    lo, hi = 10, 24
    # inputs resident in HBM: request keys are slices of a random pool, values
    # slices of an index ramp (value = index within the request)
    pool = torch.from_numpy(datagen.MT19937(1).u64((1 << hi) + (1 << 22))).to(dev)
    idx = torch.arange(1 << hi, dtype=torch.int64, device=dev)
    ramp = {32: idx.to(torch.uint32), 64: idx.to(torch.uint64)}

    def requests(rate):
        out = []
        for q in datagen.requests(args.requests, rate_per_s=rate, lo_log2=lo, hi_log2=hi, seed=1):
            n, bits = q["n"], q["bits"]
            src = pool.view(torch.uint32) if bits == 32 else pool
            off = q["key_seed"] % (src.numel() - n)
            vals = ramp[bits][:n] if q["has_values"] else None
            out.append(Request(q["id"], n, bits, q["has_values"], q["arrival_s"],
                               payload=(src[off:off + n], vals)))
        return out

    def run(reqs, open_loop):
        be = HipBackend(slots=args.slots, keep_results=False)
        # admission: each batch's real device bytes (staging, output, the
        # library's workspace) under 64 GB or the free device memory
        sch = Scheduler(be, mem_cap=be.admission_cap(64 << 30), slots=args.slots,
                        max_batch_elems=1 << 25, batch_bytes=be.batch_bytes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        be.mark_clock_zero(0.0)
        def report(now, submitted, finished):
            print(f"  t={now:.1f}s submitted {submitted} finished {finished} "
                  f"in flight {len(sch.inflight)}", file=sys.stderr, flush=True)

        done = serve(sch, reqs, lambda: time.perf_counter() - t0, open_loop=open_loop,
                     progress=report)
        torch.cuda.synchronize()
        makespan = max(r.done_s for r in done)
        st = summarize(done, makespan)
        st.update({"failed": len(sch.failed), "rejected": len(sch.rejected),
                   "peak_inflight_batches": sch.peak_inflight,
                   "peak_admitted_GB": round(sch.peak_mem / 1e9, 2),
                   "admission_cap_GB": round(sch.mem_cap / 1e9, 2)})
        return st

    # warm-up on a few requests, then the closed loop for R_max
    print(f"serving {args.requests} requests per load level", file=sys.stderr, flush=True)
    run(requests(1e6)[:64], open_loop=False)
    print("warm-up done; closed loop", file=sys.stderr, flush=True)
    closed = run(requests(1e6), open_loop=False)
    r_max = closed["requests"] / closed["makespan_s"]
    print(f"closed loop: {closed}", file=sys.stderr, flush=True)
    levels = {}
    for frac in (0.5, 0.9):
        levels[str(frac)] = run(requests(frac * r_max), open_loop=True)
        levels[str(frac)]["rate_req_s"] = round(frac * r_max, 1)
        print(f"open loop {frac} R_max: {levels[str(frac)]}", file=sys.stderr, flush=True)
    main = levels["0.9"]
    out = {
        "metric": "Mkeys/s and p50/p99 latency, serving loop with continuous batching",
        "value": main["Mkeys_s"], "unit": "Mkeys/s",
        "n_gpus": 1, "steps": args.requests, "warmup": 64,
        "ms_per_step": round(main["makespan_s"] * 1e3 / max(1, main["requests"]), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32+u64", "data": "synthetic",
        "config": {"workload": f"{args.requests} Poisson-arriving sort requests, n = "
                               f"floor(2^({lo}+{hi - lo}u)), half u32 / half u64 keys, half "
                               f"key-value; admission by each batch's device bytes under "
                               f"min(64 GB, free HBM - 2 GiB); {args.slots} streams; "
                               f"rate 0.9 R_max", "requests": args.requests},
        "r_max_req_s": round(r_max, 1),
        "closed_loop": closed,
        "open_loop": levels,
    }
    print(json.dumps(out), flush=True)


def bench_grid(args, torch, rs, datagen, dev):
    """The paper's measurement grid (Section 3): every kind (32/64-bit keys,
    with and without values) x the six distributions x n = 2^15 .. 2^25
    (2^24 for 64-bit keys) and the 2^k + 2^(k-1) lengths between them.
    Each point is the mean time of `steps` sorts after `warmup`, inputs
    resident in HBM, out-of-place; the oracle's rate on the same input gives
    the speedup up to --grid-oracle-max-log2."""
    import oracle
    sizes = []
    for k in range(args.grid_min_log2, args.grid_max_log2 + 1):
        sizes.append(1 << k)
        if k < args.grid_max_log2:
            sizes.append((1 << k) + (1 << (k - 1)))
    ctx = rs.context(0)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    points = []
    for bits, has_v in ((32, False), (32, True), (64, False), (64, True)):
        kind = f"u{bits}_{'pairs' if has_v else 'keys'}"
        limit = args.grid_max_log2 - (1 if bits == 64 else 0)
        for n in sizes:
            if n > (1 << limit):
                continue
            tuned = None
            if args.grid_tune:
                from paper_1511_03404_amd import tune
                tuned = tune.tune_sort(bits, has_v, n, ctx=ctx, reps=5, warmup=1)["index"]
            ws = torch.empty(ctx.workspace_bytes(bits, has_v, n), dtype=torch.uint8, device=dev)
            for d in datagen.DISTRIBUTIONS:
                kh = datagen.keys(d, n, bits, seed=1)
                vh = datagen.values(n, bits) if has_v else None
                k = torch.from_numpy(kh).to(dev)
                v = torch.from_numpy(vh).to(dev) if has_v else None
                ko = torch.empty_like(k)
                vo = torch.empty_like(k) if has_v else None

                def go():
                    if has_v:
                        rs.sort_pairs(k, v, ko, vo, ctx=ctx, workspace=ws)
                    else:
                        rs.sort_keys(k, ko, ctx=ctx, workspace=ws)
                for _ in range(args.warmup):
                    go()
                ev0.record()
                for _ in range(args.steps):
                    go()
                ev1.record()
                ev1.synchronize()
                ms = ev0.elapsed_time(ev1) / args.steps
                pt = {"kind": kind, "dist": d, "n": n, "ms": round(ms, 5),
                      "Mkeys_s": round(n / ms / 1e3, 1),
                      "config": ctx.tune_get(bits, has_v, False, rs.size_class(n))}
                if args.grid_graph:
                    # the same sort captured once and replayed: the launches
                    # are submitted together, so small sizes lose their host
                    # launch gaps
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g):
                        go()
                    g.replay()
                    ev0.record()
                    for _ in range(args.steps):
                        g.replay()
                    ev1.record()
                    ev1.synchronize()
                    gms = ev0.elapsed_time(ev1) / args.steps
                    pt["graph_ms"] = round(gms, 5)
                    pt["graph_Mkeys_s"] = round(n / gms / 1e3, 1)
                    del g
                if n <= (1 << args.grid_oracle_max_log2):
                    t0 = time.perf_counter()
                    oracle.sort(kh, vh)
                    cpu = time.perf_counter() - t0
                    pt["oracle_Mkeys_s"] = round(n / cpu / 1e6, 2)
                    pt["speedup"] = round(cpu * 1e3 / ms, 1)
                points.append(pt)
            print(f"{kind} n={n} done", file=sys.stderr, flush=True)
    big = [p for p in points if p["kind"] == "u32_pairs" and p["n"] == (1 << args.grid_max_log2)]
    out = {
        "metric": "Mkeys/s over the paper's grid of kinds, distributions and sizes",
        "value": round(sum(p["Mkeys_s"] for p in big) / max(1, len(big)), 1),
        "unit": "Mkeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32+u64", "data": "synthetic",
        "config": {"workload": "grid: u32/u64 keys and pairs x 6 distributions x n = 2^15.."
                               f"2^{args.grid_max_log2} and 2^k+2^(k-1); value = mean over the six "
                               f"distributions of u32 pairs at 2^{args.grid_max_log2}",
                   "sizes": sizes, "graph_replay": bool(args.grid_graph),
                   "tuned_per_size": bool(args.grid_tune)},
        "oracle_cores": 1,
        "points": points,
    }
    print(json.dumps(out), flush=True)


def bench_segmented(args, torch, rs, datagen, dev):
    print(json.dumps(measure_segmented(args, torch, rs, datagen, dev,
                                       with_cpu=not args.no_cpu_baseline)), flush=True)


def measure_segmented(args, torch, rs, datagen, dev, with_cpu=True, quick=False):
    """Batched segmented sort: S independent u32 key + u32 value sorts with
    log-uniform sizes, as one enqueue (eager and replayed from a captured
    HIP graph), against one sort call per segment on the same stream (eager
    and replayed from a captured graph).  Every leg is timed with HIP events
    on the stream the work runs on.  quick: fewer timed repetitions (for the
    default bench run, which carries this beside the headline)."""
    lo, hi = (int(x) for x in args.seg_log2.split(","))
    S = args.segments
    steps = min(args.steps, 10) if quick else args.steps
    warmup = min(args.warmup, 2) if quick else args.warmup
    t0 = time.perf_counter()
    print(f"generating {S} segments on the host", file=sys.stderr, flush=True)
    keys, vals, off = datagen.segmented(num_segments=S, lo_log2=lo, hi_log2=hi, bits=32, seed=1)
    if args.seg_dist == "zero":
        keys[:] = 0
    elif args.seg_dist == "bucket":
        table = np.unique(datagen.MT19937(2).u32(256))[:64]
        assert table.size == 64
        keys = table[keys >> np.uint32(26)]
    gen_s = time.perf_counter() - t0
    print(f"generated {off[-1]} elements in {gen_s:.1f} s", file=sys.stderr, flush=True)
    total = int(off[-1])
    sizes = np.diff(off.astype(np.int64))
    kd = torch.from_numpy(keys).to(dev)
    vd = torch.from_numpy(vals).to(dev)
    offd = torch.from_numpy(off.view(np.int64)).to(dev)
    ko = torch.empty_like(kd)
    vo = torch.empty_like(vd)
    ctx = rs.context(0)
    if args.tiny_cap >= 0:
        ctx.tiny_cap(args.tiny_cap)
    tiny_cap = ctx.tiny_cap()
    tuning = None
    if not args.no_tune:
        # the autotuner times every configuration on this batch and selects
        # the fastest; the eager runs and the captured graph below use it
        from paper_1511_03404_amd import tune
        tuning = tune.tune_segmented(kd, vd, offd, ctx=ctx, reps=3, warmup=1)
        print(f"tuned: {tuning}", file=sys.stderr, flush=True)
    cfg_index = ctx.tune_get(32, True, True, rs.size_class(total))
    cfg = rs.configs(32, True)[cfg_index]
    ws = torch.empty(ctx.segmented_workspace_bytes(32, True, total, S), dtype=torch.uint8,
                     device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def batched():
        rs.segmented_sort(kd, vd, offd, ko, vo, ctx=ctx, workspace=ws)

    for _ in range(warmup):
        batched()
    torch.cuda.synchronize()
    print("timing the batched form", file=sys.stderr, flush=True)
    ctx.profile_reset()
    ctx.profile_enable(True)
    ev0.record()
    for _ in range(steps):
        batched()
    ev1.record()
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    batched_ms = ev0.elapsed_time(ev1) / steps
    recs = ctx.profile_read()
    kern = {}
    for name, tag, ms in recs:
        kern.setdefault(name, []).append(ms)
    kern_ms = {k: round(sum(v) / steps, 4) for k, v in kern.items()}

    print(f"batched: {batched_ms:.3f} ms; graph capture and replay", file=sys.stderr, flush=True)
    # the same enqueue captured once into a graph and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batched()
    g.replay()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        g.replay()
    ev1.record()
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / steps

    # one sort call per segment, same stream, no host synchronisation: timed
    # with HIP events like the batched form, eager (the device also waits for
    # the host's launches) and replayed from one captured graph (launches
    # submitted together: the per-segment form at its best)
    ws1 = torch.empty(ctx.workspace_bytes(32, True, int(sizes.max())), dtype=torch.uint8,
                      device=dev)
    bounds = list(zip(off[:-1].tolist(), off[1:].tolist()))

    def per_segment():
        for a, b in bounds:
            if b - a > 1:
                rs.sort_pairs(kd[a:b], vd[a:b], ko[a:b], vo[a:b], ctx=ctx, workspace=ws1)
            elif b - a == 1:
                ko[a:b].copy_(kd[a:b])
                vo[a:b].copy_(vd[a:b])

    per_seg_ms = per_seg_wall_ms = per_seg_graph_ms = None
    per_seg_graph_error = None
    if args.per_segment_steps > 0:
        print("timing one sort call per segment", file=sys.stderr, flush=True)
        per_segment()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(args.per_segment_steps):
            per_segment()
        ev1.record()
        torch.cuda.synchronize()
        per_seg_wall_ms = (time.perf_counter() - t0) * 1e3 / args.per_segment_steps
        per_seg_ms = ev0.elapsed_time(ev1) / args.per_segment_steps
        try:
            print("capturing the per-segment calls in one graph", file=sys.stderr, flush=True)
            gp = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gp):
                per_segment()
            gp.replay()
            torch.cuda.synchronize()
            reps = max(1, min(steps, 5))
            ev0.record()
            for _ in range(reps):
                gp.replay()
            ev1.record()
            torch.cuda.synchronize()
            per_seg_graph_ms = ev0.elapsed_time(ev1) / reps
            del gp
        except Exception as e:  # report, do not lose the rest of the line
            per_seg_graph_error = f"{type(e).__name__}: {e}"
        # the last leg to write the outputs is a per-segment one: check it
        # against the batched form's result on a sample of segments
        bk, bv = torch.empty_like(kd), torch.empty_like(vd)
        rs.segmented_sort(kd, vd, offd, bk, bv, ctx=ctx, workspace=ws)
        torch.cuda.synchronize()
        for s_ in range(0, S, max(1, S // 50)):
            a, b = bounds[s_]
            assert torch.equal(bk[a:b], ko[a:b]) and torch.equal(bv[a:b], vo[a:b]), \
                f"per-segment and batched results differ in segment {s_}"
        del bk, bv

    large = sizes[sizes > 16384]
    pass_ms = kern.get("k_seg_pass_u32", [])
    roofline = None
    if pass_ms:
        avg = sum(pass_ms) / len(pass_ms)
        bpl = 2 * int(large.sum()) * 8
        achieved = bpl / (avg * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_seg_pass_u32", "avg_launch_ms": round(avg, 5),
                    "launches": len(pass_ms), "bytes_per_launch": bpl,
                    "elements_in_large_segments": int(large.sum())}
    tiny = sizes[(sizes > 1) & (sizes <= tiny_cap)]
    tiny_ms = kern.get("k_seg_bitonic", [])
    tiny_roofline = None
    if tiny_ms and tiny.size:
        avg = sum(tiny_ms) / len(tiny_ms)
        bpl = 2 * int(tiny.sum()) * 8  # read and write every key and value once
        achieved = bpl / (avg * 1e-3) / 1e9
        tiny_roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "kernel": "k_seg_bitonic", "avg_launch_ms": round(avg, 5),
                         "launches": len(tiny_ms), "bytes_per_launch": bpl,
                         "segments": int(tiny.size), "elements": int(tiny.sum())}
    out = {
        "metric": "Mkeys/s, batched segmented sort vs one launch per segment",
        "value": round(total / batched_ms / 1e3, 1),
        "unit": "Mkeys/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(batched_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{S} independent u32 key + u32 value segments, sizes "
                               f"floor(2^({lo}+{hi - lo}u)) log-uniform in [2^{lo}, 2^{hi}], "
                               f"{args.seg_dist} keys, value = index in segment; MT19937 "
                               f"seed 1",
                   "segments": S, "total_elements": total,
                   "elements_in_large_segments": int(large.sum()),
                   "tiny_cap": tiny_cap,
                   "segments_by_class": {"le1": int((sizes <= 1).sum()),
                                         "tiny_bitonic": int(tiny.size),
                                         "small_le4096": int(((sizes > max(1, tiny_cap)) & (sizes <= 4096)).sum()),
                                         "medium_le16384": int(((sizes > 4096) & (sizes <= 16384)).sum()),
                                         "large": int(large.size)}},
        "batched_ms": round(batched_ms, 3),
        "graph_replay_ms": round(graph_ms, 3),
        "graph_replay_Mkeys_s": round(total / graph_ms / 1e3, 1),
        "per_segment_launch_ms": round(per_seg_ms, 3) if per_seg_ms else None,
        "per_segment_launch_wall_ms": round(per_seg_wall_ms, 3) if per_seg_wall_ms else None,
        "per_segment_launch_Mkeys_s": round(total / per_seg_ms / 1e3, 1) if per_seg_ms else None,
        "per_segment_graph_replay_ms": round(per_seg_graph_ms, 3) if per_seg_graph_ms else None,
        "per_segment_graph_error": per_seg_graph_error,
        "speedup_batched_vs_per_segment": round(per_seg_ms / batched_ms, 2) if per_seg_ms else None,
        # both forms replayed from captured graphs: no host launch cost in either
        "speedup_batched_vs_per_segment_graphs": round(per_seg_graph_ms / graph_ms, 2)
        if per_seg_graph_ms else None,
        "timing": "HIP events on the launch stream for every leg; per_segment_launch_wall_ms "
                  "is the host clock around the same eager loop",
        "hbm_frac_whole_batch": round(4 * 2 * total * 8 / (batched_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "kernels_ms": kern_ms,
        "roofline": roofline,
        "tiny_roofline": tiny_roofline,
        "kernel_config": dict(cfg, index=cfg_index),
        "tuning": tuning,
        "host_generation_s": round(gen_s, 1),
    }
    if with_cpu:
        out["cpu_baseline"] = segmented_cpu_baseline(keys, vals, off, S, quick)
    return out


def segmented_cpu_baseline(keys, vals, off, S, quick):
    """The oracle's segmented sort on the host: one thread on a sample of
    segments, and every usable core (one thread per core, each sorting a
    contiguous share of the segments; the oracle's C code releases the GIL
    and keeps no global state) on the whole batch."""
    import concurrent.futures
    import oracle
    info = host_info()
    # one thread: the first segments, about 2 s of work in the quick form
    m = S // 10 if quick else S
    a, b = 0, int(off[m])
    t0 = time.perf_counter()
    oracle.segmented_sort(keys[a:b], vals[a:b], off[:m + 1])
    dt1 = time.perf_counter() - t0
    # all cores: contiguous shares of about equal element counts
    workers = max(1, min(info["usable_cpus"] or 1, 16))
    total = int(off[S])
    cuts = [0]
    for w in range(1, workers):
        cuts.append(int(np.searchsorted(off, total * w // workers)))
    cuts.append(S)
    cuts = sorted(set(cuts))

    def share(i):
        lo_s, hi_s = cuts[i], cuts[i + 1]
        lo_e, hi_e = int(off[lo_s]), int(off[hi_s])
        oracle.segmented_sort(keys[lo_e:hi_e], vals[lo_e:hi_e], off[lo_s:hi_s + 1] - off[lo_s])

    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        list(ex.map(share, range(len(cuts) - 1)))
    dtn = time.perf_counter() - t0
    return {"value": round((b - a) / dt1 / 1e6, 3), "unit": "Mkeys/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the first {m} segments ({b - a} elements), one thread, {dt1:.1f} s",
            "all_cores": {"value": round(total / dtn / 1e6, 3), "unit": "Mkeys/s",
                          "cores": workers,
                          "sample": f"all {S} segments ({total} elements) in {len(cuts) - 1} "
                                    f"contiguous shares, one thread each, {dtn:.1f} s"},
            "host": info}


def bench_merge(args, torch, rs, datagen, dev):
    """The stable merge sort (paper, Section 2.4) on the inputs of a radix
    workload: one sort per distribution per step, inputs resident, HIP-event
    timing of every kernel; the roofline is that of the merge pass, which
    reads and writes every element once per merge level."""
    import oracle
    n, bits, has_v, wdesc = WORKLOADS[args.merge_kind]
    dists = list(datagen.DISTRIBUTIONS) if args.dists == "all" else args.dists.split(",")
    kb = bits // 8
    vb = kb if has_v else 0
    ins = []
    for d in dists:
        k = torch.from_numpy(datagen.keys(d, n, bits, seed=1)).to(dev)
        v = torch.from_numpy(datagen.values(n, bits)).to(dev) if has_v else None
        ins.append((d, k, v))
    ko = torch.empty(n, dtype=ins[0][1].dtype, device=dev)
    vo = torch.empty(n, dtype=ins[0][1].dtype, device=dev) if has_v else None
    ctx = rs.context(0)
    ws = torch.empty(ctx.merge_workspace_bytes(bits, has_v, n), dtype=torch.uint8, device=dev)

    def step():
        for i, (d, k, v) in enumerate(ins):
            ctx.profile_tag(i)
            rs.merge_sort(k, v, ko, vo, ctx=ctx, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_reset()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile_enable(False)
    recs = ctx.profile_read()
    per = {}
    for i, d in enumerate(dists):
        kern = {}
        for name, tag, ms in recs:
            if tag == i:
                kern.setdefault(name, []).append(ms)
        sort_ms = sum(sum(v) for v in kern.values()) / args.steps
        per[d] = {"ms_per_sort": round(sort_ms, 4), "Mkeys_s": round(n / sort_ms / 1e3, 1),
                  "kernels_ms": {k: round(sum(v) / args.steps, 4) for k, v in kern.items()}}
    pass_name = f"k_merge_pass_u{bits}_{'pairs' if has_v else 'keys'}"
    ref = dists.index("uniform") if "uniform" in dists else 0
    pass_ms = [ms for name, tag, ms in recs if tag == ref and name == pass_name]
    roofline = None
    if pass_ms:
        avg = sum(pass_ms) / len(pass_ms)
        bytes_per_launch = 2 * n * (kb + vb)  # one merge level reads and writes everything
        achieved = bytes_per_launch / (avg * 1e-3) / 1e9
        t = "unsigned int" if bits == 32 else "unsigned long"
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": pass_name,
                    "kernel_instance": f"void rs::k_merge_pass<{t}, {t}, "
                                       f"{'true' if has_v else 'false'}, "
                                       f"{'512, 4' if bits == 64 else '256, 8'}, 1>",
                    "avg_launch_ms": round(avg, 5), "launches": len(pass_ms),
                    "bytes_per_launch": bytes_per_launch, "input": dists[ref]}
    levels = 0
    while (8192 << levels) < n:
        levels += 1
    if roofline is not None:
        roofline["traffic"] = measured_traffic("merge_" + args.merge_kind, None)
    out = {
        "metric": "Mkeys/s (stable merge sort)", "value": round(n * len(dists) * args.steps /
                                                                 elapsed / 1e6, 1),
        "unit": "Mkeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"u{bits}", "data": "synthetic",
        "config": {"workload": f"merge sort of {wdesc}; one sort per distribution per step "
                               f"({', '.join(dists)}); MT19937 seed 1; tiles of 8192 sorted "
                               f"in LDS, then {levels} merge levels of 2048-output workgroups",
                   "n": n, "key_bits": bits, "value_bits": bits if has_v else 0,
                   "distributions": dists, "merge_levels": levels},
        "roofline": roofline, "per_distribution": per,
    }
    if not args.no_cpu_baseline:
        m = 1 << min(args.cpu_sample_log2, n.bit_length() - 1, 25)
        tot = 0.0
        for d in dists:
            k = datagen.keys(d, m, bits, seed=1)
            v = datagen.values(m, bits) if has_v else None
            t0 = time.perf_counter()
            oracle.merge_sort(k, v)
            tot += time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(dists) * m / tot / 1e6, 3), "unit": "Mkeys/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's merge sort, one sort per distribution "
                                         f"at n=2^{m.bit_length() - 1}, one thread, {tot:.1f} s"}
    print(json.dumps(out), flush=True)


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs, and the CPUs this
    process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(bits, has_v, dists, sample_log2, min_seconds=12.0, max_repeats=4):
    """The oracle, as it stands, on a bounded sample of the same workload:
    one sort per distribution at n = 2^sample_log2 (single thread), the set
    repeated until it has run for at least min_seconds (at most max_repeats
    times)."""
    import datagen
    import oracle
    n = 1 << sample_log2
    inputs = [(datagen.keys(d, n, bits, seed=1), datagen.values(n, bits) if has_v else None)
              for d in dists]
    total_t = 0.0
    repeats = 0
    while repeats < max_repeats and (repeats == 0 or total_t < min_seconds):
        for k, v in inputs:
            t0 = time.perf_counter()
            oracle.sort(k, v)
            total_t += time.perf_counter() - t0
        repeats += 1
    return {
        "value": round(repeats * len(dists) * n / total_t / 1e6, 3),
        "unit": "Mkeys/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one sort per distribution ({','.join(dists)}) at n=2^{sample_log2}, "
                  f"{bits}-bit {'pairs' if has_v else 'keys'}, seed 1, {repeats} repeat(s); "
                  f"{total_t:.1f} s",
        "host": host_info(),
    }


def main():
    args = parse()
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(args.summarize_pmc), indent=1))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the sort runs on one GPU only; sharding across GPUs is "
                          "described in the design notes, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import datagen
    import paper_1511_03404_amd as rs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    rs.lib()  # fails loudly if librs.so is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "copy_calib":
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # counter readings calibrate the counters read on the sort kernels
        a = torch.ones(COPY_CALIB_BYTES // 4, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy_calib", "bytes_read": COPY_CALIB_BYTES,
                          "bytes_written": COPY_CALIB_BYTES,
                          "launches": args.warmup + args.steps}), flush=True)
        return
    if args.workload == "segmented":
        bench_segmented(args, torch, rs, datagen, dev)
        return
    if args.workload == "serving":
        bench_serving(args, torch, rs, datagen, dev)
        return
    if args.workload == "grid":
        bench_grid(args, torch, rs, datagen, dev)
        return
    if args.workload == "merge":
        bench_merge(args, torch, rs, datagen, dev)
        return
    out = measure_sorts(args, torch, rs, datagen, dev, args.workload, args.steps, args.warmup,
                        with_cpu=not args.no_cpu_baseline)
    if args.workload == "u32_pairs" and not args.no_extras:
        out["metric"] = ("Mkeys/s and % HBM roofline, 2^26 u32 pairs + u64 keys; segmented "
                         "batch vs per-launch")
        out["value_is"] = "2^26 u32 pairs, mean over the six distributions"
        # the rest of the headline metric, in the same line: the copy ceiling,
        # 2^25 64-bit keys, and the batched segmented sort against one sort
        # call per segment
        copy = measure_copy(torch, dev)
        out["copy_ceiling"] = copy
        if out.get("roofline"):
            out["roofline"]["frac_of_copy_ceiling"] = round(
                out["roofline"]["achieved"] / copy["GBs"], 4)
        print("u32 pairs done; 2^25 u64 keys", file=sys.stderr, flush=True)
        u64 = measure_sorts(args, torch, rs, datagen, dev, "u64_keys", min(args.steps, 10),
                            min(args.warmup, 3), with_cpu=False)
        out["u64_keys"] = {k: u64[k] for k in ("value", "unit", "ms_per_step", "config",
                                               "kernel_config", "hbm_frac_whole_sort",
                                               "hbm_frac_whole_sort_nontrivial", "roofline",
                                               "per_distribution")}
        if out["u64_keys"].get("roofline"):
            out["u64_keys"]["roofline"]["frac_of_copy_ceiling"] = round(
                out["u64_keys"]["roofline"]["achieved"] / copy["GBs"], 4)
        print("u64 keys done; segmented batch", file=sys.stderr, flush=True)
        seg = measure_segmented(args, torch, rs, datagen, dev,
                                with_cpu=not args.no_cpu_baseline, quick=True)
        out["segmented"] = seg
    print(json.dumps(out), flush=True)


def measure_copy(torch, dev, nbytes=1 << 30, reps=20):
    """The device's plain-copy ceiling: 1 GiB device-to-device copies timed
    with HIP events (read + write bytes per second), by the library's copy
    kernel and by torch's copy_ (the runtime's); the faster one is the
    ceiling."""
    import paper_1511_03404_amd as rs
    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(3):
            fn()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps

    ms_lib = timed(lambda: rs.device_copy(a, b))
    assert bool(torch.equal(a[:4096], b[:4096]))
    ms_rt = timed(lambda: b.copy_(a))
    del a, b
    ms = min(ms_lib, ms_rt)
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "ms_per_copy": round(ms, 4),
            "library_copy_GBs": round(2 * nbytes / (ms_lib * 1e-3) / 1e9, 1),
            "runtime_copy_GBs": round(2 * nbytes / (ms_rt * 1e-3) / 1e9, 1),
            "how": "1 GiB device-to-device copies, mean of "
                   f"{reps} after 3 warm-ups, read + write bytes: the library's copy kernel "
                   "(rs_device_copy) and torch copy_ (the runtime's); the faster one"}


def moving_passes(keys, bits, r=8):
    """Digit positions (r bits) at which the keys are not all equal: the
    passes of an LSD sort that move data (an all-equal digit is the identity
    permutation and its pass is skipped)."""
    import numpy as np
    u = keys.view(np.uint32 if bits == 32 else np.uint64)
    diff = np.bitwise_or.reduce(u ^ u[0]) if u.size else 0
    mask = (1 << r) - 1
    return sum(1 for p in range(bits // r) if (int(diff) >> (p * r)) & mask)


def measure_sorts(args, torch, rs, datagen, dev, workload, steps, warmup, with_cpu=True):
    """One radix-sort workload: one sort per distribution per step, inputs
    resident in HBM, out of place; the dict of the JSON line."""
    n, bits, has_v, wdesc = WORKLOADS[workload]
    dists = list(datagen.DISTRIBUTIONS) if args.dists == "all" else args.dists.split(",")
    kb = bits // 8
    vb = kb if has_v else 0

    # inputs resident in HBM before timing; per input, how many digit
    # positions (8-bit) are not the same for every key: the passes that move
    # data (the others are skipped)
    ins = []
    moving = {}
    for d in dists:
        kh = datagen.keys(d, n, bits, seed=1)
        moving[d] = moving_passes(kh, bits)
        k = torch.from_numpy(kh).to(dev)
        del kh
        v = torch.from_numpy(datagen.values(n, bits)).to(dev) if has_v else None
        ins.append((d, k, v))
    ko = torch.empty(n, dtype=ins[0][1].dtype, device=dev)
    vo = torch.empty(n, dtype=ins[0][1].dtype, device=dev) if has_v else None
    ctx = rs.context(0)
    tuning = None
    if not args.no_tune:
        # the autotuner times every compiled configuration on uniform keys of
        # this size and selects the fastest for the size class (untimed)
        from paper_1511_03404_amd import tune
        tuning = tune.tune_sort(bits, has_v, n, ctx=ctx, reps=5, warmup=1)
        print(f"tuned: {tuning}", file=sys.stderr, flush=True)
    cfg_index = ctx.tune_get(bits, has_v, False, rs.size_class(n))
    cfg = rs.configs(bits, has_v)[cfg_index]
    ws = torch.empty(ctx.workspace_bytes(bits, has_v, n), dtype=torch.uint8, device=dev)

    def step():
        for i, (d, k, v) in enumerate(ins):
            ctx.profile_tag(i)
            if has_v:
                rs.sort_pairs(k, v, ko, vo, ctx=ctx, workspace=ws)
            else:
                rs.sort_keys(k, ko, ctx=ctx, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    ctx.profile_reset()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile_enable(False)
    recs = ctx.profile_read()

    elapsed = t1 - t0
    ms_per_step = elapsed / steps * 1e3
    keys_total = n * len(dists) * steps
    value = keys_total / elapsed / 1e6

    # per-distribution times from the events (sum of the kernels of one sort)
    per = {}
    for i, d in enumerate(dists):
        mine = [ms for name, tag, ms in recs if tag == i]
        sort_ms = sum(mine) / steps
        # the launches of one sort are consecutive: per-sort times, median
        per_launch = len(mine) // steps
        sorts = [sum(mine[j * per_launch:(j + 1) * per_launch]) for j in range(steps)]
        b_alg = kb * 2 * n * (kb + vb)  # P8 passes x 2 x n x (k + v)
        # bytes the executed passes move (a copy when every pass is skipped)
        b_exec = max(moving[d], 1) * 2 * n * (kb + vb)
        per[d] = {"ms_per_sort": round(sort_ms, 4),
                  "ms_per_sort_median": round(statistics.median(sorts), 4),
                  "Mkeys_s": round(n / sort_ms / 1e3, 1),
                  "hbm_frac_alg": round(b_alg / (sort_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                  "passes_moving": moving[d],
                  "bytes_executed": b_exec,
                  "hbm_frac_executed": round(b_exec / (sort_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
        kern = {}
        for name, tag, ms in recs:
            if tag == i:
                kern.setdefault(name, []).append(ms)
        per[d]["kernels_ms"] = {k: round(sum(v) / steps, 4) for k, v in kern.items()}

    # roofline of the dominant kernel: the digit pass, on the input where
    # every pass moves data (uniform), per launch
    pass_name = f"k_pass_u{bits}_{'pairs' if has_v else 'keys'}"
    ref = dists.index("uniform") if "uniform" in dists else 0
    pass_ms = [ms for name, tag, ms in recs if tag == ref and name == pass_name]
    roofline = None
    if pass_ms:
        avg = sum(pass_ms) / len(pass_ms)
        bytes_per_launch = 2 * n * (kb + vb)  # read + write of keys and values, one digit
        achieved = bytes_per_launch / (avg * 1e-3) / 1e9
        traffic = measured_traffic(workload, cfg)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic,
                    # the counters' bytes over the same launch time (null without them)
                    "traffic_GBs": (round(traffic / (avg * 1e-3) / 1e9, 1) if traffic else None),
                    "kernel": pass_name, "kernel_instance": pass_kernel_name(bits, has_v, cfg),
                    "avg_launch_ms": round(avg, 5),
                    "launches": len(pass_ms), "bytes_per_launch": bytes_per_launch,
                    "input": dists[ref]}

    whole_frac = (kb * 2 * n * (kb + vb)) * len(dists) * steps / elapsed / (HBM_PEAK_GBS * 1e9)
    # the same fraction without the all-zero input, whose passes are all
    # skipped (it moves one read of the keys, not P8 passes): a timed loop
    # over the other distributions, HIP events, profiling off
    nontriv = [i for i, d in enumerate(dists) if d != "zero"]
    nt = None
    if nontriv:
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            for i in nontriv:
                _, k, v = ins[i]
                if has_v:
                    rs.sort_pairs(k, v, ko, vo, ctx=ctx, workspace=ws)
                else:
                    rs.sort_keys(k, ko, ctx=ctx, workspace=ws)
        ev1.record()
        ev1.synchronize()
        nt_ms = ev0.elapsed_time(ev1) / (steps * len(nontriv))
        nt = {"distributions": [dists[i] for i in nontriv], "ms_per_sort": round(nt_ms, 4),
              "Mkeys_s": round(n / nt_ms / 1e3, 1),
              "hbm_frac_whole_sort": round(kb * 2 * n * (kb + vb) / (nt_ms * 1e-3) /
                                           (HBM_PEAK_GBS * 1e9), 4)}
    out = {
        "metric": "Mkeys/s and % HBM roofline",
        "value": round(value, 1),
        "unit": "Mkeys/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"u{bits}",
        "data": "synthetic",
        "config": {"workload": f"{wdesc}; one sort per distribution per step "
                               f"({', '.join(dists)}); MT19937 seed 1",
                   "n": n, "key_bits": bits, "value_bits": bits if has_v else 0,
                   "distributions": dists, "digit_bits": cfg["radix_bits"],
                   "tile": f"{cfg['threads']}x{cfg['items']}"},
        "kernel_config": dict(cfg, index=cfg_index),
        "tuning": tuning,
        "hbm_frac_whole_sort": round(whole_frac, 4),
        "hbm_frac_whole_sort_nontrivial": nt["hbm_frac_whole_sort"] if nt else None,
        "nontrivial": nt,
        "roofline": roofline,
        "per_distribution": per,
        "paper_context": {"hardware": "GeForce GTX670 (2 GB) and Intel Core i7-3770K at 3.5 GHz",
                          "rates": None,
                          "note": "the paper shows its radix-sort rates only in figures; its text "
                                  "prints no number to compare with"},
    }
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(bits, has_v, dists,
                                           min(args.cpu_sample_log2, n.bit_length() - 1))
    return out


if __name__ == "__main__":
    main()
