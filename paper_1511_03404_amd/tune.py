"""Autotuner of the digit-pass configuration: digit width r (4..8 or 11
bits) and tile shape (threads x items per thread).

The radix sort's result does not depend on r (paper, Section 2.6: the keys
are cut into r-bit digits and every digit is a stable counting sort), so
every compiled configuration sorts bit-exactly and only the time differs.
Fewer bits mean more passes over the data; more bits mean more bins, hence
more look-back words and shorter scatter runs per tile; the tile shape
trades per-tile latencies against registers and occupancy.  The tuner
times each configuration on the device and writes the fastest into the
context's tune table (``rs_tune_set``) for the size class ceil(log2 n);
later sorts of that kind and size, and graphs captured after tuning, use it.

    ctx = rs.context(0)
    tune.tune_sort(32, True, 1 << 26, ctx=ctx)          # plain sort, synthetic keys
    tune.tune_segmented(keys, values, offsets, ctx=ctx)  # the caller's own batch
    tune.save([...results...], "tune.json"); tune.load("tune.json", ctx)

Timing uses HIP events on the current stream around each call, inputs
resident on the device, the median of ``reps`` calls after ``warmup``.
"""
from __future__ import annotations

import argparse
import json
import statistics

import torch

from . import (BLOCK_SORT_CAP, Context, configs, context, segmented_sort, size_class, sort_keys,
               sort_pairs)


def _median_ms(fn, reps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def _uniform_keys(n: int, bits: int, device, seed: int) -> torch.Tensor:
    """n keys with every bit uniform (two 32-bit draws per 64-bit key)."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    lo = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int64, device=device, generator=g)
    if bits == 32:
        return lo.to(torch.int32)
    hi = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int64, device=device, generator=g)
    return (hi << 32) | (lo & 0xFFFFFFFF)


def _candidates(key_bits, has_values, candidates, segmented=False):
    cfgs = configs(key_bits, has_values, segmented)
    idx = list(range(len(cfgs))) if candidates is None else list(candidates)
    for i in idx:
        if not 0 <= i < len(cfgs):
            raise ValueError(f"no configuration {i} (there are {len(cfgs)})")
    return cfgs, idx


# a configuration replaces the built-in choice only if it is faster by this
# fraction: ties would otherwise flip the choice from one run to the next
MARGIN = 0.03


def _result(key_bits, has_values, segmented, n, cls, cfgs, times, note=None, default=0):
    best = min(times, key=times.get)
    if default in times and times[default] <= times[best] * (1.0 + MARGIN):
        best = default
    r = {"key_bits": key_bits, "has_values": bool(has_values), "segmented": bool(segmented),
         "size_log2": cls, "n": int(n), "index": best, "config": cfgs[best],
         "ms": {str(i): round(t, 5) for i, t in sorted(times.items())}}
    if note:
        r["note"] = note
    return r


def tune_sort(key_bits: int, has_values: bool, n: int, ctx: Context | None = None,
              reps: int = 5, warmup: int = 1, candidates=None, seed: int = 0,
              apply: bool = True) -> dict:
    """Time every configuration (or ``candidates``, a list of indices) on n
    uniform random keys (values = index) and select the fastest for the size
    class of n.  Returns {index, config, ms per configuration, ...}."""
    ctx = ctx or context()
    dev = torch.device("cuda", ctx.device)
    cfgs, idx = _candidates(key_bits, has_values, candidates)
    cls = size_class(n)
    if n <= BLOCK_SORT_CAP[(key_bits, bool(has_values))]:
        # one workgroup sorts it in LDS whatever the table says
        return _result(key_bits, has_values, False, n, cls, cfgs, {0: 0.0},
                       note="one-workgroup sort; the table is not used at this size")
    keys = _uniform_keys(n, key_bits, dev, seed)
    vals = torch.arange(n, dtype=keys.dtype, device=dev) if has_values else None
    ko = torch.empty_like(keys)
    vo = torch.empty_like(keys) if has_values else None
    prev = ctx.tune_get(key_bits, has_values, False, cls)
    ctx.tune_set(key_bits, has_values, False, cls, -1)
    default = ctx.tune_get(key_bits, has_values, False, cls)  # the built-in choice
    need = 0
    for i in idx:
        ctx.tune_set(key_bits, has_values, False, cls, i)
        need = max(need, ctx.workspace_bytes(key_bits, has_values, n))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    times = {}
    for i in idx:
        ctx.tune_set(key_bits, has_values, False, cls, i)
        if has_values:
            fn = lambda: sort_pairs(keys, vals, ko, vo, ctx=ctx, workspace=ws)  # noqa: E731
        else:
            fn = lambda: sort_keys(keys, ko, ctx=ctx, workspace=ws)  # noqa: E731
        times[i] = _median_ms(fn, reps, warmup)
    res = _result(key_bits, has_values, False, n, cls, cfgs, times, default=default)
    ctx.tune_set(key_bits, has_values, False, cls, res["index"] if apply else prev)
    return res


def tune_segmented(keys: torch.Tensor, values: torch.Tensor | None, offsets: torch.Tensor,
                   ctx: Context | None = None, reps: int = 3, warmup: int = 1,
                   candidates=None, apply: bool = True) -> dict:
    """Time every configuration on the caller's own segmented batch (the
    inputs are read, never written) and select the fastest for the size
    class of its total length."""
    from . import key_bits as _key_bits
    ctx = ctx or context(keys.device.index)
    bits = _key_bits(keys)
    has_v = values is not None
    total = keys.numel()
    nseg = offsets.numel() - 1
    cfgs, idx = _candidates(bits, has_v, candidates, segmented=True)
    cls = size_class(total)
    ko = torch.empty_like(keys)
    vo = torch.empty_like(values) if has_v else None
    prev = ctx.tune_get(bits, has_v, True, cls)
    need = 0
    for i in idx:
        ctx.tune_set(bits, has_v, True, cls, i)
        need = max(need, ctx.segmented_workspace_bytes(bits, has_v, total, nseg))
    ws = torch.empty(need, dtype=torch.uint8, device=keys.device)
    times = {}
    for i in idx:
        ctx.tune_set(bits, has_v, True, cls, i)
        times[i] = _median_ms(
            lambda: segmented_sort(keys, values, offsets, ko, vo, ctx=ctx, workspace=ws),
            reps, warmup)
    res = _result(bits, has_v, True, total, cls, cfgs, times)
    res["segments"] = nseg
    ctx.tune_set(bits, has_v, True, cls, res["index"] if apply else prev)
    return res


def apply(results, ctx: Context | None = None) -> int:
    """Write tuning results into a context's table.  An entry whose stored
    configuration is not the library's configuration at that index (the
    library was rebuilt with another list) is skipped.  Returns the number
    applied."""
    ctx = ctx or context()
    done = 0
    for r in results:
        cfgs = configs(r["key_bits"], r["has_values"])
        i = r["index"]
        if not 0 <= i < len(cfgs) or cfgs[i] != r["config"]:
            continue
        ctx.tune_set(r["key_bits"], r["has_values"], r["segmented"], r["size_log2"], i)
        done += 1
    return done


def save(results, path: str, device_name: str | None = None):
    with open(path, "w") as f:
        json.dump({"device": device_name, "entries": list(results)}, f, indent=1)


def load(path: str, ctx: Context | None = None) -> int:
    with open(path) as f:
        return apply(json.load(f)["entries"], ctx)


def main():
    ap = argparse.ArgumentParser(description="tune the digit-pass configuration per size class")
    ap.add_argument("--out", required=True, help="JSON file to write")
    ap.add_argument("--sizes-log2", default="16,18,20,22,24,26",
                    help="comma list of log2 sizes to tune (64-bit kinds stop at 25)")
    ap.add_argument("--kinds", default="u32_keys,u32_pairs,u64_keys,u64_pairs")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    ctx = context(0)
    results = []
    for kind in args.kinds.split(","):
        bits = 32 if kind.startswith("u32") else 64
        has_v = kind.endswith("pairs")
        for s in (int(x) for x in args.sizes_log2.split(",")):
            if bits == 64 and s > 25:
                continue
            r = tune_sort(bits, has_v, 1 << s, ctx=ctx, reps=args.reps)
            print(json.dumps(r), flush=True)
            results.append(r)
    save(results, args.out, torch.cuda.get_device_name(0))


if __name__ == "__main__":
    main()
