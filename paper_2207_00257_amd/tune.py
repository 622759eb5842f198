"""Autotuner for the plain normalize path's launch parameters.

Sweeps the reduce kernel's shape (layout, block, unroll, grid, load hint)
with the map at its defaults, then the map kernel's shape (layout, block,
unroll, grid, load hint, traversal direction) with the best reduce, timing
each kernel with the HIP events the library records around it on the call's
stream. Every candidate is a valid parameter set of the C ABI, so the sweep
changes only speed and the low bits allowed by the error bound.

    python -m paper_2207_00257_amd.tune --log2n 28 [--dtype f32] [--out FILE]

Results are written as JSON: the best parameters per (arch, in/out dtype,
accumulation, size class) and the full table of measured candidates.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

TUNED_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")


def size_class(n: int) -> str:
    """Size classes used as cache keys: powers of two rounded down."""
    return "2^%d" % max(0, n.bit_length() - 1)


DEFAULT_CACHE = os.path.join(TUNED_DIR, "plain.json")


def load_params(path, in_dtype, out_dtype, accum, n):
    """Tuned parameters for this device and size class from a cache file (the
    committed one by default), or None when it has no entry."""
    import torch

    path = path or DEFAULT_CACHE
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = "%s/%s->%s/%s/%s" % (arch, in_dtype, out_dtype, accum, size_class(n))
    ent = cache.get(key)
    return dict(ent["params"]) if ent else None


def _time_call(ctx, out, inp, accum, reps):
    from . import api

    api.normalize(out, inp, accum=accum, ctx=ctx)  # warm (and allocate workspace)
    ctx.set_timing(True)
    for _ in range(reps):
        api.normalize(out, inp, accum=accum, ctx=ctx)
    r, m, c = ctx.kernel_times()
    ctx.set_timing(False)
    return r / c, m / c


def sweep(n: int, in_dtype="f32", out_dtype="f32", accum="f32", reps=5, quick=False, log=print):
    import torch

    from . import api, synth

    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    dev = torch.device("cuda:0")
    x = synth.uniform_f32(n, 3)
    inp = torch.from_numpy(x).to(dev).to(tdt[in_dtype])
    out = torch.empty(n, dtype=tdt[out_dtype], device=dev)
    ctx = api.Context()
    base = ctx.get_params()
    cus = torch.cuda.get_device_properties(dev).multi_processor_count

    grids = [cus * k for k in ((2, 4, 8) if quick else (1, 2, 4, 8, 16))]
    red_space = list(itertools.product((0, 1), (256, 512, 1024), (2, 4, 8), grids, (0, 1)))
    map_grids = [cus * k for k in ((4, 8) if quick else (2, 4, 8, 16, 32))]
    map_space = list(itertools.product((0, 1), (256, 512, 1024), (1, 2, 4, 8), map_grids, (0, 1), (0, 1)))

    table = []
    best_r, best_rt = None, float("inf")
    t0 = time.time()
    for layout, block, unroll, grid, nt in red_space:
        p = dict(base, layout=layout, block=block, unroll=unroll, grid=grid, reduce_nt=nt)
        ctx.set_params(**p)
        rt, _ = _time_call(ctx, out, inp, accum, reps)
        table.append({"kernel": "reduce", "params": p, "ms": rt})
        if rt < best_rt:
            best_r, best_rt = p, rt
    log("reduce sweep: %d candidates in %.1f s, best %.4f ms %s"
        % (len(red_space), time.time() - t0, best_rt, {k: best_r[k] for k in
                                                        ("layout", "block", "unroll", "grid", "reduce_nt")}))
    best_m, best_mt = None, float("inf")
    t0 = time.time()
    for layout, block, unroll, grid, nt, rev in map_space:
        p = dict(best_r, map_layout=layout, map_block=block, map_unroll=unroll, map_grid=grid, map_nt=nt,
                 reverse_map=rev)
        ctx.set_params(**p)
        _, mt = _time_call(ctx, out, inp, accum, reps)
        table.append({"kernel": "map", "params": p, "ms": mt})
        if mt < best_mt:
            best_m, best_mt = p, mt
    log("map sweep: %d candidates in %.1f s, best %.4f ms %s"
        % (len(map_space), time.time() - t0, best_mt, {k: best_m[k] for k in
                                                        ("map_layout", "map_block", "map_unroll", "map_grid",
                                                         "map_nt", "reverse_map")}))
    ctx.close()
    return best_m, best_rt, best_mt, table


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--out-dtype", default=None)
    ap.add_argument("--accum", default="f32")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None, help="JSON file for the best parameters")
    ap.add_argument("--table", default=None, help="JSON file for every measured candidate")
    args = ap.parse_args(argv)
    import torch

    n = 1 << args.log2n
    out_dtype = args.out_dtype or args.dtype
    best, rt, mt, table = sweep(n, args.dtype, out_dtype, args.accum, args.reps, args.quick)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = "%s/%s->%s/%s/%s" % (arch, args.dtype, out_dtype, args.accum, size_class(n))
    result = {"key": key, "params": best, "reduce_ms": rt, "map_ms": mt}
    print(json.dumps(result), flush=True)
    if args.out:
        cache = {}
        if os.path.exists(args.out):
            with open(args.out) as f:
                cache = json.load(f)
        cache[key] = {"params": best, "reduce_ms": rt, "map_ms": mt}
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    if args.table:
        with open(args.table, "w") as f:
            json.dump(table, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
