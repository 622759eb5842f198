"""Autotuner for the plain normalize path's launch parameters.

Sweeps the reduce kernel's shape (layout, block, unroll, grid, load hint,
fused combine) with the map at its defaults, then the map kernel's shape
(layout, block, unroll, grid, load hint, traversal direction) with the best
reduce, then the tile size; every candidate is scored by the time of both
kernels, measured with the HIP events the library records around them on
the call's stream. Every candidate is a valid parameter set of the C ABI, so the sweep
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


def load_batch_params(path=None, workload="ragged4096"):
    """Tuned batched parameters for this device from a cache file, or None."""
    import torch

    path = path or DEFAULT_CACHE
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    ent = cache.get("%s/batched/f32->f32/f32/%s" % (arch, workload))
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
    """Three stages, each scored by the time of both kernels (the fused
    combine moves work from the reduce into the map): the reduce's shape
    (layout, block, unroll, grid, load hint, fused combine) with the map at
    its defaults; the map's shape (layout, block, unroll, grid, load hint,
    direction) with the best reduce; then the tile size, and the temporal tail
    of the reduce jointly with the fastest reduce shapes."""
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

    grids = [cus * k for k in ((1, 2, 4) if quick else (1, 2, 4, 8, 16))]
    red_space = list(itertools.product((0, 1, 2), (256, 512, 1024), (2, 4, 8), grids, (0, 1), (0, 1)))
    map_grids = [cus * k for k in ((8, 64) if quick else (2, 4, 8, 16, 32, 64))]
    map_space = [c for c in itertools.product((0, 1, 2), (256, 512, 1024), (1, 2, 4, 8), map_grids, (0, 1), (0, 1))
                 if not (c[0] == 2 and c[5])]  # the tiled map has no reverse walk

    table = []
    best, best_t = None, float("inf")

    def measure(p, stage):
        nonlocal best, best_t
        ctx.set_params(**p)
        rt, mt = _time_call(ctx, out, inp, accum, reps)
        table.append({"kernel": stage, "params": p, "ms": rt + mt, "reduce_ms": rt, "map_ms": mt})
        if rt + mt < best_t:
            best, best_t = dict(p), rt + mt
        return rt, mt

    t0 = time.time()
    for layout, block, unroll, grid, nt, fused in red_space:
        if fused and grid > 1024:
            continue  # the fused combine takes at most 1024 partials
        measure(dict(base, layout=layout, block=block, unroll=unroll, grid=grid, reduce_nt=nt,
                     fused_combine=fused), "reduce")
    log("reduce sweep: %d candidates in %.1f s, best %.4f ms %s"
        % (len(red_space), time.time() - t0, best_t, {k: best[k] for k in
                                                       ("layout", "block", "unroll", "grid", "reduce_nt",
                                                        "fused_combine")}))
    best_r = dict(best)
    t0 = time.time()
    for layout, block, unroll, grid, nt, rev in map_space:
        measure(dict(best_r, map_layout=layout, map_block=block, map_unroll=unroll, map_grid=grid, map_nt=nt,
                     reverse_map=rev), "map")
    log("map sweep: %d candidates in %.1f s, best %.4f ms %s"
        % (len(map_space), time.time() - t0, best_t, {k: best[k] for k in
                                                       ("map_layout", "map_block", "map_unroll", "map_grid",
                                                        "map_nt", "reverse_map")}))
    # tile size (either kernel tiled), then the tail the reduce leaves in the
    # last-level cache, read first by a reverse map
    if best["layout"] == 2 or best["map_layout"] == 2:
        for tl in range(12, 20):
            measure(dict(best, tile_log2=tl), "tile")
    # The temporal tail couples the kernels: the map finds it in the
    # last-level cache, so a reduce shape that is fastest on its own can lose
    # overall without one. The tail is therefore swept with the fastest few
    # reduce shapes of the first stage, not only with the shape chosen there.
    shape_keys = ("layout", "block", "unroll", "grid", "fused_combine")
    shapes = [{k: best[k] for k in shape_keys}]
    for r in sorted((r for r in table if r["kernel"] == "reduce" and r["params"]["reduce_nt"]),
                    key=lambda r: r["reduce_ms"]):
        s = {k: r["params"][k] for k in shape_keys}
        if s not in shapes:
            shapes.append(s)
        if len(shapes) == (3 if quick else 7):
            break
    best_m = dict(best)
    for shape in shapes:
        for keep, rev, nt in itertools.product((0, 64, 128, 192, 224, 256, 288, 384), (0, 1), (0, 1)):
            if (nt == 0 and keep) or (rev and best_m["map_layout"] == 2):
                continue  # all of the reduce's loads are temporal anyway / no reverse walk when tiled
            measure(dict(best_m, reduce_keep_mib=keep, reverse_map=rev, reduce_nt=nt, **shape), "keep")
    # the leaders again, interleaved round by round with more repetitions, so
    # that neither a single noisy measurement nor drift picks the winner
    leaders = []
    for r in sorted(table, key=lambda r: r["ms"]):
        if r["params"] not in leaders:
            leaders.append(r["params"])
        if len(leaders) == (4 if quick else 10):
            break
    sums = [[0.0, 0.0] for _ in leaders]
    for _ in range(6):
        for i, p in enumerate(leaders):
            ctx.set_params(**p)
            rt, mt = _time_call(ctx, out, inp, accum, reps)
            sums[i][0] += rt
            sums[i][1] += mt
    i = min(range(len(leaders)), key=lambda i: sums[i][0] + sums[i][1])
    best, rt, mt = leaders[i], sums[i][0] / 6, sums[i][1] / 6
    for p, (r_, m_) in zip(leaders, sums):
        table.append({"kernel": "final", "params": p, "ms": (r_ + m_) / 6, "reduce_ms": r_ / 6, "map_ms": m_ / 6})
    log("final: best of %d leaders %.4f ms" % (len(leaders), rt + mt))
    ctx.close()
    return best, rt, mt, table


def sweep_batched(rows=4096, seed=4, reps=3, quick=False, log=print):
    """Sweep the batched path's launch shape on the ragged workload (rows with
    log-uniform lengths in [32, 2^20], LogNormal(0,1) FP32), timing whole
    calls (planner, short rows, resident rows, tile phases) with the
    library's events: first the resident rows' limit and grid, then the
    short rows' (one per wavefront) limit and grid, then, when some row of
    the workload is longer than the resident limit, the tile phases'
    shapes."""
    import torch

    from . import api, synth

    dev = torch.device("cuda:0")
    x, offs = synth.ragged_batch(rows, seed)
    inp = torch.from_numpy(x).to(dev)
    out = torch.empty_like(inp)
    offs_d = torch.from_numpy(offs).to(dev)
    ctx = api.Context()
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    base_p = ctx.get_batch_params()
    base_p["graph"] = 1
    table, best, best_t = [], None, float("inf")
    t0 = time.time()
    ctx.batch_reserve(rows, x.size)

    def measure(p):
        try:
            ctx.set_batch_params(**p)
        except Exception:
            return None  # shape rejected by the height bound
        api.normalize_batched(out, inp, offs_d, ctx=ctx)
        ctx.set_timing(True)
        for _ in range(reps):
            api.normalize_batched(out, inp, offs_d, ctx=ctx)
        t, c = ctx.batch_times()
        ctx.set_timing(False)
        return t / c

    # resident rows first: how many segments a row may have to be held on
    # chip (0: none, every row takes the tile phases), and how many blocks
    for segs in ((0, 64) if quick else (0, 16, 32, 64)):
        for gmul in ((2,) if quick else (1, 1.5, 2)):
            p = dict(base_p, resident_segments=segs, resident_grid=max(segs, int(cus * gmul)))
            ms = measure(p)
            if ms is None:
                continue
            table.append({"kernel": "batched", "params": p, "ms": ms})
            if ms < best_t:
                best, best_t = p, ms
    # rows per wavefront: rows up to wave_max elements one per wavefront (0:
    # none), and that kernel's grid
    for wmax in ((0, 2048) if quick else (0, 256, 1024, 2048)):
        for gmul in ((4,) if quick or wmax == 0 else (2, 4, 8)):
            p = dict(best, wave_max=wmax, wave_grid=cus * gmul)
            ms = measure(p)
            if ms is None:
                continue
            table.append({"kernel": "batched", "params": p, "ms": ms})
            if ms < best_t:
                best, best_t = p, ms
    base_p = dict(best)
    # the tile phases' shapes matter only for rows longer than the resident
    # limit; with every row of the workload resident they are not swept
    longest = int((offs[1:] - offs[:-1]).max())
    all_resident = base_p["resident_segments"] << 14 >= longest
    if all_resident:
        log("every row is resident (longest %d): tile phases not swept" % longest)
    stage1 = []
    if not all_resident:
        for block in (256, 512, 1024):
            for unroll in ((2, 4) if quick else (1, 2, 4, 8)):
                for tile_log2 in ((14, 15, 16) if quick else (13, 14, 15, 16, 17)):
                    for short_regs in ((2, 8) if quick else (1, 2, 4, 8)):
                        for gmul in ((2, 4) if quick else (1, 2, 4, 8)):
                            stage1.append(dict(base_p, block=block, unroll=unroll, tile_log2=tile_log2,
                                               short_regs=short_regs, grid=cus * gmul * max(1, 1024 // block)))
    for p in stage1:
        ms = measure(p)
        if ms is None:
            continue
        table.append({"kernel": "batched", "params": p, "ms": ms})
        if ms < best_t:
            best, best_t = p, ms
    for map_block in ((256, 512, 1024) if not all_resident else ()):
        for map_unroll in (1, 2, 4, 8):
            for gmul in (1, 2, 4, 8, 16, 32):
                p = dict(best, map_block=map_block, map_unroll=map_unroll,
                         map_grid=cus * gmul * max(1, 1024 // map_block))
                ms = measure(p)
                if ms is None:
                    continue
                table.append({"kernel": "batched", "params": p, "ms": ms})
                if ms < best_t:
                    best, best_t = p, ms
    # the temporal tail phase 1 leaves in the last-level cache for phase 2
    for keep in ((0, 64, 128, 192, 224, 256, 288) if not all_resident else ()):
        p = dict(best, keep_mib=keep)
        ms = measure(p)
        if ms is None:
            continue
        table.append({"kernel": "batched", "params": p, "ms": ms})
        if ms < best_t:
            best, best_t = p, ms
    # the leaders again, interleaved round by round with more repetitions
    leaders = []
    for r in sorted(table, key=lambda r: r["ms"]):
        if r["params"] not in leaders:
            leaders.append(r["params"])
        if len(leaders) == (3 if quick else 8):
            break
    sums = [0.0] * len(leaders)
    for _ in range(6):
        for i, p in enumerate(leaders):
            ms = measure(p)
            sums[i] += ms if ms is not None else float("inf")
    i = min(range(len(leaders)), key=lambda i: sums[i])
    best, best_t = leaders[i], sums[i] / 6
    for p, t_ in zip(leaders, sums):
        table.append({"kernel": "final", "params": p, "ms": t_ / 6})
    log("batched sweep: %d candidates in %.1f s, best %.4f ms %s" % (len(table), time.time() - t0, best_t, best))
    ctx.close()
    return best, best_t, table


def sweep_serve(quick=False, log=print):
    """Sweep the batched launch shape for the serving workload: the server
    (4 slots, spreading, graph replay) replays open-loop Poisson traces at
    100k and 200k requests/s (n log-uniform in [2^8, 2^24], 70 % FP32 / 30 %
    BF16); a candidate's score is the sum of the two p99 latencies."""
    import numpy as np
    import torch

    from . import serve

    torch.cuda.init()
    pool = serve.InputPool(1 << 24, 7)
    traces = []
    for rate in (100000.0, 200000.0):
        tr = serve.make_trace(rate, 1.2, seed=9)
        traces.append((tr, pool.pointers(tr["in_dt"], pool.offsets(tr["n"], 10))))
    shapes = [(256, 8, 4), (1024, 2, 2)]
    space = list(itertools.product(shapes, (1024, 2048), (512, 1024, 2048), (2, 4)))
    if quick:
        space = space[:4]
    table, best, best_s = [], None, float("inf")
    t0 = time.time()
    for (block, unroll, map_unroll), grid, map_grid, short_regs in space:
        bp = dict(block=block, unroll=unroll, map_unroll=map_unroll, grid=grid, tile_log2=15,
                  short_regs=short_regs, map_block=1024, map_grid=map_grid, graph=1)
        p99 = []
        for tr, pt in traces:
            srv = serve.Server(slots=4, batching=True, batch_params=bp)
            n = tr["n"].size
            t_start = srv.replay(np.arange(n), pt, tr["n"], tr["in_dt"], tr["out_dt"], tr["t_ns"])
            comps = srv.wait_all(n, timeout_s=600)
            srv.close()
            p99.append(serve.latency_stats([c for c in comps if c[2] - t_start >= int(0.2e9)])["p99_ms"])
        score = sum(p99)
        table.append({"params": bp, "p99_ms": p99, "score": score})
        log("  %s p99 %.3f / %.3f ms" % ({k: bp[k] for k in ("block", "grid", "map_grid", "short_regs")}, p99[0], p99[1]))
        if score < best_s:
            best, best_s = bp, score
    log("serve sweep: %d candidates in %.1f s, best p99 sum %.3f ms %s" % (len(space), time.time() - t0, best_s, best))
    return best, best_s, table


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
    ap.add_argument("--batched", action="store_true", help="tune the ragged batched path instead")
    ap.add_argument("--serve", action="store_true", help="tune the batched path for the serving workload")
    args = ap.parse_args(argv)
    import torch

    if args.serve:
        best, score, table = sweep_serve(quick=args.quick)
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        key = "%s/batched/f32->f32/f32/serve" % arch
        print(json.dumps({"key": key, "params": best, "p99_sum_ms": score}), flush=True)
        if args.out:
            cache = {}
            if os.path.exists(args.out):
                with open(args.out) as f:
                    cache = json.load(f)
            cache[key] = {"params": best, "p99_sum_ms": score}
            with open(args.out, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        if args.table:
            with open(args.table, "w") as f:
                json.dump(table, f)
        return 0
    if args.batched:
        best, ms, table = sweep_batched(quick=args.quick)
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        key = "%s/batched/f32->f32/f32/ragged4096" % arch
        print(json.dumps({"key": key, "params": best, "ms": ms}), flush=True)
        if args.out:
            cache = {}
            if os.path.exists(args.out):
                with open(args.out) as f:
                    cache = json.load(f)
            cache[key] = {"params": best, "ms": ms}
            with open(args.out, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        if args.table:
            with open(args.table, "w") as f:
                json.dump(table, f)
        return 0

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
