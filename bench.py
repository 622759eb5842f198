"""Benchmark of the normalize hot path on one MI355X.

Default workload: plain normalize, n = 2^28 FP32 (1 GiB in, 1 GiB out),
in[i] ~ U[0.5, 1.5) from seed 3, inputs resident in HBM before timing.
A step is one normalize call (reduce kernel + grid combine + map kernel).

Metric: effective HBM GB/s = n * (2 * sizeof(in) + sizeof(out)) / t, i.e.
three element transfers per element (read for the sum, read for the map,
write), also as % of the MI355X HBM peak (8 TB/s).

Prints one JSON line. `roofline` covers the dominant kernel (the map: it
moves two of the three transfers), timed with HIP events recorded by the
library on the call's stream during an instrumented pass of the same steps;
`cpu_baseline` times the FP64 oracle on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "normalize effective HBM GB/s (% of peak); served req/s with p50/p99 latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_plain_2p28.txt")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2207_00257_amd", "csrc", f) for f in ("nrm_kernels.hip", "nrm_device.h")]


def kernel_source_hash() -> str:
    """sha256 over the plain path's kernel sources (first 16 hex digits)."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(n_bytes_elem_in: int, n: int, params: dict):
    """HBM bytes per map launch from the committed rocprofv3 counter summary,
    or None when absent, taken on a different kernel source, or taken with
    other launch parameters than `params` (the call's)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        if json.loads(vals.get("launch_params", "null")) != params:
            return None
    except ValueError:
        return None
    try:
        return float(vals["map_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(x, budget_s: float = 12.0):
    """The FP64 oracle, as it stands, on the host: whole-array calls on the
    same input until about budget_s seconds of CPU time have been spent."""
    import oracle

    oracle.build()
    n = x.size
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.normalize(x)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 50:
            break
    gbs = 12.0 * n * reps / el / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "%d whole-array oracle calls on the n=2^%d FP32 input (%.1f s, single thread, "
                      "binary64 sequential sum + divide); value uses the same 12 B/element model"
                      % (reps, n.bit_length() - 1, el)}


def host_threads() -> int:
    """Host threads for the multicore CPU leg: the cores this process may run
    on, capped by OMP_NUM_THREADS when set (the machine's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_legs(x, budget_s: float = 4.0):
    """The multicore CPU normalize (binary64 per-thread partials in thread
    order, binary32 divide; csrc/host_baseline.cpp) and a multi-threaded host
    copy of the same bytes (the host memory ceiling), each repeated for about
    budget_s seconds on the same input."""
    import ctypes

    import numpy as np

    from paper_2207_00257_amd import build as nbuild

    if not os.path.exists(nbuild.HOST_LIB):
        nbuild.build_host()
    lib = ctypes.CDLL(nbuild.HOST_LIB)
    lib.nrm_host_normalize_mt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]
    lib.nrm_host_copy_mt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
    threads = host_threads()
    n = x.size
    out = np.empty_like(x)
    s = ctypes.c_double()

    def timed(fn):
        fn()  # first touch of the output pages
        reps, t0 = 0, time.perf_counter()
        times = []
        while True:
            a = time.perf_counter()
            fn()
            times.append(time.perf_counter() - a)
            reps += 1
            if time.perf_counter() - t0 >= budget_s or reps >= 200:
                break
        times.sort()
        return times[len(times) // 2], reps

    t_norm, r_norm = timed(lambda: lib.nrm_host_normalize_mt(out.ctypes.data, x.ctypes.data, n, threads,
                                                             ctypes.byref(s)))
    ref_s = float(np.sum(x, dtype=np.float64))
    t_copy, r_copy = timed(lambda: lib.nrm_host_copy_mt(out.ctypes.data, x.ctypes.data, 4 * n, threads))
    return {
        "threads": threads, "cpu_model": cpu_model(),
        "multicore_normalize": {"value": round(12.0 * n / t_norm / 1e9, 3), "unit": "GB/s",
                                "ms_per_call_median": round(t_norm * 1e3, 3), "calls": r_norm,
                                "sum_rel_err": abs(s.value - ref_s) / ref_s,
                                "what": "hoisted normalize on %d host threads: binary64 per-thread partials "
                                        "added in thread order, binary32 divide; same 12 B/element model"
                                        % threads},
        "host_copy_ceiling": {"value": round(8.0 * n / t_copy / 1e9, 3), "unit": "GB/s",
                              "ms_per_call_median": round(t_copy * 1e3, 3), "calls": r_copy,
                              "what": "memcpy of the 4n-byte input on %d threads (read + write counted)"
                                      % threads},
    }


def gpu_ceilings(inp, out, stream, reps: int = 20):
    """Copy (in -> out) and read-only sweeps of the input with the library's
    ceiling kernels, timed in this run: median per call and GB/s."""
    import torch

    from paper_2207_00257_amd import _lib as L

    lib = L.lib()
    nbytes = inp.numel() * inp.element_size()
    sink = torch.zeros(1 << 16, dtype=torch.int32, device=inp.device)
    res = {}
    for kind, name, dst, grid, moved in ((L.NRM_CEILING_COPY, "copy", out, 16384, 2 * nbytes),
                                         (L.NRM_CEILING_READ, "read", sink, 8192, nbytes)):
        def call():
            L.check(lib.nrm_ceiling(kind, dst.data_ptr(), inp.data_ptr(), nbytes, grid, stream.cuda_stream),
                    "nrm_ceiling")
        call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        med = ts[len(ts) // 2]
        res[name] = {"ms_median": round(med, 5), "GBps": round(moved / (med * 1e-3) / 1e9, 1), "bytes_moved": moved}
    return res


def step_stats(ms_list):
    """Median, p10 and p90 of per-step times (ms)."""
    import numpy as np

    a = np.asarray(ms_list, np.float64)
    return {"median_ms": round(float(np.median(a)), 5), "p10_ms": round(float(np.percentile(a, 10)), 5),
            "p90_ms": round(float(np.percentile(a, 90)), 5), "steps": int(a.size)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--params", default=None,
                    help="JSON file of tuned launch parameters (default: the committed tuning cache "
                         "if it has an entry for this device and size, else the library defaults)")
    ap.add_argument("--workload", default="plain",
                    choices=["plain", "ragged", "short_rows", "serve", "precision", "ladder", "softmax", "nll",
                             "barriers", "sizes", "small"],
                    help="plain: n=2^log2n FP32 (the headline); ragged: 4096 rows, lengths log-uniform "
                         "in [32, 2^20], LogNormal(0,1) FP32, one graph-replayed batched call per step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain device copy of the same size instead (torch copy_: reads and "
                         "writes 4n bytes each); used to scale HBM counter readings")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the normalize hot path here is a single-GPU build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "barriers":
        return bench_barriers(args)
    if args.workload == "nll":
        return bench_nll(args)
    if args.workload == "softmax":
        return bench_softmax(args)
    if args.workload == "ragged":
        return bench_ragged(args)
    if args.workload == "short_rows":
        return bench_short_rows(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "sizes":
        return bench_sizes(args)
    if args.workload == "small":
        return bench_small(args)
    if args.workload == "ladder":
        return bench_ladder(args)

    import numpy as np
    import torch

    from paper_2207_00257_amd import api, synth

    n = 1 << args.log2n
    x = synth.uniform_f32(n, 3)
    dev = torch.device("cuda:0")
    inp = torch.from_numpy(x).to(dev)
    out = torch.empty_like(inp)
    stream = torch.cuda.current_stream(dev)

    if args.copy_calibration:
        for _ in range(args.warmup):
            out.copy_(inp)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            out.copy_(inp)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"copy_calibration": True, "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "ms": ms, "GBps": 8.0 * n / (ms * 1e-3) / 1e9}), flush=True)
        return

    from paper_2207_00257_amd import tune

    params = tune.load_params(args.params, "f32", "f32", "f32", n)
    ctx = api.Context(**params) if params else api.Context()

    for _ in range(args.warmup):
        api.normalize(out, inp, ctx=ctx)
    torch.cuda.synchronize()

    # the timed region: K back-to-back steps between two events, with one
    # event pair per step alongside for the per-step distribution
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(args.steps):
        api.normalize(out, inp, ctx=ctx)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    per_step = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    model_bytes = 12.0 * n
    gbs = model_bytes / (ms * 1e-3) / 1e9

    # instrumented pass: per-kernel durations from HIP events on the call's stream
    ctx.set_timing(True)
    for _ in range(args.steps):
        api.normalize(out, inp, ctx=ctx)
    torch.cuda.synchronize()
    red_ms, map_ms, calls = ctx.kernel_times()
    ctx.set_timing(False)
    red_ms /= calls
    map_ms /= calls

    # dominant kernel: the map (reads in once, writes out once)
    map_bytes = 8.0 * n
    map_gbs = map_bytes / (map_ms * 1e-3) / 1e9
    red_gbs = 4.0 * n / (red_ms * 1e-3) / 1e9
    traffic = measured_traffic(4, n, ctx.get_params())

    # this machine's HBM ceilings over the same bytes, in the same run
    ceil = gpu_ceilings(inp, out, stream)
    t_ceil = ceil["read"]["ms_median"] + ceil["copy"]["ms_median"]  # the reduce's read + the map's copy
    ceilings = dict(ceil, normalize_model_GBps_at_ceiling=round(model_bytes / (t_ceil * 1e-3) / 1e9, 1),
                    normalize_pct_of_measured_ceiling=round(100.0 * t_ceil / step_stats(per_step)["median_ms"], 2),
                    what="read-only sweep and copy of the 4n-byte input with the library's ceiling kernels "
                         "(16-byte non-temporal vectors, map-shaped tiles); a normalize at the ceiling "
                         "would take their sum")
    api.normalize(out, inp, ctx=ctx)  # the output again, for the check below
    torch.cuda.synchronize()

    # spot check of the result against the oracle's definition on a sample
    idx = np.random.Generator(np.random.PCG64(0)).integers(0, n, 4096)
    got = out[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    S = float(np.sum(x.astype(np.float64)))
    rel = float(np.max(np.abs(got - x[idx].astype(np.float64) / S) / (x[idx] / S)))

    line = {
        "metric": METRIC,
        "value": round(gbs, 2),
        "unit": "GB/s",
        "pct_of_peak": round(100.0 * gbs / PEAK_HBM_GBS, 2),
        "elements_per_s": round(n / (ms * 1e-3), 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain normalize, n=2^%d FP32, in~U[0.5,1.5) seed 3, out FP32, "
                               "model 12 B/element" % args.log2n,
                   "n": n, "params": ctx.get_params()},
        "roofline": {"bound": "hbm", "kernel": "map_kernel<f32,f32>",
                     "achieved": round(map_gbs, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(map_gbs / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": map_bytes,
                     "avg_launch_ms": round(map_ms, 5),
                     "reduce_kernel": {"algorithmic_bytes_per_launch": 4.0 * n,
                                       "avg_launch_ms": round(red_ms, 5),
                                       "achieved": round(red_gbs, 2)}},
        "per_step": step_stats(per_step),
        "ceilings": ceilings,
        "sample_max_rel_err": rel,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x)
        line["cpu_baseline"].update(host_legs(x))
    print(json.dumps(line), flush=True)


def bench_ragged(args):
    """Ragged batched workload: one step = one batched call over 4096 rows
    (planner, resident rows, tile phases, replayed from a captured hipGraph).
    Also times the basic C form on the default context, and the same rows as
    one plain normalize call per row, for comparison."""
    import ctypes

    import numpy as np
    import torch

    from paper_2207_00257_amd import _lib as L
    from paper_2207_00257_amd import api, synth, tune

    rows = 4096
    x, offs = synth.ragged_batch(rows, 4)
    total = int(offs[-1])
    dev = torch.device("cuda:0")
    inp = torch.from_numpy(x).to(dev)
    out = torch.empty_like(inp)
    offs_d = torch.from_numpy(offs).to(dev)
    stream = torch.cuda.current_stream(dev)
    ctx = api.Context()
    bp = tune.load_batch_params(args.params) or {}
    bp["graph"] = 1
    ctx.set_batch_params(**bp)
    ctx.batch_reserve(rows, total)
    for _ in range(args.warmup):
        api.normalize_batched(out, inp, offs_d, ctx=ctx)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for k in range(args.steps):
        api.normalize_batched(out, inp, offs_d, ctx=ctx)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    per_step = step_stats([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    if ctx.device_error() != L.NRM_OK:
        raise RuntimeError("device reported invalid rows")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the basic C form a C caller uses: normalize_batched(out, in, offsets,
    # rows) on the default context with the library's own parameters and
    # tuning (it reads offsets[rows] back, which synchronizes the null stream)
    lib = L.lib()
    raw = lambda: L.check(lib.normalize_batched(out.data_ptr(), inp.data_ptr(), offs_d.data_ptr(), rows),
                          "normalize_batched")
    for _ in range(max(4, args.warmup)):
        raw()
    torch.cuda.synchronize()
    null = torch.cuda.default_stream(dev)
    e0.record(null)
    for _ in range(args.steps):
        raw()
    e1.record(null)
    torch.cuda.synchronize()
    raw_ms = e0.elapsed_time(e1) / args.steps
    # spot check: 64 rows against the definition
    pick = np.random.Generator(np.random.PCG64(1)).integers(0, rows, 64)
    o = out.cpu().numpy()
    worst = 0.0
    for r in pick:
        b, e = int(offs[r]), int(offs[r + 1])
        ref = x[b:e].astype(np.float64) / np.sum(x[b:e].astype(np.float64))
        worst = max(worst, float(np.max(np.abs(o[b:e] - ref) / ref)))
    # one plain call per row, from the host, on the same stream
    pctx = api.Context()
    s = stream.cuda_stream
    ip, op = inp.data_ptr(), out.data_ptr()
    bounds = [(int(offs[r]), int(offs[r + 1] - offs[r])) for r in range(rows)]

    def per_row():
        for b, n in bounds:
            st = lib.nrm_normalize_ex(pctx.handle, op + 4 * b, 0, ip + 4 * b, 0, n, 0, s)
            if st:
                raise RuntimeError("per-row call failed: %d" % st)

    per_row()
    torch.cuda.synchronize()
    e0.record(stream)
    per_row()
    e1.record(stream)
    torch.cuda.synchronize()
    per_row_ms = e0.elapsed_time(e1)
    gbs = 12.0 * total / (ms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s",
        "pct_of_peak": round(100.0 * gbs / PEAK_HBM_GBS, 2),
        "elements_per_s": round(total / (ms * 1e-3), 1), "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ragged batched normalize: 4096 rows, lengths log-uniform in [32, 2^20] "
                               "(seed 4), LogNormal(0,1) FP32, int64 CSR offsets, hipGraph replay; "
                               "model 12 B/element", "rows": rows, "elements": total,
                   "batch_params": ctx.get_batch_params()},
        "per_step": per_step,
        "basic_c_form": {"ms": round(raw_ms, 5), "vs_value_pct": round(100.0 * (raw_ms - ms) / ms, 2),
                         "what": "normalize_batched(out, in, offsets, rows): default context and parameters, "
                                 "null stream, offsets[rows] read back per call"},
        "per_row_launch": {"ms": round(per_row_ms, 4), "GBps": round(12.0 * total / (per_row_ms * 1e-3) / 1e9, 2),
                           "speedup_of_batched": round(per_row_ms / ms, 3)},
        "sample_max_rel_err": worst,
    }
    print(json.dumps(line), flush=True)


def bench_short_rows(args):
    """Many short rows: one step = one graph-replayed batched call over
    1,048,576 rows of 256 FP32 elements (U[0.5, 1.5), seed 3). Also timed,
    as medians of per-call events: 65,536 rows of 256, 1,048,576 rows of 64,
    and 200,000 rows of lengths log-uniform in [1, 4096] (LogNormal(0,1),
    seed 8), each with the short rows' kernel (the library's default batch
    parameters) and with that path off (short rows as resident segments, one
    block and one work claim each). Also timed: the row softmax with
    log-sum-exp over the same 1,048,576 rows of 256 (N(0, 4) logits)."""
    import numpy as np
    import torch

    from paper_2207_00257_amd import _lib as L
    from paper_2207_00257_amd import api, synth, tune

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    # the library's own batch parameters (the tuning cache's batched entry is
    # the 4096-row workload's), unless a parameter file is named
    base = tune.load_batch_params(args.params) if args.params else {}

    def make(rows, n=None, lo=1, hi=4096, seed=3):
        if n is not None:
            x = synth.uniform_f32(rows * n, seed)
            offs = np.arange(rows + 1, dtype=np.int64) * n
        else:
            lengths = synth.loguniform_lengths(rows, seed, lo, hi)
            offs = synth.ragged_offsets(lengths)
            x = synth.lognormal_f32(int(offs[-1]), seed + 1, 1.0)
        return x, offs

    def run(x, offs, steps, warmup, **params):
        inp = torch.from_numpy(x).to(dev)
        out = torch.empty_like(inp)
        od = torch.from_numpy(offs).to(dev)
        ctx = api.Context()
        ctx.set_batch_params(**dict(base, graph=1, **params))
        ctx.batch_reserve(offs.size - 1, x.size)
        for _ in range(warmup):
            api.normalize_batched(out, inp, od, ctx=ctx)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        for k in range(steps):
            api.normalize_batched(out, inp, od, ctx=ctx)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        if ctx.device_error() != L.NRM_OK:
            raise RuntimeError("device reported invalid rows")
        per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        res = (ev[0].elapsed_time(ev[-1]) / steps, step_stats(per), out, ctx.get_batch_params())
        ctx.close()
        return res

    rows, n = 1 << 20, 256
    x, offs = make(rows, n)
    ms, per_step, out, bp = run(x, offs, args.steps, args.warmup)
    # spot check: 256 rows against the definition
    o = out.cpu().numpy()
    worst = 0.0
    for r in np.random.Generator(np.random.PCG64(1)).integers(0, rows, 256):
        seg = x[r * n:(r + 1) * n].astype(np.float64)
        worst = max(worst, float(np.max(np.abs(o[r * n:(r + 1) * n] - seg / seg.sum()) / (seg / seg.sum()))))
    del out
    total = rows * n
    gbs = 12.0 * total / (ms * 1e-3) / 1e9
    others = {}
    for name, (xx, oo) in (("65536x256", make(65536, 256)), ("1048576x64", make(1 << 20, 64)),
                           ("200000 log-uniform [1, 4096]", make(200000, None, 1, 4096, 8))):
        t_on = run(xx, oo, 10, 3)[1]["median_ms"]
        t_off = run(xx, oo, 3, 1, wave_max=0)[1]["median_ms"]
        others[name] = {"elements": int(xx.size), "median_ms": t_on, "median_ms_wave_path_off": t_off,
                        "GBps_12B": round(12.0 * xx.size / (t_on * 1e-3) / 1e9, 1)}
    t_off_main = run(x, offs, 3, 1, wave_max=0)[1]["median_ms"]
    # row softmax + log-sum-exp over the same 1,048,576 rows of 256 (N(0, 4) logits)
    xs = synth.normal_f32(rows * n, 9, 2.0)
    inp = torch.from_numpy(xs).to(dev)
    out = torch.empty_like(inp)
    lse = torch.empty(rows, device=dev)
    od = torch.from_numpy(offs).to(dev)
    sctx = api.Context()
    sctx.set_batch_params(**dict(base, graph=1))
    sctx.batch_reserve(rows, xs.size)
    for _ in range(3):
        api.softmax_batched(out, inp, od, lse=lse, ctx=sctx)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
    ev[0].record(stream)
    for k in range(10):
        api.softmax_batched(out, inp, od, lse=lse, ctx=sctx)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    sm_ms = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(10)]))
    r0 = xs[:n].astype(np.float64)
    sm_err = float(np.max(np.abs(out[:n].cpu().numpy() - np.exp(r0 - r0.max()) / np.exp(r0 - r0.max()).sum())))
    sctx.close()
    del inp, out, lse
    line = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s",
        "pct_of_peak": round(100.0 * gbs / PEAK_HBM_GBS, 2),
        "elements_per_s": round(total / (ms * 1e-3), 1), "rows_per_s": round(rows / (ms * 1e-3), 1),
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ragged batched normalize, many short rows: 1,048,576 rows of 256 elements, "
                               "U[0.5,1.5) FP32 (seed 3), int64 CSR offsets, hipGraph replay; model 12 B/element "
                               "(the rows cross HBM twice: 8 B/element actual)",
                   "rows": rows, "elements": total, "batch_params": bp},
        "per_step": per_step,
        "wave_path_off_median_ms": t_off_main,
        "softmax_1048576x256": {"median_ms": round(sm_ms, 5), "GBps_12B": round(12.0 * total / (sm_ms * 1e-3) / 1e9, 1),
                                "row0_max_abs_err": sm_err},
        "others": others,
        "sample_max_rel_err": worst,
    }
    print(json.dumps(line), flush=True)


def bench_softmax(args):
    """Row softmax / log-sum-exp on the ragged scheduler: one step = one
    batched call over 4096 rows (lengths log-uniform in [32, 2^20], the ragged
    workload's) of N(0, 4) binary32 logits, with the log-sum-exp of every
    row, replayed from a captured hipGraph. The batched normalize over the
    same rows (positive inputs) is timed alongside: the two differ only in
    the per-element arithmetic (exp2 in both passes)."""
    import numpy as np
    import torch
    from scipy.special import logsumexp, softmax

    from paper_2207_00257_amd import _lib as L
    from paper_2207_00257_amd import api, synth, tune

    rows = 4096
    x, offs = synth.ragged_logits(rows, 4, sigma=2.0)
    total = int(offs[-1])
    dev = torch.device("cuda:0")
    inp = torch.from_numpy(x).to(dev)
    out = torch.empty_like(inp)
    lse = torch.empty(rows, device=dev)
    offs_d = torch.from_numpy(offs).to(dev)
    stream = torch.cuda.current_stream(dev)
    ctx = api.Context()
    bp = tune.load_batch_params(args.params) or {}
    bp["graph"] = 1
    ctx.set_batch_params(**bp)
    ctx.batch_reserve(rows, total)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms = timed(lambda: api.softmax_batched(out, inp, offs_d, lse=lse, ctx=ctx))
    if ctx.device_error() != L.NRM_OK:
        raise RuntimeError("device reported invalid rows")
    o, ls = out.cpu().numpy(), lse.cpu().numpy()
    # spot check: 64 rows against scipy's binary64 softmax / logsumexp
    pick = np.random.Generator(np.random.PCG64(1)).integers(0, rows, 64)
    worst, worst_lse = 0.0, 0.0
    for r in pick:
        b, e = int(offs[r]), int(offs[r + 1])
        xr = x[b:e].astype(np.float64)
        ref = softmax(xr)
        keep = ref > 2.0 ** -125
        worst = max(worst, float(np.max(np.abs(o[b:e][keep] - ref[keep]) / ref[keep])))
        worst_lse = max(worst_lse, abs(float(ls[r]) - float(logsumexp(xr))))
    pos = np.abs(x) + np.float32(0.5)
    pinp = torch.from_numpy(pos).to(dev)
    norm_ms = timed(lambda: api.normalize_batched(out, pinp, offs_d, ctx=ctx))
    gbs = 12.0 * total / (ms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s",
        "pct_of_peak": round(100.0 * gbs / PEAK_HBM_GBS, 2),
        "elements_per_s": round(total / (ms * 1e-3), 1), "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ragged batched row softmax + log-sum-exp: 4096 rows, lengths log-uniform in "
                               "[32, 2^20] (seed 4), N(0, 4) FP32 logits, int64 CSR offsets, hipGraph replay; "
                               "model 12 B/element", "rows": rows, "elements": total,
                   "batch_params": ctx.get_batch_params()},
        "batched_normalize_same_rows_ms": round(norm_ms, 5),
        "sample_max_rel_err": worst, "sample_max_lse_abs_err": worst_lse,
    }
    print(json.dumps(line), flush=True)


def bench_nll(args, n=1 << 22, c=1000):
    """Forward NLL loss (mean, class weights, 5 % ignored samples): one step
    = one call over n = 2^22 samples of C = 1000 classes. Inputs are drawn on
    the device with a seeded generator (the synth.nll_inputs distributions:
    logp = -Exponential(mean 3), targets uniform, weights U[0.5, 1.5)); the
    16.8 GB logp array is too large to draw on the host. Each kept sample
    gathers one element of its own 4000-byte row, so the traffic is set by
    the gathers' memory sectors, not by the 12 algorithmic bytes."""
    import numpy as np
    import torch
    import torch.nn.functional as F

    from paper_2207_00257_amd import _lib as L
    from paper_2207_00257_amd import api

    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(76)
    logp = torch.empty(n, c, device=dev).exponential_(1.0 / 3.0, generator=g).neg_()
    target = torch.randint(0, c, (n,), device=dev, generator=g)
    target[torch.rand(n, device=dev, generator=g) < 0.05] = -100
    weight = torch.rand(c, device=dev, generator=g) + 0.5
    out = torch.empty(1, device=dev)
    tw = torch.empty(1, device=dev)
    stream = torch.cuda.current_stream(dev)
    ctx = api.Context()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms = timed(lambda: api.nll_loss(logp, target, weight, reduction="mean", out=out, total_weight=tw, ctx=ctx))
    if ctx.device_error() != L.NRM_OK:
        raise RuntimeError("device reported invalid targets")
    got = float(out.cpu()[0])
    # check: the kept samples' gathered values, summed in binary64 on the host
    keep = target != -100
    idx = torch.nonzero(keep).squeeze(1)
    x = logp[idx, target[idx]].double().cpu().numpy()
    wt = weight[target[idx]].double().cpu().numpy()
    ref = float(np.sum(-wt * x) / np.sum(wt))
    torch_ms = timed(lambda: F.nll_loss(logp, target, weight=weight, reduction="mean"))
    kept = int(idx.numel())
    alg_gbs = 12.0 * n / (ms * 1e-3) / 1e9
    sector_gbs = (8.0 * n + 64.0 * kept) / (ms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(n / (ms * 1e-3), 1), "unit": "samples/s",
        "algorithmic_GBps": round(alg_gbs, 2), "sector_model_GBps": round(sector_gbs, 2),
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "forward NLL loss, mean, class weights: N = 2^22 samples, C = 1000 classes, "
                               "logp = -Exponential(mean 3) FP32 [N, C], int64 targets (5 %% ignored), weights "
                               "U[0.5, 1.5); device-side seeded draw; models 12 B/sample algorithmic, 8 B + one "
                               "64-byte sector per kept sample", "n": n, "classes": c},
        "torch_nll_loss_ms": round(torch_ms, 5),
        "rel_err_vs_binary64": abs(got - ref) / ref,
    }
    print(json.dumps(line), flush=True)


def bench_barriers(args):
    """The Fig. 9-shaped tile kernel in its three forms (every barrier as
    analysed; the two barriers Sec. IV-A eliminates removed; also the
    store/load Sec. IV-B promotes to a register), at R = 2^24 rows (hidden
    1 GiB: HBM-bound) and R = 2^16 rows (4 MiB: cache-resident). Inputs
    U[0.5, 1.5) for hidden and 1/16 for input, so repeated in-place calls stay
    bounded. Bytes per row: 64 read + 64 written of hidden, 4 of input, 4 of
    output."""
    import torch

    from paper_2207_00257_amd import api, synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sizes = {}
    for log2r in (24, 16):
        rows = 1 << log2r
        hidden = torch.from_numpy(synth.uniform_f32(rows * 16, 97)).to(dev)
        inp = torch.full((rows,), 0.0625, device=dev)
        out = torch.empty(rows, device=dev)
        reps = args.steps if log2r == 24 else args.steps * 50
        res = {}
        for form in ("all", "eliminated", "promoted", "registers"):
            for _ in range(args.warmup):
                api.layerforward(hidden, inp, out, form=form)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                api.layerforward(hidden, inp, out, form=form)
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            res[form] = {"us": round(us, 3), "GBps": round(136.0 * rows / (us * 1e-6) / 1e9, 1)}
        res["eliminated_speedup"] = round(res["all"]["us"] / res["eliminated"]["us"], 4)
        res["promoted_speedup"] = round(res["all"]["us"] / res["promoted"]["us"], 4)
        res["registers_speedup"] = round(res["all"]["us"] / res["registers"]["us"], 4)
        sizes["rows_2^%d" % log2r] = res
    big = sizes["rows_2^24"]
    line = {
        "metric": METRIC, "value": big["all"]["GBps"], "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(big["all"]["us"] / 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Fig. 9-shaped tile kernel (16 x 16 tiles, 256-thread blocks): R = 2^24 and 2^16 "
                               "rows, hidden U[0.5, 1.5) FP32 [R, 16] updated in place, input 1/16; forms all barriers / "
                               "eliminated / promoted / registers; value = the all-barriers form; model 136 B/row"},
        "forms": sizes,
    }
    print(json.dumps(line), flush=True)


def bench_serve(args, rate=20000.0, warm_s=1.0, measure_s=10.0, pairs=3):
    """Serving workload: an open-loop Poisson trace (20k req/s; n log-uniform
    in [2^8, 2^24]; 70% FP32 / 30% BF16 requests, BF16 in and out) replayed
    with a 64 GiB HBM budget into the continuous-batching server with its
    device queue (one persistent kernel runs the requests of up to 2^20
    elements as they arrive, the longer ones run as plain calls beside it),
    and into the same server in per-request mode (one plain call per request,
    4 slots); three interleaved pairs of 10 s runs. The launch-batched server
    (one batched call per admitted group) and a rate sweep are reported
    beside them. Latency runs from each request's scheduled arrival to the
    observed completion; statistics exclude the first warm_s seconds."""
    import numpy as np
    import torch

    from paper_2207_00257_amd import serve, tune
    import oracle

    torch.cuda.init()
    trace = serve.make_trace(rate, warm_s + measure_s, seed=6)
    k = trace["n"].size
    pool = serve.InputPool(1 << 24, 7)
    offs = pool.offsets(trace["n"], 8)
    ptrs = pool.pointers(trace["in_dt"], offs)
    bp = tune.load_batch_params(args.params, workload="serve")
    warm_ns = int(warm_s * 1e9)
    modes = {
        "device_queue": dict(slots=16, device_queue=True),
        "per_request_launch": dict(slots=4, batching=False, batch_params=bp),
        "launch_batched": dict(slots=4, batching=True, batch_params=bp),
    }

    def run(mode, budget=64 << 30, tr=trace, pt=ptrs, warm_ns=warm_ns):
        n_req = tr["n"].size
        srv = serve.Server(budget_bytes=budget, **modes[mode])
        t0 = srv.replay(np.arange(n_req), pt, tr["n"], tr["in_dt"], tr["out_dt"], tr["t_ns"])
        comps = srv.wait_all(n_req, timeout_s=600)
        st = srv.stats()
        srv.close()
        meas = [c for c in comps if c[2] - t0 >= warm_ns]
        out = serve.latency_stats(meas)
        lat = np.array([c[4] - c[2] for c in meas], np.float64) / 1e3
        ns = np.array([tr["n"][c[0]] for c in meas])
        out["p50_us_n_le_2p20"] = float(np.median(lat[ns <= (1 << 20)]))
        out["p50_us_n_gt_2p23"] = float(np.median(lat[ns > (1 << 23)]))
        out["library_calls"] = st["launches"]
        return out

    # device queue and per-request runs of the same trace, interleaved pair by pair
    pair_runs = []
    for _ in range(pairs):
        pair_runs.append({"device_queue": run("device_queue"), "per_request_launch": run("per_request_launch")})
    dq = pair_runs[0]["device_queue"]
    per_req = pair_runs[0]["per_request_launch"]
    launch_batched = run("launch_batched")
    short = serve.make_trace(rate, 3.0, seed=8)
    spt = pool.pointers(short["in_dt"], pool.offsets(short["n"], 11))
    stress = run("device_queue", tr=short, pt=spt, budget=256 << 20)
    sweep = []
    for r in (10000.0, 50000.0, 100000.0, 200000.0, 400000.0):
        tr = serve.make_trace(r, 1.2, seed=9)
        pt = pool.pointers(tr["in_dt"], pool.offsets(tr["n"], 10))
        sweep.append({"offered_req_per_s": r,
                      **{m: run(m, tr=tr, pt=pt, warm_ns=int(0.2e9)) for m in modes}})
    # results of a sample of requests, held and checked against the oracle
    srv = serve.Server(hold_outputs=True, **modes["device_queue"])
    sel = np.arange(0, k, max(1, k // 64))[:64]
    srv.submit(sel, ptrs[sel], trace["n"][sel], trace["in_dt"][sel], trace["out_dt"][sel])
    worst, worst_bf16 = 0.0, 0.0
    import ctypes
    paths = sorted({ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln})
    hip = ctypes.CDLL(paths[0])
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    for c in srv.wait_all(len(sel)):
        i = c[0]
        n, dt, o = int(trace["n"][i]), int(trace["in_dt"][i]), int(offs[i])
        if dt == 0:
            host = np.empty(n, np.float32)
            hip.hipMemcpy(host.ctypes.data, c[1], 4 * n, 2)
            ref = oracle.normalize(pool.host_f32[o:o + n])
            worst = max(worst, float(np.max(np.abs(host - ref) / ref)))
        else:
            bits = np.empty(n, np.uint16)
            hip.hipMemcpy(bits.ctypes.data, c[1], 2 * n, 2)
            got = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
            ref = oracle.normalize(pool.host_bf16[o:o + n], "bf16")
            ulp = np.exp2(np.floor(np.log2(ref)) - 7)
            worst_bf16 = max(worst_bf16, float(np.max(np.abs(got - ref) / ulp)))
        srv.release(i)
    srv.close()
    line = {
        "metric": METRIC, "value": round(dq["req_per_s"], 1), "unit": "req/s",
        "p50_ms": round(dq["p50_ms"], 4), "p99_ms": round(dq["p99_ms"], 4),
        "n_gpus": 1, "steps": None, "warmup": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": "serving: Poisson %.0f req/s for %.0f s (+%.0f s warm-up), n log-uniform in "
                               "[2^8, 2^24], 70%% FP32 / 30%% BF16 (BF16 in and out), inputs device-resident, "
                               "64 GiB HBM admission budget, open-loop replay, latency from scheduled arrival; "
                               "continuous batching through the device queue (16 slots) against one plain call "
                               "per request (4 slots)" % (rate, measure_s, warm_s), "requests": int(k)},
        "pairs": pair_runs,
        "device_queue_p99_below_per_request_in_every_pair": all(
            r["device_queue"]["p99_ms"] < r["per_request_launch"]["p99_ms"] for r in pair_runs),
        "device_queue": dq, "per_request_launch": per_req, "launch_batched": launch_batched,
        "device_queue_budget_256MiB": stress, "rate_sweep": sweep,
        "sample_max_rel_err_f32": worst, "sample_max_err_bf16_ulps": worst_bf16,
    }
    print(json.dumps(line), flush=True)


def bench_precision(args):
    """Precision workload: n = 2^26 BF16 inputs, values bf16(exp(2 N(0,1)))
    (seed 5), binary32 plain vs Kahan-compensated accumulation, BF16 and FP32
    outputs. For each variant: time per call, effective GB/s (2 x 2 B read +
    sizeof(out) written per element), the sum's error in binary32 ulps and
    the outputs' errors against the FP64 oracle (which sees the quantised
    BF16 inputs)."""
    import numpy as np
    import torch

    import oracle
    from paper_2207_00257_amd import api, synth, tune

    n = 1 << 26
    bits = synth.lognormal_bf16(n, 5, 2.0)
    ref, S_ref = oracle.normalize(bits, "bf16", return_sum=True)
    ref_bf16 = oracle.round_bf16(ref)
    dev = torch.device("cuda:0")
    inp = torch.from_numpy(bits.view(np.int16)).to(dev).view(torch.bfloat16)
    stream = torch.cuda.current_stream(dev)
    ulp_S = float(np.spacing(np.float32(S_ref)))
    results = []
    for accum in ("f32", "kahan"):
        for odt in ("bf16", "f32"):
            out = torch.empty(n, dtype=torch.bfloat16 if odt == "bf16" else torch.float32, device=dev)
            ctx = api.Context()
            tuned = tune.load_params(args.params, "bf16", odt, accum, n)
            if tuned:
                ctx.set_params(**tuned)
            for _ in range(args.warmup):
                api.normalize(out, inp, accum=accum, ctx=ctx)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                api.normalize(out, inp, accum=accum, ctx=ctx)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            S = ctx.last_sum()
            so = 2 if odt == "bf16" else 4
            r = {"accum": accum, "out": odt, "params": "tuned" if tuned else "defaults", "ms": round(ms, 5),
                 "GBps": round((4 + so) * n / (ms * 1e-3) / 1e9, 1),
                 "sum_err_ulps": round(abs(S - S_ref) / ulp_S, 3),
                 "sum_rel_err": abs(S - S_ref) / S_ref}
            if odt == "f32":
                got = out.cpu().numpy().astype(np.float64)
                rel = np.abs(got - ref) / ref
                r.update(max_rel_err=float(rel.max()), mean_rel_err=float(rel.mean()),
                         max_err_f32_ulps=float(np.max(np.abs(got - ref) / np.spacing(ref.astype(np.float32)))))
            else:
                ob = out.view(torch.int16).cpu().numpy().view(np.uint16)
                got = (ob.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
                ulp = np.exp2(np.floor(np.log2(ref)) - 7)
                r.update(max_err_bf16_ulps=float(np.max(np.abs(got - ref) / ulp)),
                         frac_correctly_rounded=float(np.mean(ob == ref_bf16)),
                         max_rel_err=float(np.max(np.abs(got - ref) / ref)))
            results.append(r)
            ctx.close()
    main_r = results[0]
    line = {
        "metric": METRIC, "value": main_r["GBps"], "unit": "GB/s",
        "pct_of_peak": round(100.0 * main_r["GBps"] / PEAK_HBM_GBS, 2), "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_r["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 in, f32 accumulate", "data": "synthetic",
        "config": {"workload": "precision: n=2^26 BF16 in, values bf16(exp(2 N(0,1))) seed 5; plain vs Kahan "
                               "binary32 accumulation; BF16 and FP32 out; errors against the FP64 oracle",
                   "n": n, "oracle_sum": S_ref},
        "variants": results,
    }
    print(json.dumps(line), flush=True)


def bench_small(args, n=1 << 20, reps=50):
    """The small plain case: n = 2^20 FP32, in ~ U[0.5, 1.5) (seed 1). Each
    timed call sits between its own pair of events on the stream (device time
    including the launch) right behind other work on that stream, so the
    clocks are up: warm, behind an untimed call on the same input (in the
    caches); cold, behind a 512 MiB copy with the ceiling kernel, which evicts
    the input from the 256 MB last-level cache and the L2s. Host: wall time
    per call of 200 back-to-back calls through the Python binding (what a
    caller pays)."""
    import numpy as np
    import torch

    from paper_2207_00257_amd import _lib as L
    from paper_2207_00257_amd import api, synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    x = synth.uniform_f32(n, 1)
    inp = torch.from_numpy(x).to(dev)
    out = torch.empty_like(inp)
    ctx = api.Context()
    scratch_a = torch.empty(1 << 27, dtype=torch.float32, device=dev)  # 512 MiB
    scratch_b = torch.empty_like(scratch_a)
    lib = L.lib()

    def flush():
        L.check(lib.nrm_ceiling(L.NRM_CEILING_COPY, scratch_b.data_ptr(), scratch_a.data_ptr(), 4 << 27, 16384,
                                stream.cuda_stream), "nrm_ceiling")

    def timed(cold):
        ts = []
        for _ in range(reps):
            # the timed call follows work on the same stream (no idle gap, so
            # the clocks are up either way): the flush, or an untimed call
            if cold:
                flush()
            else:
                api.normalize(out, inp, ctx=ctx)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            api.normalize(out, inp, ctx=ctx)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return step_stats(ts)

    for _ in range(max(3, args.warmup)):
        api.normalize(out, inp, ctx=ctx)
    torch.cuda.synchronize()
    warm = timed(False)
    cold = timed(True)
    t0 = time.perf_counter()
    for _ in range(200):
        api.normalize(out, inp, ctx=ctx)
    torch.cuda.synchronize()
    host_us = (time.perf_counter() - t0) / 200 * 1e6
    got = out.cpu().numpy().astype(np.float64)
    import oracle

    ref = oracle.normalize(x)
    rel = float(np.max(np.abs(got - ref) / ref))
    model = 12.0 * n
    line = {
        "metric": METRIC, "value": round(model / (warm["median_ms"] * 1e-3) / 1e9, 2), "unit": "GB/s",
        "pct_of_peak": round(100.0 * model / (warm["median_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 2),
        "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": warm["median_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain normalize, n=2^20 FP32, in~U[0.5,1.5) seed 1, the library's default "
                               "path for this size; model 12 B/element", "n": n},
        "warm": warm, "cold": cold, "host_us_per_call": round(host_us, 2),
        "cold_GBps": round(model / (cold["median_ms"] * 1e-3) / 1e9, 2),
        "max_rel_err": rel,
    }
    print(json.dumps(line), flush=True)


def bench_sizes(args):
    """The plain path across sizes: n = 2^16 .. 2^30 FP32, in ~ U[0.5, 1.5)
    (seed 3 per size), default launch parameters. For each size, the time per
    call over back-to-back calls (HIP events around the whole sequence, so
    per-call host overhead counts at small n) and the library's per-kernel
    times. The line's value is the n = 2^20 case's effective GB/s."""
    import torch

    from paper_2207_00257_amd import api

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = api.Context()
    rows = []
    for lg in (16, 18, 20, 22, 24, 26, 27, 28, 29, 30):
        n = 1 << lg
        g = torch.Generator(device=dev)
        g.manual_seed(3)
        inp = torch.rand(n, device=dev, generator=g).add_(0.5)
        out = torch.empty_like(inp)
        for _ in range(args.warmup):
            api.normalize(out, inp, ctx=ctx)
        torch.cuda.synchronize()
        reps = 200 if lg <= 22 else max(args.steps, 5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            api.normalize(out, inp, ctx=ctx)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        # per-kernel times in a pass of their own (the library's events add host work per call)
        ctx.set_timing(True)
        for _ in range(min(reps, 20)):
            api.normalize(out, inp, ctx=ctx)
        torch.cuda.synchronize()
        r, m, c = ctx.kernel_times()
        ctx.set_timing(False)
        rows.append({"log2n": lg, "us_per_call": round(us, 2), "GBps": round(12.0 * n / us / 1e3, 1),
                     "pct_of_peak": round(100.0 * 12.0 * n / us / 1e3 / PEAK_HBM_GBS, 1),
                     "reduce_us": round(r / c * 1e3, 2) if c else None, "map_us": round(m / c * 1e3, 2) if c else None})
        print("n=2^%d %.2f us per call" % (lg, us), file=sys.stderr, flush=True)
        del inp, out
        torch.cuda.empty_cache()
    main_r = next(r for r in rows if r["log2n"] == 20)
    line = {
        "metric": METRIC, "value": main_r["GBps"], "unit": "GB/s", "pct_of_peak": main_r["pct_of_peak"],
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main_r["us_per_call"] / 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain normalize across sizes, n = 2^16..2^30 FP32, in~U[0.5,1.5) seed 3, "
                               "model 12 B/element; value: the n = 2^20 case"},
        "sizes": rows,
    }
    print(json.dumps(line), flush=True)


def bench_ladder(args):
    """The transformation ladder of Fig. 1 on the GPU: the naive form (every
    thread sums the input, O(n^2)), the per-block form (one sum per block of
    256 behind a barrier, O(n^2/256)) and the hoisted form (this library's
    normalize, O(n)), timed at n = 2^10 .. 2^18 (FP32, U[0.5,1.5), seed 12)."""
    import numpy as np
    import torch

    from paper_2207_00257_amd import api, synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for k in (10, 12, 14, 16, 18):
        n = 1 << k
        inp = torch.from_numpy(synth.uniform_f32(n, 12)).to(dev)
        out = torch.empty_like(inp)
        r = {"n": n}
        for form in ("naive", "perblock", "hoisted"):
            def call():
                if form == "hoisted":
                    api.normalize(out, inp)
                else:
                    api.normalize_form(out, inp, form, block=256)
            call()
            torch.cuda.synchronize()
            reps = 3 if (form == "naive" and k >= 16) else 10
            e0.record(stream)
            for _ in range(reps):
                call()
            e1.record(stream)
            torch.cuda.synchronize()
            r[form + "_us"] = round(e0.elapsed_time(e1) / reps * 1e3, 2)
        rows.append(r)
    def slope(key):
        xs = np.log2([r["n"] for r in rows[-3:]])
        ys = np.log2([r[key] for r in rows[-3:]])
        return round(float(np.polyfit(xs, ys, 1)[0]), 2)
    line = {"metric": METRIC, "value": rows[-1]["naive_us"] / rows[-1]["hoisted_us"], "unit": "x (naive/hoisted at n=2^18)",
            "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "transformation ladder: naive O(n^2), per-block O(n^2/256), hoisted O(n); "
                                   "FP32 U[0.5,1.5) seed 12"},
            "ladder": rows,
            "log2_time_slope_last_three": {"naive": slope("naive_us"), "perblock": slope("perblock_us"),
                                           "hoisted": slope("hoisted_us")}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
