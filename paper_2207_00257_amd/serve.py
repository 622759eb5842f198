"""Python driver of the continuous-batching server (nrm_server_* in
include/nrm.h): argument marshalling, request traces, latency statistics.

The server itself (admission by HBM budget, slots, batch formation, launch,
completion) runs natively in libnrm.so's scheduler thread; the open-loop
replay of a trace runs in its replay thread.
"""
from __future__ import annotations

import ctypes
import time
from typing import Optional

import numpy as np

from . import _lib as L
from . import synth

DTYPE_CODES = {"f32": L.NRM_F32, "bf16": L.NRM_BF16, "f16": L.NRM_F16}
ELEM_SIZE = {L.NRM_F32: 4, L.NRM_BF16: 2, L.NRM_F16: 2}


class Server:
    def __init__(self, slots: int = 4, budget_bytes: int = 64 << 30, batching: bool = True, graph: bool = True,
                 hold_outputs: bool = False, max_batch_rows: int = 256, max_batch_elems: int = 1 << 27,
                 accum: str = "f32", batch_params: Optional[dict] = None, arena_bytes: int = 0, device: int = -1,
                 single_plain: bool = True, spread: bool = True, idle_spin_us: int = 1000, min_batch_rows: int = 4,
                 device_queue: bool = False, dq_blocks: int = 0, dq_idle_us: int = 100000,
                 dq_plain_above: int = 1 << 20, dq_slice_us: int = 10000):
        lib = L.lib()
        cfg = L.NrmServerConfig()
        L.check(lib.nrm_server_default_config(ctypes.byref(cfg)), "nrm_server_default_config")
        cfg.slots = slots
        cfg.batching = int(batching)
        cfg.graph = int(graph)
        cfg.accum = {"f32": L.NRM_ACC_F32, "kahan": L.NRM_ACC_KAHAN}[accum]
        cfg.hold_outputs = int(hold_outputs)
        cfg.budget_bytes = budget_bytes
        cfg.arena_bytes = arena_bytes
        cfg.max_batch_rows = max_batch_rows
        cfg.max_batch_elems = max_batch_elems
        cfg.single_plain = int(single_plain)
        cfg.spread = int(spread)
        cfg.idle_spin_us = int(idle_spin_us)
        cfg.min_batch_rows = int(min_batch_rows)
        cfg.device_queue = int(device_queue)
        cfg.dq_blocks = int(dq_blocks)
        cfg.dq_idle_us = int(dq_idle_us)
        cfg.dq_plain_above = int(dq_plain_above)
        cfg.dq_slice_us = int(dq_slice_us)
        if batch_params:
            lib.nrm_default_batch_params(ctypes.byref(cfg.batch_params))
            for k, v in batch_params.items():
                setattr(cfg.batch_params, k, v)
            cfg.batch_params.graph = int(graph)
            cfg.use_batch_params = 1
        h = ctypes.c_void_p()
        L.check(lib.nrm_server_create(ctypes.byref(h), device, ctypes.byref(cfg)), "nrm_server_create")
        self.handle = h
        self.cfg = cfg

    @staticmethod
    def _requests(ids, ptrs, ns, in_dts, out_dts, t_ns):
        k = len(ids)
        arr = (L.NrmRequest * max(k, 1))()
        for i in range(k):
            arr[i].id = int(ids[i])
            arr[i].in_ = int(ptrs[i])
            arr[i].n = int(ns[i])
            arr[i].in_dtype = int(in_dts[i])
            arr[i].out_dtype = int(out_dts[i])
            arr[i].t_arrival_ns = int(t_ns[i])
        return arr, k

    def submit(self, ids, ptrs, ns, in_dts, out_dts):
        arr, k = self._requests(ids, ptrs, ns, in_dts, out_dts, [0] * len(ids))
        L.check(L.lib().nrm_server_submit(self.handle, arr, k), "nrm_server_submit")

    def replay(self, ids, ptrs, ns, in_dts, out_dts, t_offsets_ns) -> int:
        arr, k = self._requests(ids, ptrs, ns, in_dts, out_dts, t_offsets_ns)
        t0 = ctypes.c_int64()
        L.check(L.lib().nrm_server_replay(self.handle, arr, k, ctypes.byref(t0)), "nrm_server_replay")
        self._keep = arr
        return t0.value

    def poll(self, max_n: int = 65536):
        buf = (L.NrmCompletion * max_n)()
        cnt = ctypes.c_int64()
        L.check(L.lib().nrm_server_poll(self.handle, buf, max_n, ctypes.byref(cnt)), "nrm_server_poll")
        return [(buf[i].id, buf[i].out, buf[i].t_arrival_ns, buf[i].t_launch_ns, buf[i].t_done_ns, buf[i].status)
                for i in range(cnt.value)]

    def release(self, rid: int) -> None:
        L.check(L.lib().nrm_server_release(self.handle, int(rid)), "nrm_server_release")

    def stats(self) -> dict:
        c = L.NrmServerCounters()
        L.check(L.lib().nrm_server_stats(self.handle, ctypes.byref(c)), "nrm_server_stats")
        return {f: getattr(c, f) for f, _ in L.NrmServerCounters._fields_}

    def wait_all(self, expected: int, timeout_s: float = 60.0, on_done=None):
        """Poll until `expected` completions have been seen; returns them."""
        out, t_end = [], time.time() + timeout_s
        while len(out) < expected:
            got = self.poll()
            if on_done:
                for c in got:
                    on_done(c)
            out.extend(got)
            if len(out) >= expected:
                break
            if time.time() > t_end:
                raise TimeoutError("server: %d of %d requests completed; %s" % (len(out), expected, self.stats()))
            time.sleep(0.0005)
        return out

    def close(self) -> None:
        if self.handle:
            L.check(L.lib().nrm_server_destroy(self.handle), "nrm_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_trace(rate: float, duration_s: float, seed: int, lo: int = 1 << 8, hi: int = 1 << 24,
               bf16_frac: float = 0.3):
    """Open-loop request trace: Poisson arrivals at `rate` per second, sizes
    log-uniform in [lo, hi], a fraction bf16_frac of BF16 requests (BF16 in,
    BF16 out), the rest FP32."""
    t = synth.poisson_arrivals(rate, duration_s, seed)
    k = t.size
    n = synth.loguniform_lengths(k, seed + 1, lo, hi)
    is_bf16 = np.random.Generator(np.random.PCG64(seed + 2)).random(k) < bf16_frac
    dts = np.where(is_bf16, L.NRM_BF16, L.NRM_F32).astype(np.int32)
    return {"t_ns": (t * 1e9).astype(np.int64), "n": n, "in_dt": dts, "out_dt": dts.copy()}


class InputPool:
    """Device-resident request inputs: each request reads a slice of a
    pre-filled pool (U[0.5, 1.5) values), at a 256-byte aligned offset."""

    def __init__(self, max_n: int, seed: int, device="cuda:0", span: int = 1 << 25):
        import torch

        self.span = max(span, max_n)
        x = synth.uniform_f32(self.span, seed)
        self.f32 = torch.from_numpy(x).to(device)
        self.bf16 = torch.from_numpy(synth.f32_to_bf16_bits(x).view(np.int16)).to(device).view(torch.bfloat16)
        self.host_f32 = x
        self.host_bf16 = synth.f32_to_bf16_bits(x)
        self.max_n = max_n

    def offsets(self, ns: np.ndarray, seed: int) -> np.ndarray:
        g = np.random.Generator(np.random.PCG64(seed))
        room = self.span - ns
        return (g.integers(0, np.maximum(room // 64, 1)) * 64).astype(np.int64)  # 64 elements = 256 B (f32)

    def pointers(self, dts: np.ndarray, offs: np.ndarray) -> np.ndarray:
        base = np.where(dts == L.NRM_F32, self.f32.data_ptr(), self.bf16.data_ptr()).astype(np.int64)
        size = np.where(dts == L.NRM_F32, 4, 2)
        return base + offs * size


def latency_stats(comps, t0_ns=None) -> dict:
    lat = np.array([c[4] - c[2] for c in comps], np.float64) / 1e6  # ms
    done = np.array([c[4] for c in comps], np.int64)
    arr = np.array([c[2] for c in comps], np.int64)
    span_s = (done.max() - arr.min()) / 1e9 if len(comps) > 1 else float("nan")
    return {"requests": len(comps), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "req_per_s": len(comps) / span_s,
            "span_s": span_s, "failed": int(sum(1 for c in comps if c[5] != 0))}
