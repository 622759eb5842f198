"""GPU tests of the continuous-batching server: results against the oracle,
each result identical alone and in the mix, admission under a tight HBM
budget, open-loop replay, and the per-request launch mode."""
import numpy as np
import pytest
import torch

import oracle
from paper_2207_00257_amd import _lib as L
from paper_2207_00257_amd import serve
from parity_util import assert_f32_close, assert_within_ulp, bf16_bits_to_f64, ulp_bf16

pytestmark = pytest.mark.gpu


_hip = None


def loaded_hip():
    """The HIP runtime this process already uses (the copy libnrm.so is bound
    to), opened by its path so that no second runtime is loaded."""
    global _hip
    if _hip is None:
        import ctypes

        L.lib()
        paths = sorted({ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln})
        assert len(paths) == 1, paths
        _hip = ctypes.CDLL(paths[0])
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip


def read_out(ptr, n, dt):
    """Copy a device output (raw pointer) to the host."""
    esz = 4 if dt == L.NRM_F32 else 2
    host = np.empty(n, np.float32 if dt == L.NRM_F32 else np.uint16)
    if n:
        assert loaded_hip().hipMemcpy(host.ctypes.data, ptr, n * esz, 2) == 0  # device to host
    return host


def check_against_oracle(pool, n, dt, off, host_out, what):
    if dt == L.NRM_F32:
        ref = oracle.normalize(pool.host_f32[off:off + n])
        assert_f32_close(host_out, ref, what=what)
    else:
        ref = oracle.normalize(pool.host_bf16[off:off + n], "bf16")
        assert_within_ulp(bf16_bits_to_f64(host_out), ref, ulp_bf16, what=what)


def make_requests(count, seed, hi=1 << 18):
    tr = serve.make_trace(rate=1e6, duration_s=count / 1e6 * 1.5, seed=seed, lo=1, hi=hi)
    k = min(count, tr["n"].size)
    return tr["n"][:k], tr["in_dt"][:k]


@pytest.mark.parametrize("batching,spread", [(True, True), (True, False), (False, True)])
def test_mix_matches_oracle_and_alone(batching, spread):
    ns, dts = make_requests(120, 5)
    pool = serve.InputPool(int(ns.max()), 7)
    offs = pool.offsets(ns, 8)
    ptrs = pool.pointers(dts, offs)
    ids = np.arange(ns.size)
    # groups of any size run the batched kernels, so that alone and in the mix
    # the same kernel computes each request (bitwise comparison below)
    srv = serve.Server(slots=3, hold_outputs=True, batching=batching, max_batch_rows=32, single_plain=False,
                       spread=spread, min_batch_rows=1)
    srv.submit(ids, ptrs, ns, dts, dts)
    comps = srv.wait_all(ns.size)
    assert sorted(c[0] for c in comps) == list(ids)
    mixed = {}
    for c in comps:
        i = c[0]
        assert c[5] == L.NRM_OK
        mixed[i] = read_out(c[1], int(ns[i]), int(dts[i]))
        check_against_oracle(pool, int(ns[i]), int(dts[i]), int(offs[i]), mixed[i], "request %d" % i)
        srv.release(i)
    assert srv.stats()["budget_used"] == 0
    srv.close()
    # each request alone, on a fresh server with the same configuration
    solo = serve.Server(slots=1, hold_outputs=True, batching=batching, max_batch_rows=32, single_plain=False,
                        min_batch_rows=1)
    for i in range(0, ns.size, 7):
        solo.submit([i], [ptrs[i]], [ns[i]], [dts[i]], [dts[i]])
        (c,) = solo.wait_all(1)
        alone = read_out(c[1], int(ns[i]), int(dts[i]))
        assert np.array_equal(alone, mixed[i]), "request %d differs alone and in the mix" % i
        solo.release(i)
    solo.close()


def test_tight_budget_admission():
    """A 4 MiB budget: requests of up to 256 KiB in + out queue for memory,
    all complete, and the budget is never exceeded."""
    ns, dts = make_requests(200, 11, hi=1 << 15)
    pool = serve.InputPool(int(ns.max()), 12, span=1 << 20)
    offs = pool.offsets(ns, 13)
    ptrs = pool.pointers(dts, offs)
    budget = 4 << 20
    srv = serve.Server(slots=4, budget_bytes=budget, max_batch_rows=16)
    srv.submit(np.arange(ns.size), ptrs, ns, dts, dts)
    seen_max = 0
    done = []
    while len(done) < ns.size:
        st = srv.stats()
        seen_max = max(seen_max, st["budget_used"])
        done.extend(srv.poll())
    assert seen_max <= budget
    assert srv.stats()["budget_used"] == 0
    srv.close()


def test_request_larger_than_budget_is_rejected():
    pool = serve.InputPool(1 << 16, 14, span=1 << 16)
    srv = serve.Server(slots=1, budget_bytes=1 << 16)
    with pytest.raises(L.NrmError):
        srv.submit([0], [pool.f32.data_ptr()], [1 << 16], [L.NRM_F32], [L.NRM_F32])
    srv.close()


def test_open_loop_replay_completes_and_measures_latency():
    tr = serve.make_trace(rate=20000, duration_s=0.1, seed=21, hi=1 << 20)
    k = tr["n"].size
    pool = serve.InputPool(int(tr["n"].max()), 22)
    offs = pool.offsets(tr["n"], 23)
    ptrs = pool.pointers(tr["in_dt"], offs)
    srv = serve.Server(slots=4)
    srv.replay(np.arange(k), ptrs, tr["n"], tr["in_dt"], tr["out_dt"], tr["t_ns"])
    comps = srv.wait_all(k, timeout_s=60)
    stats = serve.latency_stats(comps)
    assert stats["requests"] == k
    assert all(c[4] >= c[2] for c in comps)  # done after scheduled arrival
    assert stats["p50_ms"] > 0 and stats["p99_ms"] >= stats["p50_ms"]
    srv.close()


def test_single_request_plain_policy_matches_oracle():
    """With single_plain (the default), a lone request takes the plain path and
    a group the batched one: both within the error bound of the oracle."""
    ns, dts = make_requests(40, 31)
    pool = serve.InputPool(int(ns.max()), 32)
    offs = pool.offsets(ns, 33)
    ptrs = pool.pointers(dts, offs)
    srv = serve.Server(slots=2, hold_outputs=True, max_batch_rows=8)
    for i in range(0, 10):  # one at a time: groups of one
        srv.submit([i], [ptrs[i]], [ns[i]], [dts[i]], [dts[i]])
        (c,) = srv.wait_all(1)
        check_against_oracle(pool, int(ns[i]), int(dts[i]), int(offs[i]), read_out(c[1], int(ns[i]), int(dts[i])),
                             "alone %d" % i)
        srv.release(i)
    srv.submit(np.arange(10, 40), ptrs[10:], ns[10:], dts[10:], dts[10:])
    for c in srv.wait_all(30):
        i = c[0]
        check_against_oracle(pool, int(ns[i]), int(dts[i]), int(offs[i]), read_out(c[1], int(ns[i]), int(dts[i])),
                             "grouped %d" % i)
        srv.release(i)
    srv.close()


# ---- device queue (one persistent kernel, no launch per request) ------------------------


def dq_requests(count, seed, hi=1 << 22):
    """Sizes log-uniform in [1, hi] (requests above 2^20 take the two-pass
    long form), 70 % FP32 / 30 % BF16."""
    tr = serve.make_trace(rate=1e6, duration_s=count / 1e6 * 1.5, seed=seed, lo=1, hi=hi)
    k = min(count, tr["n"].size)
    return tr["n"][:k], tr["in_dt"][:k]


# dq_plain_above: 2^20 (the default) runs the requests above 2^20 as plain
# calls beside the kernel; 2^25 keeps every request in the kernel (the
# two-pass long form)
@pytest.mark.parametrize("accum,plain_above", [("f32", 1 << 20), ("kahan", 1 << 20), ("f32", 1 << 25),
                                               ("kahan", 1 << 25)])
def test_device_queue_mix_matches_oracle_and_alone(accum, plain_above):
    ns, dts = dq_requests(150, 41)
    # the boundaries of the two forms: one element, one resident segment, the
    # largest resident request, the smallest long one, a ragged long one
    edge = np.array([1, 1 << 14, 1 << 20, (1 << 20) + 1, 3 * (1 << 20) + 17], np.int64)
    ns = np.concatenate([ns, edge])
    dts = np.concatenate([dts, np.full(edge.size, L.NRM_F32, np.int32)])
    pool = serve.InputPool(int(ns.max()), 42)
    offs = pool.offsets(ns, 43)
    offs[-1] += 5  # an input that does not start on a 16-byte boundary
    ptrs = pool.pointers(dts, offs)
    ids = np.arange(ns.size)
    srv = serve.Server(slots=16, hold_outputs=True, device_queue=True, accum=accum, dq_plain_above=plain_above)
    srv.submit(ids, ptrs, ns, dts, dts)
    comps = srv.wait_all(ns.size, timeout_s=120)
    assert sorted(c[0] for c in comps) == list(ids)
    mixed = {}
    for c in comps:
        i = c[0]
        assert c[5] == L.NRM_OK, "request %d status %d" % (i, c[5])
        mixed[i] = read_out(c[1], int(ns[i]), int(dts[i]))
        check_against_oracle(pool, int(ns[i]), int(dts[i]), int(offs[i]), mixed[i], "request %d (n=%d)" % (i, ns[i]))
        srv.release(i)
    assert srv.stats()["budget_used"] == 0
    srv.close()
    solo = serve.Server(slots=1, hold_outputs=True, device_queue=True, accum=accum, dq_plain_above=plain_above)
    for i in list(range(0, ns.size, 9)) + list(range(ns.size - edge.size, ns.size)):
        solo.submit([i], [ptrs[i]], [ns[i]], [dts[i]], [dts[i]])
        (c,) = solo.wait_all(1, timeout_s=60)
        alone = read_out(c[1], int(ns[i]), int(dts[i]))
        assert np.array_equal(alone, mixed[i]), "request %d differs alone and in the mix" % i
        solo.release(i)
    solo.close()


@pytest.mark.parametrize("plain_above", [1 << 20, 1 << 25])
def test_device_queue_largest_request_and_empty(plain_above):
    """n = 2^25 (in the kernel: 1024 parts, the largest request) and n = 0; a
    request above 2^25 is rejected before it is queued."""
    n = 1 << 25
    pool = serve.InputPool(n, 44, span=n)
    srv = serve.Server(slots=2, hold_outputs=True, device_queue=True, dq_plain_above=plain_above)
    srv.submit([0, 1], [pool.f32.data_ptr(), pool.f32.data_ptr()], [n, 0], [L.NRM_F32] * 2, [L.NRM_F32] * 2)
    comps = {c[0]: c for c in srv.wait_all(2, timeout_s=60)}
    assert comps[0][5] == L.NRM_OK and comps[1][5] == L.NRM_OK
    got = read_out(comps[0][1], n, L.NRM_F32)
    idx = np.random.Generator(np.random.PCG64(45)).integers(0, n, 4096)
    ref = oracle.normalize(pool.host_f32[:n])
    assert_f32_close(got[idx], ref[idx], what="n=2^25 sampled")
    np.testing.assert_allclose(float(np.sum(got, dtype=np.float64)), 1.0, rtol=1e-5)
    with pytest.raises(L.NrmError):
        srv.submit([2], [pool.f32.data_ptr()], [n + 1], [L.NRM_F32], [L.NRM_F32])
    srv.close()


def test_device_queue_restarts_after_idle_exit():
    """With a 2 ms idle limit the kernel ends between bursts; the next request
    starts it again, and results stay exact across the restarts."""
    ns, dts = dq_requests(30, 46, hi=1 << 21)
    pool = serve.InputPool(int(ns.max()), 47)
    offs = pool.offsets(ns, 48)
    ptrs = pool.pointers(dts, offs)
    srv = serve.Server(slots=4, hold_outputs=True, device_queue=True, dq_idle_us=2000, dq_plain_above=1 << 25)
    import time

    for burst in range(3):
        sel = list(range(burst * 10, burst * 10 + 10))
        srv.submit(sel, ptrs[sel], ns[sel], dts[sel], dts[sel])
        for c in srv.wait_all(len(sel), timeout_s=60):
            i = c[0]
            assert c[5] == L.NRM_OK
            check_against_oracle(pool, int(ns[i]), int(dts[i]), int(offs[i]), read_out(c[1], int(ns[i]), int(dts[i])),
                                 "burst %d request %d" % (burst, i))
            srv.release(i)
        time.sleep(0.02)  # ten idle limits: the kernel has ended
    srv.close()


def test_device_queue_open_loop_replay():
    tr = serve.make_trace(rate=20000, duration_s=0.2, seed=49, hi=1 << 22)
    k = tr["n"].size
    pool = serve.InputPool(int(tr["n"].max()), 50)
    offs = pool.offsets(tr["n"], 51)
    ptrs = pool.pointers(tr["in_dt"], offs)
    srv = serve.Server(slots=16, device_queue=True)
    srv.replay(np.arange(k), ptrs, tr["n"], tr["in_dt"], tr["out_dt"], tr["t_ns"])
    comps = srv.wait_all(k, timeout_s=60)
    stats = serve.latency_stats(comps)
    assert stats["requests"] == k and stats["failed"] == 0
    assert all(c[4] >= c[2] for c in comps)
    srv.close()


def test_device_queue_plain_calls_do_not_wait_behind_the_kernel():
    """Requests above dq_plain_above run as plain calls on the slots' own
    streams while the persistent kernel stays resident (a 2 s idle limit): a
    slot stream on the kernel's hardware queue would hold its call until the
    kernel ended, so every call finishing well inside the idle limit shows
    the set-up probe kept them apart."""
    import time

    n = (1 << 21) + 3
    pool = serve.InputPool(n, 52, span=n + 1024)
    # no slice: the kernel stays until its 2 s idle limit, so a call stuck
    # behind it would show
    srv = serve.Server(slots=16, hold_outputs=True, device_queue=True, dq_idle_us=2000000, dq_slice_us=0)
    srv.submit([0], [pool.f32.data_ptr()], [1 << 12], [L.NRM_F32], [L.NRM_F32])  # the kernel is resident
    srv.wait_all(1, timeout_s=30)
    srv.release(0)
    for burst in range(3):
        ids = list(range(1 + 16 * burst, 17 + 16 * burst))
        t0 = time.perf_counter()
        srv.submit(ids, [pool.f32.data_ptr()] * 16, [n] * 16, [L.NRM_F32] * 16, [L.NRM_F32] * 16)
        comps = srv.wait_all(16, timeout_s=30)
        took = time.perf_counter() - t0
        assert took < 0.3, "burst %d took %.3f s: a plain call waited behind the kernel" % (burst, took)
        for c in comps:
            assert c[5] == L.NRM_OK
            srv.release(c[0])
    got = read_out(comps[0][1], n, L.NRM_F32)
    assert_f32_close(got, oracle.normalize(pool.host_f32[:n]), what="plain call beside the kernel")
    srv.close()


def test_device_queue_every_dtype_pair():
    """All nine input/output dtype pairs through the kernel (resident
    segments and, with every request in the kernel, the two-pass form)."""
    pairs = [(i, o) for i in (L.NRM_F32, L.NRM_BF16, L.NRM_F16) for o in (L.NRM_F32, L.NRM_BF16, L.NRM_F16)]
    ns = np.array([1000, (1 << 14) + 7, (1 << 20) - 3, (1 << 21) + 11], np.int64)
    x = np.random.Generator(np.random.PCG64(53)).random(int(ns.max()) + 64).astype(np.float32) + np.float32(0.5)
    dev = {L.NRM_F32: torch.from_numpy(x).cuda(),
           L.NRM_BF16: torch.from_numpy(x).to(torch.bfloat16).cuda(),
           L.NRM_F16: torch.from_numpy(x).to(torch.float16).cuda()}
    # the oracle sees each request's stored values: binary32, or the 2-byte bit patterns
    host = {L.NRM_F32: (x, "f32"), L.NRM_BF16: (dev[L.NRM_BF16].cpu().view(torch.int16).numpy().view(np.uint16), "bf16"),
            L.NRM_F16: (dev[L.NRM_F16].cpu().view(torch.int16).numpy().view(np.uint16), "f16")}
    srv = serve.Server(slots=8, hold_outputs=True, device_queue=True, dq_plain_above=1 << 25)
    rid = 0
    for di, do in pairs:
        ids = list(range(rid, rid + ns.size))
        rid += ns.size
        srv.submit(ids, [dev[di].data_ptr()] * ns.size, ns, [di] * ns.size, [do] * ns.size)
        for c in srv.wait_all(ns.size, timeout_s=60):
            assert c[5] == L.NRM_OK
            n = int(ns[c[0] - ids[0]])
            esz = 4 if do == L.NRM_F32 else 2
            raw = np.empty(n * esz, np.uint8)
            assert loaded_hip().hipMemcpy(raw.ctypes.data, c[1], n * esz, 2) == 0
            if do == L.NRM_F32:
                got = raw.view(np.float32).astype(np.float64)
            elif do == L.NRM_BF16:
                got = bf16_bits_to_f64(raw.view(np.uint16))
            else:
                got = raw.view(np.float16).astype(np.float64)
            ref = oracle.normalize(host[di][0][:n], host[di][1])
            # binary32 out: 4e-6 relative; a 2-byte output: one ulp of its
            # format (FP16 below 2^-14 is subnormal, with spacing 2^-24)
            if do == L.NRM_F32:
                tol = 4e-6 * ref
            elif do == L.NRM_BF16:
                tol = ulp_bf16(ref)
            else:
                tol = np.maximum(np.exp2(np.floor(np.log2(ref)) - 10), 2.0 ** -24)
            bad = np.abs(got - ref) > tol
            assert not bad.any(), "pair %d->%d n=%d: %d outputs outside the bound" % (di, do, n, int(bad.sum()))
            srv.release(c[0])
    srv.close()


def test_device_queue_slice_bounds_the_wait_of_other_streams():
    """A kernel queued on a stream that shares the persistent kernel's
    hardware queue waits for that launch to end: with a 2 ms slice (and a
    2 s idle limit) work on a dozen fresh streams, one of which shares it on
    this runtime, finishes within milliseconds, and requests keep
    completing across the slices."""
    import time

    pool = serve.InputPool(1 << 16, 54, span=1 << 16)
    srv = serve.Server(slots=4, hold_outputs=True, device_queue=True, dq_idle_us=2000000, dq_slice_us=2000)
    srv.submit([0], [pool.f32.data_ptr()], [1 << 12], [L.NRM_F32], [L.NRM_F32])
    srv.wait_all(1, timeout_s=30)
    srv.release(0)
    x = torch.rand(1 << 12, device="cuda")
    torch.cuda.synchronize()
    worst = 0.0
    for _ in range(12):
        st = torch.cuda.Stream()
        t0 = time.perf_counter()
        with torch.cuda.stream(st):
            y = x * 2.0
        st.synchronize()
        worst = max(worst, time.perf_counter() - t0)
        assert torch.equal(y, x * 2.0)
    assert worst < 0.2, "a fresh stream waited %.3f s behind the kernel" % worst
    for i in range(1, 41):  # requests across several slices
        srv.submit([i], [pool.f32.data_ptr()], [1 << 15], [L.NRM_F32], [L.NRM_F32])
        (c,) = srv.wait_all(1, timeout_s=30)
        assert c[5] == L.NRM_OK
        check_against_oracle(pool, 1 << 15, L.NRM_F32, 0, read_out(c[1], 1 << 15, L.NRM_F32), "request %d" % i)
        srv.release(i)
        time.sleep(0.001)
    srv.close()
