"""GPU parity of the plain normalize path against the FP64 oracle.

Every call goes through the C ABI (libnrm.so via the ctypes binding). Inputs
are seeded synthetic arrays from paper_2207_00257_amd.synth; expected values
come from oracle/ only.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2207_00257_amd import _lib as L
from paper_2207_00257_amd import api, synth
from parity_util import (REL_F32, assert_f32_close, assert_within_ulp, bf16_bits_to_f64, ulp_bf16,
                         ulp_f16)

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run_f32(x: np.ndarray, ctx=None, accum="f32") -> np.ndarray:
    inp = gpu(x)
    out = torch.empty_like(inp)
    api.normalize(out, inp, accum=accum, ctx=ctx)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_plain_2p20_uniform_matches_oracle():
    """n = 2^20 FP32, in ~ U[0.5, 1.5), seed 1."""
    x = synth.uniform_f32(1 << 20, 1)
    got = run_f32(x)
    ref = oracle.normalize(x)
    assert_f32_close(got, ref, what="n=2^20")


def test_brute_force_naive_1024():
    """n = 1024 against the naive per-thread-sum form of Fig. 1 (O(n^2))."""
    x = synth.uniform_f32(1024, 2)
    got = run_f32(x)
    ref = oracle.normalize_naive(x)
    assert_f32_close(got, ref, what="naive n=1024")


SMALL_CTX = {}


MODES = {"default": {}, "two_kernels": dict(small_n=0, resident_n=0), "resident_2p20": dict(small_n=0, resident_n=1 << 20),
         "small": dict(small_n=65536, resident_n=0)}


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 33, 63, 64, 65, 255, 256, 257, 1000,
                               1023, 1025, 4095, 4097, 65535, 65536, 65537, 262143, 1000003, 1 << 20,
                               (1 << 20) + 1, 3000017])
def test_sizes_and_ragged_tails(n, mode):
    """Every size through the default launch (n <= 2^18: one block per 4096
    elements, each held in registers across the exchange of sums; above: two
    kernels), with both one-launch forms off (two kernels), with the
    resident form up to 2^20 (the single published total beyond 64
    segments), and with the one-block form (n <= 2^16)."""
    if mode not in SMALL_CTX:
        SMALL_CTX[mode] = api.Context(**MODES[mode])
    x = synth.lognormal_f32(n, 10 + n % 97, 1.0)
    assert_f32_close(run_f32(x, SMALL_CTX[mode]), oracle.normalize(x), what="n=%d %s" % (n, mode))


@pytest.mark.parametrize("accum", ["f32", "kahan"])
@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_small_path_two_byte_inputs(accum, dt):
    """2-byte inputs through the one-block form (8 vectors per thread), to
    binary32 and to their own type, at the form's capacity and below; then
    the same through the default launch."""
    small = api.Context(small_n=65536, resident_n=0)
    for n, ctx in ((1, small), (777, small), (65536, small), (65536, None), (200_001, None)):
        x = synth.lognormal_f32(n, 20 + n % 13, 1.0)
        bits = synth.f32_to_bf16_bits(x) if dt == "bf16" else synth.f32_to_f16_bits(x)
        tdt = torch.bfloat16 if dt == "bf16" else torch.float16
        inp = gpu(bits.view(np.int16)).view(tdt)
        ref = oracle.normalize(bits, dt)
        out32 = torch.empty(n, device=DEV)
        api.normalize(out32, inp, accum=accum, ctx=ctx)
        out16 = torch.empty_like(inp)
        api.normalize(out16, inp, accum=accum, ctx=ctx)
        torch.cuda.synchronize()
        assert_f32_close(out32.cpu().numpy(), ref, what="%s->f32 n=%d" % (dt, n))
        if dt == "bf16":
            got = bf16_bits_to_f64(out16.view(torch.int16).cpu().numpy().view(np.uint16))
            assert_within_ulp(got, ref, ulp_bf16, what="bf16->bf16 n=%d" % n)
        else:
            from parity_util import ulp_f16
            assert_within_ulp(out16.cpu().numpy().astype(np.float64), ref, ulp_f16, what="f16->f16 n=%d" % n)


def test_small_path_in_place_and_last_sum():
    x = synth.uniform_f32(50_000, 21)
    ctx = api.Context(small_n=65536)
    t = gpu(x)
    api.normalize(t, t, ctx=ctx)
    torch.cuda.synchronize()
    assert_f32_close(t.cpu().numpy(), oracle.normalize(x), what="in place")
    _, s_ref = oracle.normalize(x, return_sum=True)
    assert abs(ctx.last_sum() - s_ref) <= 4e-6 * s_ref
    ctx.close()


def test_single_element_is_exactly_one():
    for v in (1.0, 3.5, 1e-30, 7e30):
        assert run_f32(np.array([v], np.float32))[0] == 1.0


@pytest.mark.parametrize("c", [1.0, 0.5, 2.0])
def test_constant_input_exact_at_power_of_two(c):
    """Constant c at n = 2^k: every partial is an exact multiple of c, so the
    binary32 sum is exact and every output is exactly 2^-k."""
    for k in list(range(0, 21)) + [24]:
        n = 1 << k
        got = run_f32(np.full(n, c, np.float32))
        assert np.all(got == np.float32(2.0 ** -k)), (c, k)


def test_power_of_two_scaling_is_bitwise_invariant():
    x = synth.lognormal_f32(777777, 21, 1.0)
    ref = run_f32(x)
    for m in (-10, 3, 17):
        y = (x * np.float32(2.0 ** m)).astype(np.float32)
        assert np.array_equal(run_f32(y), ref), m


def test_deterministic_repeat():
    x = synth.uniform_f32(5_000_011, 22)
    a = run_f32(x)
    b = run_f32(x)
    assert np.array_equal(a, b)


def test_n_zero_writes_nothing():
    out = torch.full((16,), 7.0, device=DEV)
    inp = torch.ones(16, device=DEV)
    st = L.lib().nrm_normalize_ex(None, out.data_ptr(), 0, inp.data_ptr(), 0, 0, 0, None)
    torch.cuda.synchronize()
    assert st == L.NRM_OK
    assert torch.all(out == 7.0)


def test_raw_fp32_entry_point():
    """normalize(out, in, n) itself: FP32, default context, null stream."""
    x = synth.uniform_f32(123457, 23)
    inp = gpu(x)
    out = torch.empty_like(inp)
    torch.cuda.synchronize()
    st = L.lib().normalize(out.data_ptr(), inp.data_ptr(), x.size)
    torch.cuda.synchronize()
    assert st == L.NRM_OK
    assert_f32_close(out.cpu().numpy(), oracle.normalize(x), what="raw normalize")


def test_in_place():
    x = synth.lognormal_f32(1_000_001, 24, 1.0)
    t = gpu(x)
    api.normalize(t, t)
    torch.cuda.synchronize()
    assert_f32_close(t.cpu().numpy(), oracle.normalize(x), what="in place")


@pytest.mark.parametrize("n", [100_003, 3_000_011], ids=["one_launch", "two_kernels"])
@pytest.mark.parametrize("in_off,out_off", [(1, 1), (2, 2), (3, 3), (1, 0), (0, 3), (2, 1)])
def test_misaligned_pointers(in_off, out_off, n):
    """Element offsets inside larger buffers: unaligned heads, and outputs whose
    alignment differs from the input's (element-wise stores)."""
    x = synth.lognormal_f32(n, 25, 1.0)
    big_in = torch.zeros(n + 8, device=DEV)
    big_in[in_off:in_off + n] = gpu(x)
    big_out = torch.full((n + 8,), -1.0, device=DEV)
    inp = big_in[in_off:in_off + n]
    out = big_out[out_off:out_off + n]
    api.normalize(out, inp)
    torch.cuda.synchronize()
    o = big_out.cpu().numpy()
    assert_f32_close(o[out_off:out_off + n], oracle.normalize(x), what="offsets %d/%d" % (in_off, out_off))
    assert np.all(o[:out_off] == -1.0) and np.all(o[out_off + n:] == -1.0), "wrote outside out"


def test_rejects_element_misaligned_pointer():
    inp = torch.ones(64, device=DEV)
    out = torch.empty(64, device=DEV)
    st = L.lib().nrm_normalize_ex(None, out.data_ptr(), 0, inp.data_ptr() + 1, 0, 10, 0, None)
    assert st == L.NRM_EINVAL


def test_mixed_signs_within_condition_scaled_bound():
    n = 200_003
    g = np.random.Generator(np.random.PCG64(26))
    x = (g.standard_normal(n) + 0.05).astype(np.float32)
    ref = oracle.normalize(x)
    kappa = np.abs(x.astype(np.float64)).sum() / abs(x.astype(np.float64).sum())
    assert_f32_close(run_f32(x), ref, tol=REL_F32 * kappa, what="mixed signs")


PARAM_SETS = [
    dict(block=64, unroll=1, map_block=64, map_unroll=1),
    dict(block=128, unroll=2, map_unroll=8),
    dict(block=512, unroll=8, map_block=1024, map_unroll=2),
    dict(block=1024, unroll=4, map_unroll=4, grid=300, map_grid=77),
    dict(layout=1, map_layout=1),
    dict(layout=1, map_layout=1, reverse_map=1, unroll=8),
    dict(reverse_map=1),
    dict(reduce_nt=0, map_nt=0, grid=1, map_grid=1),
    dict(max_height=24, grid=4),
    dict(max_height=40, grid=65536, map_grid=65536),
    dict(layout=1, grid=8, unroll=8, block=1024, max_height=40),
    dict(layout=0, grid=3, unroll=1, block=64, max_height=40),
    dict(reduce_keep_mib=1, reverse_map=1),
    dict(reduce_keep_mib=4096, reverse_map=0, layout=0),
    dict(reduce_keep_mib=0),                          # chunked, every load non-temporal
    dict(reduce_keep_mib=2, grid=7, unroll=2),        # the temporal tail starts inside a block's chunk
    # tiled layout (2) and the fused combine
    dict(layout=2, map_layout=2),
    dict(layout=2, map_layout=2, fused_combine=1, grid=1024, map_grid=1024, block=1024, unroll=2,
         map_block=1024, map_unroll=2, tile_log2=15),
    dict(layout=2, map_layout=2, fused_combine=1, tile_log2=10, block=64, unroll=1, map_block=64, map_unroll=1),
    dict(layout=2, tile_log2=22, max_height=24, grid=4),
    dict(layout=2, map_layout=2, tile_log2=22, grid=1, map_grid=1, fused_combine=1),
    dict(fused_combine=1),
    dict(fused_combine=1, max_height=24, grid=4096),
    dict(fused_combine=1, layout=0, map_layout=0, reverse_map=1),
    dict(layout=2, map_layout=1, reduce_keep_mib=1, fused_combine=1, map_nt=0, reduce_nt=0),
]


@pytest.mark.parametrize("params", PARAM_SETS, ids=lambda p: ",".join("%s=%s" % kv for kv in p.items()))
def test_launch_parameters(params):
    ctx = api.Context(**dict(params, small_n=0, resident_n=0))  # the two kernels at every size
    for n, seed in ((1_000_003, 30), (4097, 31), (1 << 20, 32)):
        x = synth.lognormal_f32(n, seed, 1.0)
        assert_f32_close(run_f32(x, ctx), oracle.normalize(x), what="%s n=%d" % (params, n))
    ctx.close()


def test_kahan_f32():
    x = synth.lognormal_f32(1 << 22, 33, 2.0)
    ref = oracle.normalize(x)
    assert_f32_close(run_f32(x, accum="kahan"), ref, what="kahan")


@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_bf16_in_bf16_out(accum):
    bits = synth.lognormal_bf16((1 << 20) + 5, 40, 2.0)
    inp = gpu(bits.view(np.int16)).view(torch.bfloat16)
    out = torch.empty_like(inp)
    api.normalize(out, inp, accum=accum)
    torch.cuda.synchronize()
    got = bf16_bits_to_f64(out.view(torch.int16).cpu().numpy().view(np.uint16))
    ref = oracle.normalize(bits, "bf16")
    assert_within_ulp(got, ref, ulp_bf16, what="bf16->bf16 " + accum)


@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_bf16_in_f32_out(accum):
    bits = synth.lognormal_bf16((1 << 20) + 3, 41, 2.0)
    inp = gpu(bits.view(np.int16)).view(torch.bfloat16)
    out = torch.empty(inp.numel(), device=DEV)
    api.normalize(out, inp, accum=accum)
    torch.cuda.synchronize()
    assert_f32_close(out.cpu().numpy(), oracle.normalize(bits, "bf16"), what="bf16->f32 " + accum)


def test_f16_in_f32_and_f16_out():
    x = synth.lognormal_f32(300_001, 42, 1.0)
    bits = synth.f32_to_f16_bits(x)
    inp = gpu(bits.view(np.int16)).view(torch.float16)
    ref = oracle.normalize(bits, "f16")
    out32 = torch.empty(inp.numel(), device=DEV)
    api.normalize(out32, inp)
    out16 = torch.empty_like(inp)
    api.normalize(out16, inp)
    torch.cuda.synchronize()
    assert_f32_close(out32.cpu().numpy(), ref, what="f16->f32")
    assert_within_ulp(out16.cpu().numpy().astype(np.float64), ref, ulp_f16, what="f16->f16")


def test_f32_in_bf16_out():
    x = synth.uniform_f32(1 << 20, 43)
    inp = gpu(x)
    out = torch.empty(x.size, dtype=torch.bfloat16, device=DEV)
    api.normalize(out, inp)
    torch.cuda.synchronize()
    got = bf16_bits_to_f64(out.view(torch.int16).cpu().numpy().view(np.uint16))
    assert_within_ulp(got, oracle.normalize(x), ulp_bf16, what="f32->bf16")


def test_full_size_2p28_default_launch():
    """n = 2^28 FP32, U[0.5, 1.5), seed 3, in the default launch configuration
    (the one the benchmark times): every output against the oracle, and the
    outputs sum to one."""
    n = 1 << 28
    x = synth.uniform_f32(n, 3)
    inp = gpu(x)
    out = torch.empty_like(inp)
    api.normalize(out, inp)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    del inp, out
    ref = oracle.normalize(x)
    for b in range(0, n, 1 << 24):
        assert_f32_close(got[b:b + (1 << 24)], ref[b:b + (1 << 24)], what="2^28 block %d" % b)
    s = np.sum(got.astype(np.float64))
    assert abs(s - 1.0) <= 4e-6 + n * 2.0 ** -53


@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_precision_workload_full_size(accum):
    """The precision workload at its full size and in the launch configuration
    the benchmark times (each variant's tuned shape, else the defaults):
    n = 2^26 BF16 inputs bf16(exp(2 N(0,1))) (seed 5). Every output against
    the FP64 oracle on the same quantised inputs: BF16 outputs within one BF16
    ulp, FP32 outputs within the binary32 tolerance."""
    from paper_2207_00257_amd import tune

    n = 1 << 26
    bits = synth.lognormal_bf16(n, 5, 2.0)
    ref = oracle.normalize(bits, "bf16")
    inp = gpu(bits.view(np.int16)).view(torch.bfloat16)
    for odt, tdt in (("bf16", torch.bfloat16), ("f32", torch.float32)):
        ctx = api.Context(**(tune.load_params(None, "bf16", odt, accum, n) or {}))
        out = torch.empty(n, dtype=tdt, device=DEV)
        api.normalize(out, inp, accum=accum, ctx=ctx)
        torch.cuda.synchronize()
        what = "2^26 bf16->%s %s" % (odt, accum)
        if odt == "bf16":
            got = bf16_bits_to_f64(out.view(torch.int16).cpu().numpy().view(np.uint16))
            assert_within_ulp(got, ref, ulp_bf16, what=what)
        else:
            assert_f32_close(out.cpu().numpy(), ref, what=what)
        ctx.close()


def test_parameter_validation():
    ctx = api.Context()
    good = ctx.get_params()
    for bad in (dict(block=96), dict(map_block=2048), dict(unroll=3), dict(map_unroll=16), dict(grid=0),
                dict(layout=3), dict(map_layout=-1), dict(max_height=23), dict(max_height=41),
                dict(reverse_map=2), dict(map_nt=-1), dict(tile_log2=9), dict(tile_log2=23),
                dict(fused_combine=2), dict(small_n=-1), dict(reduce_keep_mib=-1), dict(reduce_keep_mib=4097),
                dict(resident_n=-1), dict(resident_n=(1 << 20) + 1)):
        with pytest.raises(L.NrmError):
            ctx.set_params(**bad)
        assert ctx.get_params() == good, bad
    p = L.NrmParams()
    assert L.lib().nrm_default_params(ctypes.byref(p)) == L.NRM_OK
    assert {f: getattr(p, f) for f, _ in L.NrmParams._fields_ if f != "reserved"} == good
    p.small_n = -1
    assert L.lib().nrm_set_params(ctx.handle, ctypes.byref(p)) == L.NRM_EINVAL
    p.small_n = (1 << 16) + 1
    assert L.lib().nrm_set_params(ctx.handle, ctypes.byref(p)) == L.NRM_EINVAL
    ctx.close()


def test_too_many_blocks_is_rejected():
    """The combine handles at most 65536 reduce blocks; a launch shape that
    would need more is an argument error, not a wrong result."""
    # 64 threads x 1 vector x 80 iterations per block (the most max_height
    # 24 allows) x 65536 blocks covers 1,342,177,280 elements; use more. The
    # buffers are real allocations, so even a launch would stay in bounds.
    n = 1_400_000_000
    ctx = api.Context(block=64, unroll=1, max_height=24, grid=65536)
    x = torch.empty(n, device=DEV)
    out = torch.empty_like(x)
    with pytest.raises(L.NrmError):
        api.normalize(out, x, ctx=ctx)
    ctx.close()
    del x, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_sum_error_bound(accum):
    """The hoisted sum itself: plain binary32 within the tree-height bound
    gamma_62 * S (non-negative inputs), compensated within a few ulps."""
    bits = synth.lognormal_bf16(1 << 24, 44, 2.0)
    _, S_ref = oracle.normalize(bits, "bf16", return_sum=True)
    inp = gpu(bits.view(np.int16)).view(torch.bfloat16)
    out = torch.empty(inp.numel(), device=DEV)
    ctx = api.Context()
    api.normalize(out, inp, accum=accum, ctx=ctx)
    S = ctx.last_sum()
    ulp = float(np.spacing(np.float32(S_ref)))
    if accum == "kahan":
        assert abs(S - S_ref) <= 2 * ulp, (S, S_ref)
    else:
        u = 2.0 ** -24
        assert abs(S - S_ref) <= 62 * u / (1 - 62 * u) * S_ref + ulp, (S, S_ref)
    ctx.close()


@pytest.mark.parametrize("form", ["naive", "perblock"])
@pytest.mark.parametrize("n", [1, 33, 1000, 1024, 4097, 65536])
def test_unhoisted_forms_match_oracle(form, n):
    """Fig. 1's naive and per-block forms on the GPU agree with the oracle's
    naive and per-block forms (and so with the hoisted result)."""
    x = synth.uniform_f32(n, 60 + n % 89)
    inp = gpu(x)
    out = torch.empty_like(inp)
    api.normalize_form(out, inp, form, block=256 if n > 64 else 64)
    torch.cuda.synchronize()
    ref = oracle.normalize_naive(x) if form == "naive" else oracle.normalize_perblock(x, 256)
    assert_f32_close(out.cpu().numpy(), ref, what="%s n=%d" % (form, n))


@pytest.mark.parametrize("accum", ["f32", "kahan"])
@pytest.mark.parametrize("layout", [1, 2])
def test_fused_combine_is_bitwise_the_ticket_combine(accum, layout):
    """With at most 1024 reduce blocks the fused combine (every map block
    merges the partials) uses the same fixed merge order as the last-block
    combine: outputs and the sum are bitwise equal."""
    bits = synth.lognormal_bf16((1 << 22) + 77, 45, 2.0)
    inp = gpu(bits.view(np.int16)).view(torch.bfloat16)
    outs, sums = [], []
    for fused in (0, 1):
        ctx = api.Context(layout=layout, map_layout=layout, grid=1000, fused_combine=fused)
        out = torch.empty(inp.numel(), device=DEV)
        api.normalize(out, inp, accum=accum, ctx=ctx)
        sums.append(ctx.last_sum())
        outs.append(out.cpu().numpy())
        ctx.close()
    assert sums[0] == sums[1]
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    assert_f32_close(outs[1], oracle.normalize(bits, "bf16"), what="fused " + accum)


@pytest.mark.parametrize("in_off,out_off", [(1, 1), (3, 3), (1, 0), (0, 3)])
def test_fused_tiled_misaligned_pointers(in_off, out_off):
    """Offsets from 128-byte alignment with the tiled layout and the fused
    combine (a differently aligned out falls back to the element-wise map and
    the last-block combine)."""
    n = 300_017
    x = synth.lognormal_f32(n + 8, 46, 1.0)
    base_in = gpu(x)
    base_out = torch.zeros(n + 8, device=DEV)
    ctx = api.Context(layout=2, map_layout=2, fused_combine=1, tile_log2=12, resident_n=0)
    api.normalize(base_out[out_off:out_off + n], base_in[in_off:in_off + n], ctx=ctx)
    torch.cuda.synchronize()
    got = base_out.cpu().numpy()
    assert_f32_close(got[out_off:out_off + n], oracle.normalize(x[in_off:in_off + n]), what="fused misaligned")
    assert not got[:out_off].any() and not got[out_off + n:].any()
    ctx.close()


RESIDENT_SIZES = [65537, 4096 * 17 - 1, 4096 * 17, 4096 * 17 + 1, 4096 * 64, 4096 * 64 + 1, 4096 * 100 + 33,
                  (1 << 20) - 1, 1 << 20]


@pytest.mark.parametrize("accum", ["f32", "kahan"])
def test_resident_plain_sizes_dtypes_and_repeats(accum):
    """The one-launch mid-size form (a block per 4096 elements, exchanging
    tagged sums): sizes at segment boundaries up to 2^20, FP32 / BF16 / FP16,
    three calls in a row on one context (each call's partials carry its own
    call number, so a later call never takes an earlier one's) with the same
    bits each time, and the sum it leaves for nrm_get_last_sum. resident_n =
    2^20: up to 64 segments every block reads every partial, beyond that the
    last block to arrive publishes the total."""
    ctx = api.Context(resident_n=1 << 20)
    for n in RESIDENT_SIZES:
        x = synth.lognormal_f32(n, 300 + n % 89, 1.0)
        ref = oracle.normalize(x)
        first = None
        for _ in range(3):
            got = run_f32(x, ctx, accum=accum)
            assert_f32_close(got, ref, what="resident n=%d %s" % (n, accum))
            if first is None:
                first = got
            assert np.array_equal(got.view(np.uint32), first.view(np.uint32)), "repeat differs at n=%d" % n
        s = ctypes.c_float()
        L.check(L.lib().nrm_get_last_sum(ctx.handle, None, ctypes.byref(s)), "nrm_get_last_sum")
        S = float(np.sum(x, dtype=np.float64))
        assert abs(s.value - S) <= 4e-6 * S, (n, s.value, S)
    bits = synth.lognormal_bf16((1 << 19) + 7, 310, 2.0)
    inp = gpu(bits.view(np.int16)).view(torch.bfloat16)
    out = torch.empty_like(inp)
    api.normalize(out, inp, accum=accum, ctx=ctx)
    torch.cuda.synchronize()
    ref = oracle.normalize(bits, "bf16")
    got = bf16_bits_to_f64(out.view(torch.int16).cpu().numpy().view(np.uint16))
    assert_within_ulp(got, ref, ulp_bf16, what="resident bf16")
    h = synth.f32_to_f16_bits(synth.lognormal_f32(300_001, 311, 1.0))
    inp = gpu(h.view(np.int16)).view(torch.float16)
    out = torch.empty(inp.numel(), dtype=torch.float32, device=DEV)
    api.normalize(out, inp, accum=accum, ctx=ctx)
    torch.cuda.synchronize()
    assert_f32_close(out.cpu().numpy(), oracle.normalize(h, "f16"), what="resident f16->f32")
    assert ctx.device_error() == L.NRM_OK
    ctx.close()


def test_resident_plain_matches_alternating_contexts_and_in_place():
    """Two contexts used in turn (each its own call numbers) and an in-place
    call: all within the bound, and the same bits as a fresh context."""
    n = 4096 * 150 + 5
    x = synth.lognormal_f32(n, 320, 1.0)
    ref = oracle.normalize(x)
    a, b = api.Context(resident_n=1 << 20), api.Context(resident_n=1 << 20)
    outs = [run_f32(x, c) for c in (a, b, a, b, a)]
    for o in outs:
        assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32))
    assert_f32_close(outs[0], ref, what="alternating contexts")
    t = gpu(x)
    api.normalize(t, t, ctx=a)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy().view(np.uint32), outs[0].view(np.uint32)), "in place differs"
    a.close()
    b.close()


def test_default_context_shared_by_host_threads():
    """Four host threads call normalize through the default context (ctx NULL)
    on the null stream at once, each with its own size (so each first call
    adds its own tuning-cache key and may grow the shared workspace): the
    context's host state is locked per call and the null stream orders the
    device work, so every thread's result matches the oracle."""
    import threading

    sizes = [(1 << 19) + 3, (1 << 21) + 5, (1 << 22) + 7, (1 << 23) + 11]
    xs = [synth.lognormal_f32(n, 500 + i, 1.0) for i, n in enumerate(sizes)]
    ins = [gpu(x) for x in xs]
    outs = [torch.empty_like(t) for t in ins]
    errors = []
    start = threading.Barrier(len(sizes))

    def work(i):
        try:
            start.wait()
            for _ in range(30):
                api.normalize(outs[i], ins[i], stream=0)
        except Exception as e:  # reported below, on the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(sizes))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, x in enumerate(xs):
        assert_f32_close(outs[i].cpu().numpy(), oracle.normalize(x), what="thread %d n=%d" % (i, sizes[i]))
