"""The allocation-free plain entry point, nrm_normalize_noalloc, called
through the C ABI: its outputs must equal nrm_normalize_ex's on a context
with the device's default parameters (same kernels, same plan: the same bits),
and the oracle's within the FP32 bound, on two calls in a row with the second
smaller; sizes beyond its scratch are rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2207_00257_amd import _lib as L
from paper_2207_00257_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

F32_TOL = 4e-6  # per-element relative bound of the FP32 path (gamma_62 + u)


_CODES = {torch.float32: L.NRM_F32, torch.bfloat16: L.NRM_BF16, torch.float16: L.NRM_F16}


def _noalloc(out, inp, accum=L.NRM_ACC_F32):
    s = torch.cuda.current_stream(inp.device).cuda_stream
    return L.lib().nrm_normalize_noalloc(out.data_ptr(), _CODES[out.dtype], inp.data_ptr(),
                                         _CODES[inp.dtype], inp.numel(), accum, s)


def _ex(ctx, out, inp, accum=L.NRM_ACC_F32):
    s = torch.cuda.current_stream(inp.device).cuda_stream
    return L.lib().nrm_normalize_ex(ctx, out.data_ptr(), _CODES[out.dtype], inp.data_ptr(),
                                    _CODES[inp.dtype], inp.numel(), accum, s)


@pytest.fixture(scope="module")
def ctx():
    # the device's default parameters, set explicitly: no tuning-cache entries
    h = ctypes.c_void_p()
    L.check(L.lib().nrm_create(ctypes.byref(h), 0), "nrm_create")
    p = L.NrmParams()
    L.check(L.lib().nrm_get_params(h, ctypes.byref(p)), "nrm_get_params")
    L.check(L.lib().nrm_set_params(h, ctypes.byref(p)), "nrm_set_params")
    yield h
    L.check(L.lib().nrm_destroy(h), "nrm_destroy")


@pytest.mark.parametrize("sizes,accum", [
    (((1 << 24) + 1021, (1 << 20) + 3), L.NRM_ACC_F32),   # two-kernel path, then a smaller one
    (((1 << 22) + 77, 40000), L.NRM_ACC_KAHAN),           # two-kernel path, then the one-block path
    ((70000, 513), L.NRM_ACC_F32),                         # both just around the one-block limit
    (((1 << 20), (1 << 17) + 3), L.NRM_ACC_KAHAN),         # the one-launch mid-size form twice
])
def test_matches_existing_entry_point_twice(ctx, sizes, accum):
    for k, n in enumerate(sizes):
        print("noalloc: call %d n=%d accum=%d" % (k, n, accum), flush=True)
        x = synth.uniform_f32(n, 40 + k)
        inp = torch.from_numpy(x).cuda()
        got = torch.full_like(inp, float("nan"))
        want = torch.full_like(inp, float("nan"))
        L.check(_noalloc(got, inp, accum), "nrm_normalize_noalloc")
        L.check(_ex(ctx, want, inp, accum), "nrm_normalize_ex")
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        assert np.array_equal(g.view(np.uint32), w.view(np.uint32)), "differs from nrm_normalize_ex"
        ref = oracle.normalize(x)
        rel = np.max(np.abs(g.astype(np.float64) - ref) / np.abs(ref))
        assert rel <= F32_TOL, rel


def test_bf16_in_bf16_out_then_smaller(ctx):
    for k, n in enumerate(((1 << 23) + 9, (1 << 18) + 5)):
        x = synth.lognormal_bf16(n, 60 + k)
        inp = torch.from_numpy(x.view(np.int16)).cuda().view(torch.bfloat16)
        got = torch.empty_like(inp)
        want = torch.empty_like(inp)
        L.check(_noalloc(got, inp), "nrm_normalize_noalloc")
        L.check(_ex(ctx, want, inp), "nrm_normalize_ex")
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int16), want.view(torch.int16))


def test_rejects_sizes_beyond_scratch_without_launching():
    # 2^34 + 2^20 elements need more than 16384 reduce blocks; the pointers are
    # only compared on the host (nothing is read or written at them)
    n = (1 << 34) + (1 << 20)
    base = torch.empty(64, dtype=torch.float32, device="cuda").data_ptr()
    out = base + 4 * n + 4096  # disjoint from [base, base + 4 n) on the host's arithmetic
    st = L.lib().nrm_normalize_noalloc(out, L.NRM_F32, base, L.NRM_F32, n, L.NRM_ACC_F32, None)
    assert st == L.NRM_EINVAL
    assert b"16384" in L.lib().nrm_last_error()
    torch.cuda.synchronize()


def test_argument_errors():
    lib = L.lib()
    assert lib.nrm_normalize_noalloc(None, 0, None, 0, -1, 0, None) == L.NRM_EINVAL
    assert lib.nrm_normalize_noalloc(None, 0, None, 0, 0, 0, None) == L.NRM_OK
    assert lib.nrm_normalize_noalloc(4096, 0, 4100, 0, 10, 0, None) == L.NRM_EOVERLAP
