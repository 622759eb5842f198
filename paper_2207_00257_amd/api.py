"""Python binding of libnrm.so: argument marshalling only.

Every step of normalize runs in the library's HIP kernels. torch provides the
device memory (tensors) and the stream (the current stream of the tensor's
device); this module passes their raw pointers through the C ABI.

    normalize(out, inp)               out = inp / inp.sum(), FP32 or BF16/FP16
    Context(...).normalize(out, inp)  with launch parameters and timing
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import _lib as L

_ACCUM = {"f32": L.NRM_ACC_F32, "kahan": L.NRM_ACC_KAHAN}


def _dtype_code(t) -> int:
    import torch

    codes = {torch.float32: L.NRM_F32, torch.bfloat16: L.NRM_BF16, torch.float16: L.NRM_F16}
    if t.dtype not in codes:
        raise TypeError("unsupported dtype %s (float32, bfloat16, float16)" % t.dtype)
    return codes[t.dtype]


def _stream_of(t) -> int:
    import torch

    return torch.cuda.current_stream(t.device).cuda_stream


def _check_tensors(out, inp):
    if not inp.is_cuda or not out.is_cuda:
        raise ValueError("normalize needs device tensors (the library has no CPU path)")
    if inp.device != out.device:
        raise ValueError("in and out are on different devices")
    if not inp.is_contiguous() or not out.is_contiguous():
        raise ValueError("in and out must be contiguous")
    if inp.numel() != out.numel():
        raise ValueError("in and out differ in length")


class Context:
    """An nrm_ctx: owns device workspace and launch parameters."""

    def __init__(self, device: int = -1, **params):
        h = ctypes.c_void_p()
        L.check(L.lib().nrm_create(ctypes.byref(h), int(device)), "nrm_create")
        self.handle = h
        if params:
            self.set_params(**params)

    def close(self) -> None:
        if self.handle:
            L.check(L.lib().nrm_destroy(self.handle), "nrm_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> dict:
        p = L.NrmParams()
        L.check(L.lib().nrm_get_params(self.handle, ctypes.byref(p)), "nrm_get_params")
        return {f: getattr(p, f) for f, _ in L.NrmParams._fields_ if f != "reserved"}

    def set_params(self, **kw) -> None:
        cur = self.get_params()
        unknown = set(kw) - set(cur)
        if unknown:
            raise ValueError("unknown parameters %s" % sorted(unknown))
        cur.update(kw)
        p = L.NrmParams(**cur)
        L.check(L.lib().nrm_set_params(self.handle, ctypes.byref(p)), "nrm_set_params")

    def normalize(self, out, inp, accum: str = "f32", stream: Optional[int] = None):
        return normalize(out, inp, accum=accum, ctx=self, stream=stream)

    def normalize_batched(self, out, inp, offsets, accum: str = "f32", stream: Optional[int] = None):
        return normalize_batched(out, inp, offsets, accum=accum, ctx=self, stream=stream)

    def softmax_batched(self, out, inp, offsets, lse=None, stream: Optional[int] = None):
        return softmax_batched(out, inp, offsets, lse=lse, ctx=self, stream=stream)

    def normalize_rows(self, pairs, accum: str = "f32", stream: Optional[int] = None):
        return normalize_rows(pairs, accum=accum, ctx=self, stream=stream)

    def get_batch_params(self) -> dict:
        p = L.NrmBatchParams()
        L.check(L.lib().nrm_get_batch_params(self.handle, ctypes.byref(p)), "nrm_get_batch_params")
        return {f: getattr(p, f) for f, _ in L.NrmBatchParams._fields_ if f != "reserved"}

    def set_batch_params(self, **kw) -> None:
        cur = self.get_batch_params()
        unknown = set(kw) - set(cur)
        if unknown:
            raise ValueError("unknown batch parameters %s" % sorted(unknown))
        cur.update(kw)
        p = L.NrmBatchParams(**cur)
        L.check(L.lib().nrm_set_batch_params(self.handle, ctypes.byref(p)), "nrm_set_batch_params")

    def batch_reserve(self, max_rows: int, max_elems: int) -> None:
        L.check(L.lib().nrm_batch_reserve(self.handle, int(max_rows), int(max_elems)), "nrm_batch_reserve")

    def device_error(self, stream: Optional[int] = None) -> int:
        """Synchronize and return the status of the device-side row checks
        (NRM_OK or NRM_EDEVICE), clearing the flag."""
        return device_error(self, stream)

    def batch_times(self):
        """(total_ms, calls) summed over the batched calls recorded since timing was enabled."""
        t, c = ctypes.c_double(), ctypes.c_int64()
        L.check(L.lib().nrm_batch_times(self.handle, ctypes.byref(t), ctypes.byref(c)), "nrm_batch_times")
        return t.value, c.value

    def last_sum(self, stream: Optional[int] = None) -> float:
        """The hoisted sum of the last plain call (synchronizes the stream)."""
        import torch

        v = ctypes.c_float()
        s = torch.cuda.current_stream().cuda_stream if stream is None else stream
        L.check(L.lib().nrm_get_last_sum(self.handle, s, ctypes.byref(v)), "nrm_get_last_sum")
        return v.value

    def set_timing(self, enable: bool) -> None:
        L.check(L.lib().nrm_set_timing(self.handle, int(bool(enable))), "nrm_set_timing")

    def kernel_times(self):
        """(reduce_ms, map_ms, calls) summed over the calls recorded since timing was enabled."""
        r, m, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        L.check(L.lib().nrm_kernel_times(self.handle, ctypes.byref(r), ctypes.byref(m), ctypes.byref(c)),
                "nrm_kernel_times")
        return r.value, m.value, c.value


def normalize(out, inp, accum: str = "f32", ctx: Optional[Context] = None, stream: Optional[int] = None):
    """out[i] = inp[i] / sum(inp) on the device, enqueued on the current stream.

    inp: float32 / bfloat16 / float16 device tensor; out: same length, any of
    those dtypes (out may be inp itself). accum: "f32" or "kahan"."""
    _check_tensors(out, inp)
    if accum not in _ACCUM:
        raise ValueError("accum must be 'f32' or 'kahan'")
    s = _stream_of(inp) if stream is None else stream
    st = L.lib().nrm_normalize_ex(ctx.handle if ctx else None, out.data_ptr(), _dtype_code(out),
                                  inp.data_ptr(), _dtype_code(inp), inp.numel(), _ACCUM[accum], s)
    L.check(st, "nrm_normalize_ex")
    return out


def normalize_batched(out, inp, offsets, accum: str = "f32", ctx: Optional[Context] = None,
                      stream: Optional[int] = None):
    """Ragged batched normalize, CSR form: row r is inp[offsets[r]:offsets[r+1]]
    (and the same slice of out), normalized on its own. offsets: int64 device
    tensor of rows + 1 entries. The device checks every row against the
    tensors' length; see device_error()."""
    import torch

    _check_tensors(out, inp)
    if accum not in _ACCUM:
        raise ValueError("accum must be 'f32' or 'kahan'")
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 device tensor")
    if offsets.device != inp.device:
        raise ValueError("offsets is on another device")
    rows = offsets.numel() - 1
    if rows < 0:
        raise ValueError("offsets needs rows + 1 >= 1 entries")
    s = _stream_of(inp) if stream is None else stream
    st = L.lib().nrm_normalize_batched_ex(ctx.handle if ctx else None, out.data_ptr(), _dtype_code(out),
                                          inp.data_ptr(), _dtype_code(inp), offsets.data_ptr(), rows,
                                          inp.numel(), _ACCUM[accum], s)
    L.check(st, "nrm_normalize_batched_ex")
    return out


def softmax_batched(out, inp, offsets, lse=None, ctx: Optional[Context] = None, stream: Optional[int] = None):
    """Row softmax and log-sum-exp of a ragged batch, CSR form: row r is
    inp[offsets[r]:offsets[r+1]]; out gets exp(x) / sum exp over the row and,
    if given, lse[r] = log(sum exp) of the row (-inf for an empty row).
    Binary32 device tensors; offsets: int64 device tensor of rows + 1 entries;
    lse: float32 device tensor of rows entries, or None."""
    import torch

    _check_tensors(out, inp)
    if inp.dtype != torch.float32 or out.dtype != torch.float32:
        raise ValueError("softmax_batched takes float32 in and out")
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 device tensor")
    if offsets.device != inp.device:
        raise ValueError("offsets is on another device")
    rows = offsets.numel() - 1
    if rows < 0:
        raise ValueError("offsets needs rows + 1 >= 1 entries")
    lse_ptr = None
    if lse is not None:
        if lse.dtype != torch.float32 or not lse.is_cuda or not lse.is_contiguous() or lse.numel() != rows:
            raise ValueError("lse must be a contiguous float32 device tensor of rows entries")
        lse_ptr = lse.data_ptr()
    s = _stream_of(inp) if stream is None else stream
    st = L.lib().nrm_softmax_batched(ctx.handle if ctx else None, out.data_ptr(), inp.data_ptr(), offsets.data_ptr(),
                                     rows, inp.numel(), lse_ptr, s)
    L.check(st, "nrm_softmax_batched")
    return out


_LF_FORMS = {"all": 0, "eliminated": 1, "promoted": 2, "registers": 3}


def layerforward(hidden, inp, output, form: str = "all", stream: Optional[int] = None):
    """The Fig. 9-shaped tile kernel (see nrm_layerforward in include/nrm.h):
    hidden float32 [R, 16] (updated in place), inp and output float32 [R],
    R a multiple of 16; form "all" (every barrier), "eliminated", "promoted"
    or "registers"."""
    import torch

    if form not in _LF_FORMS:
        raise ValueError("form must be one of %s" % sorted(_LF_FORMS))
    for t in (hidden, inp, output):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("hidden, inp and output must be contiguous float32 device tensors")
    rows = inp.numel()
    if hidden.numel() != 16 * rows or output.numel() != rows:
        raise ValueError("hidden must be [R, 16] and output [R] for R = len(inp)")
    s = _stream_of(inp) if stream is None else stream
    L.check(L.lib().nrm_layerforward(_LF_FORMS[form], hidden.data_ptr(), inp.data_ptr(), output.data_ptr(), rows, s),
            "nrm_layerforward")
    return output


_REDUCTION = {"none": L.NRM_NLL_NONE, "sum": L.NRM_NLL_SUM, "mean": L.NRM_NLL_MEAN}


def nll_loss(logp, target, weight=None, ignore_index: int = -100, reduction: str = "mean", accum: str = "f32",
             out=None, total_weight=None, ctx: Optional[Context] = None, stream: Optional[int] = None):
    """Forward NLL loss: logp float32 [N, C] device tensor (row-major),
    target int64 [N], weight float32 [C] or None. Returns out: float32 [N]
    for reduction "none", else a one-element tensor; total_weight (one
    element, sum and mean) is written when given. Targets outside [0, C)
    other than ignore_index are reported by device_error()."""
    import torch

    if reduction not in _REDUCTION:
        raise ValueError("reduction must be 'none', 'sum' or 'mean'")
    if accum not in _ACCUM:
        raise ValueError("accum must be 'f32' or 'kahan'")
    if logp.dim() != 2 or logp.dtype != torch.float32 or not logp.is_cuda or not logp.is_contiguous():
        raise ValueError("logp must be a contiguous float32 [N, C] device tensor")
    n, c = logp.shape
    if target.dtype != torch.int64 or target.numel() != n or not target.is_contiguous() or target.device != logp.device:
        raise ValueError("target must be a contiguous int64 device tensor of N entries")
    if weight is not None and (weight.dtype != torch.float32 or weight.numel() != c or not weight.is_contiguous()
                               or weight.device != logp.device):
        raise ValueError("weight must be a contiguous float32 device tensor of C entries")
    want = n if reduction == "none" else 1
    if out is None:
        out = torch.empty(want, dtype=torch.float32, device=logp.device)
    elif out.dtype != torch.float32 or out.numel() != want or not out.is_contiguous() or out.device != logp.device:
        raise ValueError("out must be a contiguous float32 device tensor of %d entries" % want)
    if total_weight is not None and (total_weight.dtype != torch.float32 or total_weight.numel() != 1
                                     or total_weight.device != logp.device):
        raise ValueError("total_weight must be a one-element float32 device tensor")
    s = _stream_of(logp) if stream is None else stream
    st = L.lib().nrm_nll_loss(ctx.handle if ctx else None, out.data_ptr(),
                              total_weight.data_ptr() if total_weight is not None else None, logp.data_ptr(),
                              target.data_ptr(), weight.data_ptr() if weight is not None else None, n, c,
                              int(ignore_index), _REDUCTION[reduction], _ACCUM[accum], s)
    L.check(st, "nrm_nll_loss")
    return out


def normalize_rows(pairs, accum: str = "f32", ctx: Optional[Context] = None, stream: Optional[int] = None):
    """Batched normalize of independent rows: pairs is a sequence of
    (out, inp) device tensors (each pair contiguous, same length; dtypes may
    differ between rows). One launch sequence for the whole batch."""
    if accum not in _ACCUM:
        raise ValueError("accum must be 'f32' or 'kahan'")
    pairs = list(pairs)
    table = (L.NrmRow * max(1, len(pairs)))()
    dev = None
    for i, (out, inp) in enumerate(pairs):
        _check_tensors(out, inp)
        dev = inp.device if dev is None else dev
        if inp.device != dev:
            raise ValueError("rows on different devices")
        table[i].in_ = inp.data_ptr()
        table[i].out = out.data_ptr()
        table[i].n = inp.numel()
        table[i].in_dtype = _dtype_code(inp)
        table[i].out_dtype = _dtype_code(out)
    if not pairs:
        return
    s = _stream_of(pairs[0][1]) if stream is None else stream
    st = L.lib().nrm_normalize_rows(ctx.handle if ctx else None, table, len(pairs), _ACCUM[accum], s)
    L.check(st, "nrm_normalize_rows")


def device_error(ctx: Optional[Context] = None, stream: Optional[int] = None) -> int:
    import torch

    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    return L.lib().nrm_get_device_error(ctx.handle if ctx else None, s)


def normalize_form(out, inp, form: str, block: int = 256, stream: Optional[int] = None):
    """One of Fig. 1's un-hoisted forms on the device, for measurement:
    form "naive" (every thread sums the input) or "perblock" (one sum per
    block behind a block barrier). FP32 tensors, n <= 2^20, out != inp."""
    _check_tensors(out, inp)
    codes = {"naive": L.NRM_FORM_NAIVE, "perblock": L.NRM_FORM_PERBLOCK}
    if form not in codes:
        raise ValueError("form must be 'naive' or 'perblock'")
    s = _stream_of(inp) if stream is None else stream
    st = L.lib().nrm_normalize_form(codes[form], out.data_ptr(), inp.data_ptr(), inp.numel(), int(block), s)
    L.check(st, "nrm_normalize_form")
    return out
