"""FP64 CPU oracle for normalize (arXiv 2207.00257, Fig. 1, Sec. II-A, Sec. IV-C).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path. It shares no code
with the HIP library. The arithmetic lives in normalize_oracle.c,
softmax_oracle.c, nll_oracle.c and layerforward_oracle.c (plain C, binary64);
this module only loads them with ctypes and marshals numpy arrays.

Functions (all return float64 arrays):
  sum_(x)                      Fig. 1's elided `sum`: sequential binary64
  normalize(x)                 hoisted form: S = sum once, out = x / S
  normalize_naive(x)           Fig. 1 as printed: every thread recomputes S
  normalize_perblock(x, B)     shared-memory variant: one S per block of B
  normalize_batched(x, offs)   each CSR row [offs[r], offs[r+1]) on its own
  softmax_batched(x, offs)     row softmax and log-sum-exp (softmax_oracle.c)
  nll_loss(logp, t, w)         forward NLL loss, none / sum / mean (nll_oracle.c)
  layerforward(hidden, inp)    Fig. 9-shaped tile kernel (layerforward_oracle.c)
  decode(x)                    exact widening of FP32 / BF16 / FP16 storage
  round_bf16(y)                binary64 -> nearest bfloat16 (ties to even)

Inputs: numpy float32 arrays, or uint16 arrays holding BF16 / FP16 bit
patterns with dtype="bf16" / "f16".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "normalize_oracle.c")
_SOFTMAX_SRC = os.path.join(_HERE, "softmax_oracle.c")
_NLL_SRC = os.path.join(_HERE, "nll_oracle.c")
_LF_SRC = os.path.join(_HERE, "layerforward_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

DTYPES = {"f32": 0, "bf16": 1, "f16": 2}


def build(force: bool = False, src: str = _SRC, out: str = _LIB_PATH, softmax_src: str = _SOFTMAX_SRC,
          nll_src: str = _NLL_SRC, lf_src: str = _LF_SRC) -> str:
    """Compile the oracle with gcc: binary64 as written (no fast-math, no
    contraction of a*b+c into fma). src, softmax_src, nll_src and lf_src are
    its sources (a test may pass a changed copy of any of them)."""
    srcs = [src, softmax_src, nll_src, lf_src]
    if force or not os.path.exists(out) or os.path.getmtime(out) < max(os.path.getmtime(s) for s in srcs):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, out)
    return out


def _bind(lib):
    i64, p, d = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    lib.oracle_decode.argtypes = [p, ctypes.c_int, i64, p]
    lib.oracle_sum.argtypes = [p, ctypes.c_int, i64]
    lib.oracle_sum.restype = d
    lib.oracle_normalize.argtypes = [p, ctypes.c_int, i64, p, p]
    lib.oracle_normalize_naive.argtypes = [p, ctypes.c_int, i64, p]
    lib.oracle_normalize_perblock.argtypes = [p, ctypes.c_int, i64, i64, p]
    lib.oracle_normalize_batched.argtypes = [p, ctypes.c_int, p, i64, p, p]
    lib.oracle_round_bf16.argtypes = [p, i64, p]
    lib.oracle_round_bf16_one.argtypes = [d]
    lib.oracle_round_bf16_one.restype = ctypes.c_uint16
    lib.oracle_softmax_batched.argtypes = [p, p, i64, p, p]
    lib.oracle_nll_loss.argtypes = [p, p, p, i64, i64, i64, ctypes.c_int, p, p]
    lib.oracle_layerforward.argtypes = [p, p, i64, p, p]
    for name in ("oracle_decode", "oracle_normalize", "oracle_normalize_naive",
                 "oracle_normalize_perblock", "oracle_normalize_batched", "oracle_round_bf16",
                 "oracle_softmax_batched", "oracle_nll_loss", "oracle_layerforward"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


def _prep(x, dtype):
    if dtype not in DTYPES:
        raise ValueError("dtype must be one of %s" % list(DTYPES))
    want = np.float32 if dtype == "f32" else np.uint16
    x = np.ascontiguousarray(x)
    if x.dtype != want:
        raise TypeError("dtype %s needs a %s array, got %s" % (dtype, np.dtype(want), x.dtype))
    return x.reshape(-1)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle rejected its arguments (status %d)" % rc)


class Oracle:
    """The oracle's entry points bound to one compiled copy of the C source."""

    def __init__(self, lib_path: str):
        self.lib = _bind(ctypes.CDLL(lib_path))

    def decode(self, x, dtype="f32"):
        x = _prep(x, dtype)
        out = np.empty(x.size, np.float64)
        _check(self.lib.oracle_decode(x.ctypes.data, DTYPES[dtype], x.size, out.ctypes.data))
        return out

    def sum(self, x, dtype="f32"):
        x = _prep(x, dtype)
        return float(self.lib.oracle_sum(x.ctypes.data, DTYPES[dtype], x.size))

    def normalize(self, x, dtype="f32", return_sum=False):
        x = _prep(x, dtype)
        out = np.empty(x.size, np.float64)
        s = ctypes.c_double(0.0)
        _check(self.lib.oracle_normalize(x.ctypes.data, DTYPES[dtype], x.size, out.ctypes.data,
                                         ctypes.byref(s)))
        return (out, s.value) if return_sum else out

    def normalize_naive(self, x, dtype="f32"):
        x = _prep(x, dtype)
        out = np.empty(x.size, np.float64)
        _check(self.lib.oracle_normalize_naive(x.ctypes.data, DTYPES[dtype], x.size,
                                               out.ctypes.data))
        return out

    def normalize_perblock(self, x, block, dtype="f32"):
        x = _prep(x, dtype)
        out = np.empty(x.size, np.float64)
        _check(self.lib.oracle_normalize_perblock(x.ctypes.data, DTYPES[dtype], x.size, int(block),
                                                  out.ctypes.data))
        return out

    def normalize_batched(self, x, offsets, dtype="f32", return_sums=False):
        x = _prep(x, dtype)
        offs = np.ascontiguousarray(offsets, dtype=np.int64).reshape(-1)
        if offs.size < 1:
            raise ValueError("offsets needs rows + 1 >= 1 entries")
        rows = offs.size - 1
        if rows > 0 and offs[-1] > x.size:
            raise ValueError("offsets run past the input")
        out = np.full(x.size, np.nan, np.float64)
        sums = np.empty(max(rows, 1), np.float64)
        _check(self.lib.oracle_normalize_batched(x.ctypes.data, DTYPES[dtype], offs.ctypes.data,
                                                 rows, out.ctypes.data, sums.ctypes.data))
        return (out, sums[:rows]) if return_sums else out

    def softmax_batched(self, x, offsets):
        """Row softmax and log-sum-exp of a binary32 CSR batch: (out, lse)."""
        x = _prep(x, "f32")
        offs = np.ascontiguousarray(offsets, dtype=np.int64).reshape(-1)
        if offs.size < 1:
            raise ValueError("offsets needs rows + 1 >= 1 entries")
        rows = offs.size - 1
        if rows > 0 and offs[-1] > x.size:
            raise ValueError("offsets run past the input")
        out = np.full(x.size, np.nan, np.float64)
        lse = np.empty(max(rows, 1), np.float64)
        _check(self.lib.oracle_softmax_batched(x.ctypes.data, offs.ctypes.data, rows, out.ctypes.data,
                                               lse.ctypes.data))
        return out, lse[:rows]

    def nll_loss(self, logp, target, weight=None, ignore_index=-100, reduction="mean"):
        """Forward NLL loss: logp float32 [N, C], target int64 [N], weight
        float32 [C] or None. Returns (out, total_weight): out is float64 [N]
        for reduction "none", else a float."""
        red = {"none": 0, "sum": 1, "mean": 2}[reduction]
        logp = np.ascontiguousarray(logp, dtype=np.float32)
        if logp.ndim != 2:
            raise ValueError("logp must be [N, C]")
        n, c = logp.shape
        target = np.ascontiguousarray(target, dtype=np.int64).reshape(-1)
        if target.size != n:
            raise ValueError("target needs N entries")
        wp = None
        if weight is not None:
            weight = np.ascontiguousarray(weight, dtype=np.float32).reshape(-1)
            if weight.size != c:
                raise ValueError("weight needs C entries")
            wp = weight.ctypes.data
        out = np.empty(max(n, 1) if red == 0 else 1, np.float64)
        tw = np.empty(1, np.float64)
        _check(self.lib.oracle_nll_loss(logp.ctypes.data, target.ctypes.data, wp, n, c, int(ignore_index), red,
                                        out.ctypes.data, tw.ctypes.data))
        return (out[:n] if red == 0 else float(out[0])), float(tw[0])

    def layerforward(self, hidden, inp):
        """The Fig. 9-shaped tile kernel: hidden float32 [R, 16], inp float32
        [R] (R a multiple of 16). Returns (new_hidden [R, 16], output [R]) in
        binary64: each row after the tile's halving tree, and each tile's 16
        column sums."""
        hidden = np.ascontiguousarray(hidden, dtype=np.float32)
        inp = np.ascontiguousarray(inp, dtype=np.float32).reshape(-1)
        if hidden.ndim != 2 or hidden.shape[1] != 16 or hidden.shape[0] != inp.size:
            raise ValueError("hidden must be [R, 16] with R = len(input)")
        rows = inp.size
        new_hidden = np.empty((rows, 16), np.float64)
        out = np.empty(max(rows, 1), np.float64)
        _check(self.lib.oracle_layerforward(hidden.ctypes.data, inp.ctypes.data, rows, new_hidden.ctypes.data,
                                            out.ctypes.data))
        return new_hidden, out[:rows]

    def round_bf16(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        out = np.empty(y.size, np.uint16)
        _check(self.lib.oracle_round_bf16(y.ctypes.data, y.size, out.ctypes.data))
        return out

    def round_bf16_one(self, v: float) -> int:
        return int(self.lib.oracle_round_bf16_one(float(v)))


_default = None


def _get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def decode(x, dtype="f32"):
    return _get().decode(x, dtype)


def sum_(x, dtype="f32"):
    return _get().sum(x, dtype)


def normalize(x, dtype="f32", return_sum=False):
    return _get().normalize(x, dtype, return_sum)


def normalize_naive(x, dtype="f32"):
    return _get().normalize_naive(x, dtype)


def normalize_perblock(x, block, dtype="f32"):
    return _get().normalize_perblock(x, block, dtype)


def normalize_batched(x, offsets, dtype="f32", return_sums=False):
    return _get().normalize_batched(x, offsets, dtype, return_sums)


def softmax_batched(x, offsets):
    return _get().softmax_batched(x, offsets)


def nll_loss(logp, target, weight=None, ignore_index=-100, reduction="mean"):
    return _get().nll_loss(logp, target, weight, ignore_index, reduction)


def layerforward(hidden, inp):
    return _get().layerforward(hidden, inp)


def round_bf16(y):
    return _get().round_bf16(y)
