"""Tolerances and comparison helpers shared by the GPU parity tests.

Acceptance against the FP64 oracle (out_ref):
  FP32 out : |out - ref| <= 4e-6 * |ref| element-wise. The bound follows from
             binary32 summation with at most h ~ 60 levels of additions for
             non-negative inputs (|S^ - S| <= gamma_h * S, gamma_h = h u /
             (1 - h u), u = 2^-24) plus one correctly rounded division.
  BF16 out : |out - ref| <= one BF16 ulp of ref, 2^(floor(log2|ref|) - 7).
  FP16 out : |out - ref| <= one FP16 ulp of ref (subnormal quantum 2^-24).
Mixed-sign inputs scale the FP32 bound by kappa = sum|x| / |sum x|.
"""
from __future__ import annotations

import numpy as np

REL_F32 = 4e-6


def rel_err(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    got = got.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.abs(got - ref) / np.abs(ref)
    e[(ref == 0) & (got == 0)] = 0.0
    e[(ref == 0) & (got != 0)] = np.inf
    return e


def assert_f32_close(got, ref, tol=REL_F32, what=""):
    e = rel_err(np.asarray(got), np.asarray(ref))
    bad = ~(e <= tol)
    if bad.any():
        i = int(np.argmax(np.where(np.isnan(e), np.inf, e)))
        raise AssertionError("%s: %d of %d outputs off by more than %g relative; worst at %d: got %r ref %r (rel %g)"
                             % (what, int(bad.sum()), e.size, tol, i, float(got[i]), float(ref[i]), float(e[i])))
    return float(e.max()) if e.size else 0.0


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def ulp_bf16(ref: np.ndarray) -> np.ndarray:
    a = np.abs(ref)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -126)
    return np.exp2(e - 7)


def ulp_f16(ref: np.ndarray) -> np.ndarray:
    a = np.abs(ref)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -14)
    return np.exp2(e - 10)


def assert_within_ulp(got_f64, ref, ulp_fn, what=""):
    err = np.abs(got_f64 - ref)
    u = ulp_fn(ref)
    bad = ~(err <= u)
    if bad.any():
        i = int(np.argmax(np.where(bad, err / u, 0)))
        raise AssertionError("%s: %d of %d outputs off by more than one ulp; worst at %d: got %r ref %r"
                             % (what, int(bad.sum()), err.size, i, float(got_f64[i]), float(ref[i])))
    return float(np.max(err / u)) if err.size else 0.0
