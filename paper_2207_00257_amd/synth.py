"""Seeded synthetic inputs for normalize workloads.

This module draws inputs only; it performs none of normalize's arithmetic, so
both the HIP path's callers and the FP64 oracle's tests can take their inputs
from here. Every generator is numpy's PCG64 seeded explicitly, so an input is a
pure function of (recipe, size, seed).

Recipes (the workloads this library is measured on):
  uniform_f32          in[i] ~ Uniform[lo, hi) in binary32 (default [0.5, 1.5))
  lognormal_f32        in[i] = fl32(exp(sigma * N(0,1)))
  lognormal_bf16       the same value rounded to bfloat16 (ties to even from
                       the binary32 draw), returned as uint16 bit patterns
  loguniform_lengths   integer lengths floor(exp(U[ln lo, ln(hi+1)))), clipped
  ragged_offsets       CSR offsets (int64, rows + 1) from a length vector
  poisson_arrivals     open-loop arrival times with exponential gaps
  normal_f32           logits in[i] = fl32(sigma * N(0,1))
  ragged_logits        a ragged batch of normal logits (the softmax workload)
  nll_inputs           log-probabilities, targets and class weights (NLL loss)
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_f32(n: int, seed: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """n binary32 values in [lo, hi): lo + (hi - lo) * U, U a binary32 draw in [0, 1)."""
    u = _rng(seed).random(int(n), dtype=np.float32)
    x = np.float32(lo) + np.float32(hi - lo) * u
    # binary32 rounding of lo + w*u can land on hi; keep the half-open range
    np.minimum(x, np.nextafter(np.float32(hi), np.float32(lo)), out=x)
    return x


def lognormal_f32(n: int, seed: int, sigma: float = 1.0) -> np.ndarray:
    g = _rng(seed).standard_normal(int(n), dtype=np.float64)
    return np.exp(sigma * g).astype(np.float32)


def normal_f32(n: int, seed: int, sigma: float = 2.0) -> np.ndarray:
    """Logits: fl32(sigma * N(0,1))."""
    return (sigma * _rng(seed).standard_normal(int(n), dtype=np.float64)).astype(np.float32)


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Quantise binary32 inputs to bfloat16 bit patterns (round to nearest even).
    Input preparation only: the workload's stored BF16 values are defined by it."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = np.isnan(x)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    r = r.astype(np.uint16)
    r[nan] = 0x7FC0
    return r


def lognormal_bf16(n: int, seed: int, sigma: float = 2.0) -> np.ndarray:
    return f32_to_bf16_bits(lognormal_f32(n, seed, sigma))


def f32_to_f16_bits(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


def loguniform_lengths(count: int, seed: int, lo: int, hi: int) -> np.ndarray:
    """Integer lengths log-uniform on [lo, hi]: floor(exp(U[ln lo, ln(hi + 1)))),
    clipped to [lo, hi]."""
    u = _rng(seed).random(int(count))
    v = np.floor(np.exp(np.log(lo) + u * (np.log(hi + 1.0) - np.log(lo))))
    return np.clip(v, lo, hi).astype(np.int64)


def ragged_offsets(lengths: np.ndarray) -> np.ndarray:
    offs = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(np.asarray(lengths, np.int64), out=offs[1:])
    return offs


def ragged_batch(rows: int, seed: int, lo: int = 32, hi: int = 1 << 20, sigma: float = 1.0):
    """The ragged batched workload: `rows` rows with log-uniform lengths in
    [lo, hi] and LogNormal(0, sigma) binary32 values. Returns (values, offsets)."""
    lengths = loguniform_lengths(rows, seed, lo, hi)
    offs = ragged_offsets(lengths)
    vals = lognormal_f32(int(offs[-1]), seed + 1000003, sigma)
    return vals, offs


def ragged_logits(rows: int, seed: int, lo: int = 32, hi: int = 1 << 20, sigma: float = 2.0):
    """The softmax workload: `rows` rows with log-uniform lengths in [lo, hi]
    (the ragged batch's lengths) and N(0, sigma^2) binary32 logits.
    Returns (values, offsets)."""
    lengths = loguniform_lengths(rows, seed, lo, hi)
    offs = ragged_offsets(lengths)
    return normal_f32(int(offs[-1]), seed + 1000003, sigma), offs


def nll_inputs(n: int, c: int, seed: int, ignore_frac: float = 0.05, ignore_index: int = -100):
    """The NLL-loss workload: log-probabilities logp[n][c] = fl32(-E), E ~
    Exponential(mean 3) (values in (-inf, 0], like log-softmax outputs), targets
    uniform in [0, c) with a fraction ignore_frac replaced by ignore_index,
    and class weights uniform in [0.5, 1.5). Returns (logp, target, weight)."""
    rng = _rng(seed)
    logp = (-rng.exponential(3.0, size=(int(n), int(c)))).astype(np.float32)
    target = rng.integers(0, int(c), size=int(n), dtype=np.int64)
    target[rng.random(int(n)) < ignore_frac] = ignore_index
    weight = uniform_f32(int(c), seed + 7, 0.5, 1.5)
    return logp, target, weight


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds, increasing) of a Poisson process of the given rate."""
    rng = _rng(seed)
    expect = int(rate_per_s * duration_s * 1.2 + 64)
    gaps = rng.exponential(1.0 / rate_per_s, expect)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate_per_s, expect)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]
