"""Pins for the FP64 oracle: checks against facts fixed by the paper's
definition and by mathematics, never by the oracle's own formula.

normalize (arXiv 2207.00257, Fig. 1): out[i] = in[i] / sum_{j<n} in[j]. The
paper prints no numeric example, so the pins are closed forms worked by hand
(tests/golden/closed_forms.txt), exact rational arithmetic (fractions),
brute force, invariants (the outputs sum to one), metamorphic relations
(power-of-two scaling, permutation), the legality of hoisting the sum
(Sec. IV-C: the naive, per-block and hoisted forms agree) and library
decoders for the storage formats.

Every pin is a function taking an `oracle.Oracle`; test_oracle_pins.py runs
them on the real oracle and test_oracle_mutations.py runs them on copies of
the oracle with a planted mistake, each of which must fail at least one pin.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

from paper_2207_00257_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.txt")
U64 = 2.0 ** -53  # binary64 unit roundoff


def _rat(tok: str) -> Fraction:
    if "*2^" in tok:
        m, e = tok.split("*2^")
        return Fraction(int(m)) * (Fraction(2) ** int(e))
    return Fraction(tok)


def golden_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split("|")]
            cases.append(parts)
    return cases


def pin_golden_plain(orc):
    for parts in golden_cases():
        if parts[0] != "plain":
            continue
        x = np.array([float(Fraction(t)) for t in parts[2].split()], np.float32)
        want = [float(_rat(t)) for t in parts[3].split()]
        got = orc.normalize(x)
        assert list(got) == want, (parts[1], list(got), want)


def pin_golden_batched(orc):
    for parts in golden_cases():
        if parts[0] != "batch":
            continue
        x = np.array([float(Fraction(t)) for t in parts[2].split()], np.float32)
        offs = np.array([int(t) for t in parts[3].split()], np.int64)
        want = [float(_rat(t)) for t in parts[4].split()]
        got = orc.normalize_batched(x, offs)
        assert list(got) == want, (parts[1], list(got), want)


def pin_golden_bf16_decode(orc):
    for parts in golden_cases():
        if parts[0] != "bf16":
            continue
        bits = np.array([int(parts[2], 16)], np.uint16)
        want = float(_rat(parts[3]))
        got = orc.decode(bits, "bf16")[0]
        assert got == want, (parts[1], got, want)


def pin_golden_sum(orc):
    """The elided `sum` of Fig. 1 on hand-worked inputs: exact integers and
    dyadic rationals whose binary64 sum is exact in any order (a binary32
    accumulator loses the 1s after 2^24, a dropped or repeated term changes
    the total)."""
    seen = 0
    for parts in golden_cases():
        if parts[0] != "sum":
            continue
        toks = parts[2].split()
        x = np.array([float(Fraction(t)) for t in toks], np.float32)
        want = float(_rat(parts[3]))
        got = orc.sum(x)
        assert got == want, (parts[1], got, want)
        seen += 1
    assert seen >= 5


def pin_sum_exact_rational(orc):
    """The exported sum against exact rationals: within the sequential bound
    (n-1) u sum|x| of the exact sum, for FP32, BF16 and FP16 storage, and equal
    to the sum the hoisted normalize divides by."""
    for seed in range(4):
        for n in (1, 2, 5, 64, 300):
            x = synth.lognormal_f32(n, 500 + seed * 11 + n, 2.0)
            exact = sum(Fraction(float(v)) for v in x)
            s = orc.sum(x)
            gamma = (n - 1) * U64 / (1 - (n - 1) * U64)
            assert abs(Fraction(s) - exact) <= Fraction(gamma) * exact, (n, seed)
            _, s_norm = orc.normalize(x, return_sum=True)
            assert s == s_norm, (n, seed)
            bits = synth.lognormal_bf16(n, 900 + seed + n, 1.0)
            vals = (bits.astype(np.uint32) << 16).view(np.float32)
            exact = sum(Fraction(float(v)) for v in vals)
            assert abs(Fraction(orc.sum(bits, "bf16")) - exact) <= Fraction(gamma) * exact, (n, seed, "bf16")
            h = np.abs(synth.lognormal_f32(n, 77 + seed + n, 1.0)).astype(np.float16)
            exact = sum(Fraction(float(v)) for v in h)
            assert abs(Fraction(orc.sum(h.view(np.uint16), "f16")) - exact) <= Fraction(gamma) * exact
    # an asymmetric input: the first and the last element both count
    assert orc.sum(np.array([1024.0, 1.0, 2.0, 4096.0], np.float32)) == 5123.0
    assert orc.sum(np.zeros(0, np.float32)) == 0.0


def pin_exact_rational(orc):
    """Brute force with exact rationals on small random inputs: the oracle's
    sum is within the sequential-summation bound (n-1)*u*sum|x| of the exact
    sum, and each output within that plus one rounding of the exact quotient."""
    for seed in range(6):
        for n in (1, 2, 3, 7, 33, 200):
            x = synth.lognormal_f32(n, 100 + seed * 7 + n, 1.5)
            exact_s = sum(Fraction(float(v)) for v in x)
            out, s = orc.normalize(x, return_sum=True)
            gamma = (n - 1) * U64 / (1 - (n - 1) * U64)
            assert abs(Fraction(s) - exact_s) <= Fraction(gamma) * exact_s, (n, seed)
            for i in range(n):
                q = Fraction(float(x[i])) / exact_s
                tol = Fraction(gamma + 2 * U64) * q
                assert abs(Fraction(out[i]) - q) <= tol, (n, seed, i)


def pin_exact_rational_signed(orc):
    """Mixed signs: exact rationals give the quotient; tolerance is scaled by
    the condition number sum|x| / |sum x|."""
    for seed in range(4):
        n = 50
        g = np.random.Generator(np.random.PCG64(7 + seed))
        x = (g.standard_normal(n) + 0.3).astype(np.float32)
        exact_s = sum(Fraction(float(v)) for v in x)
        abs_s = sum(abs(Fraction(float(v))) for v in x)
        out = orc.normalize(x)
        gamma = (n - 1) * U64 / (1 - (n - 1) * U64)
        for i in range(n):
            q = Fraction(float(x[i])) / exact_s
            tol = Fraction(gamma) * abs_s / abs(exact_s) * abs(q) + Fraction(2 * U64) * abs(q)
            assert abs(Fraction(out[i]) - q) <= tol + Fraction(1, 10**300), (seed, i)


def pin_hoist_legal(orc):
    """Sec. IV-C / Fig. 1 caption: computing the invariant sum once (hoisted),
    once per block (shared memory), or once per thread (naive) gives the same
    result, bit for bit."""
    for n in (1, 2, 3, 31, 32, 33, 100, 1000, 1024):
        x = synth.uniform_f32(n, 2 + n)
        ref = orc.normalize(x)
        assert np.array_equal(orc.normalize_naive(x), ref), n
        for b in (1, 32, 64, 256):
            assert np.array_equal(orc.normalize_perblock(x, b), ref), (n, b)


def pin_constant_power_of_two(orc):
    """Constant input c at n = 2^k: the binary64 sum n*c is exact (at most
    24 + k <= 53 significant bits), so every output is exactly 2^-k."""
    for c in (1.0, 0.5, 2.0, 0.7, 3.3, 1.4999999):
        c32 = np.float32(c)
        for k in list(range(0, 13)) + [16, 20]:
            n = 1 << k
            out = orc.normalize(np.full(n, c32, np.float32))
            assert np.all(out == 2.0 ** -k), (c, k)
    # BF16 and FP16 constants: same argument, fewer significant bits
    for bits, dt in ((0x3FC0, "bf16"), (0x4049, "bf16"), (0x3E00, "f16"), (0x4248, "f16")):
        for k in (0, 5, 10, 17):
            n = 1 << k
            out = orc.normalize(np.full(n, bits, np.uint16), dt)
            assert np.all(out == 2.0 ** -k), (hex(bits), dt, k)


def pin_sums_to_one(orc):
    """Invariant: the outputs sum to one; the exact sum (math.fsum) of the
    binary64 outputs is within a few n*u of 1."""
    for n, seed in ((10, 1), (1000, 2), (100000, 3)):
        for x in (synth.uniform_f32(n, seed), synth.lognormal_f32(n, seed, 2.0)):
            out = orc.normalize(x)
            assert abs(math.fsum(out) - 1.0) <= 4 * n * U64, n


def pin_power_of_two_scaling(orc):
    """Metamorphic: scaling every input by 2^m scales the sum by 2^m exactly
    and leaves every quotient unchanged, bit for bit."""
    for n in (5, 64, 4097):
        x = synth.lognormal_f32(n, 40 + n, 1.0)
        ref = orc.normalize(x)
        for m in (-20, -3, 1, 7, 30):
            y = (x * np.float32(2.0 ** m)).astype(np.float32)
            assert np.array_equal(orc.normalize(y), ref), (n, m)


def pin_permutation(orc):
    """Metamorphic: permuting the input permutes the output (up to the sum's
    reordering, within 2 (n-1) u)."""
    n = 3001
    x = synth.lognormal_f32(n, 9, 1.0)
    perm = np.random.Generator(np.random.PCG64(11)).permutation(n)
    a = orc.normalize(x)[perm]
    b = orc.normalize(x[perm])
    assert np.all(np.abs(a - b) <= 2 * (n + 2) * U64 * np.abs(a))
    # an asymmetric input catches a shifted or reversed index
    y = np.arange(1, 9, dtype=np.float32)
    assert np.array_equal(orc.normalize(y[::-1].copy()), orc.normalize(y)[::-1])


def pin_batched_rows(orc):
    """Ragged batch: each CSR row equals the plain normalize of its slice, bit
    for bit; rows of length 0 and 1 are covered."""
    lengths = np.array([0, 1, 2, 31, 0, 33, 1000, 1, 0, 257], np.int64)
    offs = synth.ragged_offsets(lengths)
    x = synth.lognormal_f32(int(offs[-1]), 5, 1.0)
    out, sums = orc.normalize_batched(x, offs, return_sums=True)
    for r in range(len(lengths)):
        b, e = offs[r], offs[r + 1]
        assert np.array_equal(out[b:e], orc.normalize(x[b:e])), r
        exact = sum(Fraction(float(v)) for v in x[b:e])
        assert abs(Fraction(sums[r]) - exact) <= Fraction((e - b) * U64) * exact, r
    # an offsets array starting past zero leaves the prefix untouched
    offs2 = np.array([3, 5, 9], np.int64)
    out2 = orc.normalize_batched(x, offs2)
    assert np.all(np.isnan(out2[:3])) and np.all(np.isnan(out2[9:]))
    assert np.array_equal(out2[3:5], orc.normalize(x[3:5]))


def pin_decode_bf16_library(orc):
    """Every one of the 65536 BF16 bit patterns decodes to torch's own
    bfloat16 -> float32 widening (a library routine), NaN to NaN."""
    import torch

    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ref = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).float().double().numpy()
    got = orc.decode(bits, "bf16")
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])


def pin_decode_f16_library(orc):
    """Every one of the 65536 FP16 bit patterns decodes to numpy's float16."""
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    got = orc.decode(bits, "f16")
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])


def pin_round_bf16(orc):
    """binary64 -> bfloat16, ties to even: on binary32-representable values it
    equals torch's float32 -> bfloat16 conversion (a library routine, which
    rounds once from an exact value); hand-worked ties and a case where going
    through binary32 first would round twice."""
    import torch

    g = np.random.Generator(np.random.PCG64(3))
    f = np.concatenate([
        g.standard_normal(20000).astype(np.float32) * np.float32(1e3),
        np.exp(g.uniform(-95, 88, 20000)).astype(np.float32),
        (g.integers(0, 2**16, 5000).astype(np.uint32) << 16 | 0x8000).view(np.float32),  # exact ties
        np.array([3.0e38, 3.4e38, 1e-40, -1e-42, 0.0, -0.0], np.float32),
    ])
    f = f[np.isfinite(f)]
    ref = torch.from_numpy(f).bfloat16().view(torch.int16).numpy().view(np.uint16)
    got = orc.round_bf16(f.astype(np.float64))
    assert np.array_equal(got, ref)
    assert orc.round_bf16_one(1.0 + 2.0 ** -8) == 0x3F80  # tie -> even (down)
    assert orc.round_bf16_one(1.0 + 3 * 2.0 ** -8) == 0x3F82  # tie -> even (up)
    assert orc.round_bf16_one(1.0 + 2.0 ** -8 + 2.0 ** -40) == 0x3F81  # binary32 first would tie
    assert orc.round_bf16_one(-(1.0 + 2.0 ** -8 + 2.0 ** -40)) == 0xBF81
    assert orc.round_bf16_one(float("inf")) == 0x7F80
    assert orc.round_bf16_one(2.0 ** -134) == 0x0000  # half the smallest subnormal: tie -> 0
    assert orc.round_bf16_one(3 * 2.0 ** -134) == 0x0002  # tie between 1 and 2 quanta -> even


def pin_ieee_specials(orc):
    """Silent in the paper; IEEE semantics: zero sum gives NaN (0/0) and +-inf,
    and a NaN input poisons every output."""
    out = orc.normalize(np.zeros(4, np.float32))
    assert np.all(np.isnan(out))
    out = orc.normalize(np.array([1.0, -1.0], np.float32))
    assert out[0] == math.inf and out[1] == -math.inf
    out = orc.normalize(np.array([1.0, np.nan, 2.0], np.float32))
    assert np.all(np.isnan(out))
    assert orc.normalize(np.zeros(0, np.float32)).size == 0


ALL_PINS = [
    pin_golden_plain, pin_golden_batched, pin_golden_bf16_decode, pin_golden_sum, pin_sum_exact_rational,
    pin_exact_rational,
    pin_exact_rational_signed, pin_hoist_legal, pin_constant_power_of_two, pin_sums_to_one,
    pin_power_of_two_scaling, pin_permutation, pin_batched_rows, pin_decode_bf16_library,
    pin_decode_f16_library, pin_round_bf16, pin_ieee_specials,
]
