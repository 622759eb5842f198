"""Pins for the FP64 row-softmax / log-sum-exp oracle (oracle/softmax_oracle.c).

softmax_i = exp(x_i) / sum_j exp(x_j) and lse = log sum_j exp(x_j) per CSR
row: the aggregation kernel named among the PyTorch kernels of arXiv
2207.00257 (Sec. V-B), with the reduce-then-map shape of the paper's
normalize (Fig. 1). The pins check the oracle against facts fixed by the
mathematics, never by its own formula: closed forms (constant, one- and
two-element rows), a 50-digit evaluation of the definition itself (mpmath,
no max shift), an independent library implementation (scipy), invariants
(shift, permutation, sums to one, rows independent of each other) and the
overflow-free evaluation at large magnitudes.

Every pin takes an `oracle.Oracle`; test_oracle_pins.py runs them on the
real oracle and test_oracle_mutations.py on copies with a planted mistake.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np

from paper_2207_00257_amd import synth

U64 = 2.0 ** -53


def _rows(orc, rows):
    """Run the oracle on a list of float32 rows as one CSR batch."""
    x = np.concatenate([np.asarray(r, np.float32) for r in rows]) if rows else np.zeros(0, np.float32)
    offs = np.zeros(len(rows) + 1, np.int64)
    offs[1:] = np.cumsum([len(r) for r in rows])
    out, lse = orc.softmax_batched(x, offs)
    return [out[offs[i]:offs[i + 1]] for i in range(len(rows))], lse


def pin_sm_constant_rows(orc):
    """A row of n equal values c: every output is 1/n and lse = c + log n."""
    cases = [(1, 0.0), (2, 1.5), (3, -7.25), (7, 1000.0), (1000, -1000.0), (4096, 0.125)]
    outs, lse = _rows(orc, [np.full(n, c, np.float32) for n, c in cases])
    for (n, c), o, l in zip(cases, outs, lse):
        assert np.all(np.abs(o - 1.0 / n) <= 4 * U64 / n), (n, c)
        assert abs(l - (c + math.log(n))) <= 8 * U64 * max(1.0, abs(c) + math.log(n)), (n, c, l)


def pin_sm_single_element(orc):
    """One-element rows: the output is exactly 1 and lse is the element."""
    vals = [0.0, -3.5, 88.0, -1e4, 1e4, 2.0 ** -20]
    outs, lse = _rows(orc, [[v] for v in vals])
    for v, o, l in zip(vals, outs, lse):
        assert o[0] == 1.0 and l == np.float32(v), (v, o, l)


def pin_sm_two_elements(orc):
    """[a, b]: the outputs are the logistic function of a - b and 1 minus it
    (50-digit closed form 1 / (1 + e^(b - a))), and lse = log(e^a + e^b)."""
    pairs = [(0.0, 0.0), (1.0, 0.0), (0.0, 3.0), (-2.5, 4.0), (30.0, -30.0), (500.0, 499.0)]
    outs, lse = _rows(orc, [[a, b] for a, b in pairs])
    mpmath.mp.dps = 50
    for (a, b), o, l in zip(pairs, outs, lse):
        p0 = 1 / (1 + mpmath.exp(mpmath.mpf(b) - mpmath.mpf(a)))
        assert abs(o[0] - float(p0)) <= 8 * U64 * float(p0), (a, b, o[0], p0)
        assert abs(o[1] - float(1 - p0)) <= 8 * U64 * float(1 - p0), (a, b, o[1])
        ref = mpmath.log(mpmath.exp(a) + mpmath.exp(b))
        assert abs(l - float(ref)) <= 8 * U64 * max(1.0, abs(float(ref))), (a, b, l, ref)


def pin_sm_multiprecision(orc):
    """Random ragged rows against the definition evaluated at 50 digits
    (exp of each element, no max shift, then the ratios and the log)."""
    mpmath.mp.dps = 50
    rng = np.random.default_rng(11)
    rows = [rng.normal(0.0, 3.0, size=n).astype(np.float32) for n in (1, 2, 5, 17, 64, 300)]
    outs, lse = _rows(orc, rows)
    for x, o, l in zip(rows, outs, lse):
        e = [mpmath.exp(mpmath.mpf(float(v))) for v in x]
        s = mpmath.fsum(e)
        for i, v in enumerate(e):
            ref = float(v / s)
            assert abs(o[i] - ref) <= (8 + x.size) * U64 * ref, (x.size, i, o[i], ref)
        ref_l = float(mpmath.log(s))
        assert abs(l - ref_l) <= (8 + x.size) * U64 * max(1.0, abs(ref_l)), (x.size, l, ref_l)


def pin_sm_library(orc):
    """Against scipy.special.softmax / logsumexp (an independent
    implementation), on synthetic logits with the workload's distribution."""
    from scipy.special import logsumexp, softmax

    x, offs = synth.ragged_logits(40, 21, lo=1, hi=5000, sigma=2.0)
    out, lse = orc.softmax_batched(x, offs)
    for r in range(offs.size - 1):
        b, e = int(offs[r]), int(offs[r + 1])
        xr = x[b:e].astype(np.float64)
        ref = softmax(xr)
        assert np.all(np.abs(out[b:e] - ref) <= (16 + e - b) * U64 * ref), r
        assert abs(lse[r] - logsumexp(xr)) <= (16 + e - b) * U64 * max(1.0, abs(lse[r])), r


def pin_sm_shift(orc):
    """Adding a constant to a row leaves its softmax and moves its lse by the
    constant. Values k/256 plus 64 are exact in binary32, so the shifted row
    is exactly x + 64."""
    rng = np.random.default_rng(12)
    x = (rng.integers(-2048, 2048, size=500) / 256.0).astype(np.float32)
    xs = (x.astype(np.float64) + 64.0).astype(np.float32)
    assert np.array_equal(xs.astype(np.float64), x.astype(np.float64) + 64.0)
    (o1,), l1 = _rows(orc, [x])
    (o2,), l2 = _rows(orc, [xs])
    assert np.all(np.abs(o1 - o2) <= 4 * 500 * U64 * o1)
    assert abs((l2[0] - l1[0]) - 64.0) <= 64 * U64 * 100


def pin_sm_sums_to_one_and_order(orc):
    """Every row's outputs sum to one; outputs follow the order of the inputs
    (monotone); permuting a row permutes its outputs."""
    rng = np.random.default_rng(13)
    x = rng.normal(0.0, 2.0, size=777).astype(np.float32)
    (o,), _ = _rows(orc, [x])
    assert abs(math.fsum(o) - 1.0) <= 777 * 4 * U64
    idx = np.argsort(x, kind="stable")
    assert np.all(np.diff(o[idx]) >= 0)
    perm = rng.permutation(x.size)
    (op,), _ = _rows(orc, [x[perm]])
    assert np.all(np.abs(op - o[perm]) <= 777 * 4 * U64 * o[perm])


def pin_sm_rows_independent(orc):
    """In a batch every row equals the row alone, empty rows write nothing
    and have lse = -inf, and the first and last elements of each row count."""
    rng = np.random.default_rng(14)
    rows = [rng.normal(0, 1, size=n).astype(np.float32) for n in (3, 0, 1, 50, 0, 8)]
    rows[0][0] = 9.0   # the maximum at the first element
    rows[5][-1] = 9.0  # and at the last
    outs, lse = _rows(orc, rows)
    for i, r in enumerate(rows):
        if r.size == 0:
            assert lse[i] == -math.inf and outs[i].size == 0
            continue
        (alone,), la = _rows(orc, [r])
        assert np.array_equal(outs[i], alone) and lse[i] == la[0], i
        assert abs(math.fsum(outs[i]) - 1.0) <= r.size * 4 * U64, i
    assert outs[0][0] > 0.99 and outs[5][-1] > 0.99


def pin_sm_large_magnitudes(orc):
    """Magnitudes where exp overflows or underflows in binary64 (|x| ~ 1000)
    give finite outputs: [0, 1000] is one-hot to within e^-1000, and a row
    at -1000 behaves like the same row at 0."""
    outs, lse = _rows(orc, [[0.0, 1000.0], [-1000.0, -1001.0, -1000.5], [0.0, -1.0, -0.5]])
    assert outs[0][1] == 1.0 and outs[0][0] < 1e-300 and lse[0] == 1000.0
    assert np.all(np.isfinite(outs[1])) and np.all(np.abs(outs[1] - outs[2]) <= 8 * U64)
    assert abs((lse[1] - lse[2]) + 1000.0) <= 1e-12


SOFTMAX_PINS = [
    pin_sm_constant_rows, pin_sm_single_element, pin_sm_two_elements, pin_sm_multiprecision,
    pin_sm_library, pin_sm_shift, pin_sm_sums_to_one_and_order, pin_sm_rows_independent,
    pin_sm_large_magnitudes,
]
