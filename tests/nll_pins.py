"""Pins for the FP64 forward NLL-loss oracle (oracle/nll_oracle.c).

loss_n = -w[t_n] logp[n][t_n] (0 for ignored samples); reductions none, sum
and mean = sum / total_weight: the loss kernel of arXiv 2207.00257, Sec. V-B,
defined from the loss's definition. The pins check the oracle against a
closed form, a case worked by hand, exact rational arithmetic,
torch.nn.functional.nll_loss in float64 (an independent implementation),
the ignore_index semantics, invariants (power-of-two weight scaling,
sample permutation) and argument errors.

Every pin takes an `oracle.Oracle`; test_oracle_pins.py runs them on the
real oracle and test_oracle_mutations.py on copies with a planted mistake.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from paper_2207_00257_amd import synth

U64 = 2.0 ** -53


def pin_nll_uniform_closed_form(orc):
    """Every log-probability equal to v = fl32(-log C), no weights: the mean
    is -v exactly, the sum -N v exactly, the total weight N."""
    for n, c in ((1, 1), (7, 10), (1000, 1000), (4096, 3)):
        v = np.float32(-math.log(c)) if c > 1 else np.float32(-0.25)
        logp = np.full((n, c), v, np.float32)
        t = np.arange(n, dtype=np.int64) % c
        mean, tw = orc.nll_loss(logp, t, reduction="mean")
        s, _ = orc.nll_loss(logp, t, reduction="sum")
        assert mean == -float(v) and s == -float(v) * n and tw == n, (n, c, mean, s, tw)


def pin_nll_hand_worked(orc):
    """N = 2, C = 3, logp = [[-1, -2, -3], [-0.5, -0.25, -4]], targets [2, 0],
    weights [1, 2, 0.5]: losses 0.5 * 3 = 1.5 and 1 * 0.5 = 0.5; sum 2,
    total weight 1.5, mean 4/3; a third sample with ignore_index changes
    nothing and has loss 0."""
    logp = np.array([[-1, -2, -3], [-0.5, -0.25, -4], [-9, -9, -9]], np.float32)
    t = np.array([2, 0, -100], np.int64)
    w = np.array([1, 2, 0.5], np.float32)
    none, _ = orc.nll_loss(logp, t, w, reduction="none")
    assert list(none) == [1.5, 0.5, 0.0]
    s, tw = orc.nll_loss(logp, t, w, reduction="sum")
    assert s == 2.0 and tw == 1.5
    mean, _ = orc.nll_loss(logp, t, w, reduction="mean")
    assert abs(mean - 4.0 / 3.0) <= U64 * 4.0 / 3.0


def pin_nll_exact_rational(orc):
    """Random small problems against exact rational arithmetic (every
    binary32 value is a dyadic rational): the sum of non-negative terms is
    within (n + 1) ulps of binary64, the mean within (n + 3)."""
    for seed in range(3):
        logp, t, w = synth.nll_inputs(57, 13, 100 + seed, ignore_frac=0.2)
        exact_s, exact_w = Fraction(0), Fraction(0)
        for i in range(t.size):
            if t[i] == -100:
                continue
            wi = Fraction(float(w[t[i]]))
            exact_s += -wi * Fraction(float(logp[i, t[i]]))
            exact_w += wi
        s, tw = orc.nll_loss(logp, t, w, reduction="sum")
        mean, _ = orc.nll_loss(logp, t, w, reduction="mean")
        assert abs(Fraction(s) - exact_s) <= (t.size + 1) * U64 * exact_s
        assert abs(Fraction(tw) - exact_w) <= (t.size + 1) * U64 * exact_w
        exact_m = exact_s / exact_w
        assert abs(Fraction(mean) - exact_m) <= (t.size + 3) * U64 * exact_m


def pin_nll_torch(orc):
    """Against torch.nn.functional.nll_loss in float64 on the CPU, with class
    weights and ignored samples, for all three reductions."""
    import torch
    import torch.nn.functional as F

    logp, t, w = synth.nll_inputs(3000, 37, 7, ignore_frac=0.1)
    lt, tt, wt = torch.from_numpy(logp).double(), torch.from_numpy(t), torch.from_numpy(w).double()
    none, _ = orc.nll_loss(logp, t, w, reduction="none")
    ref = F.nll_loss(lt, tt, weight=wt, reduction="none").numpy()
    assert np.array_equal(none, ref)
    for red in ("sum", "mean"):
        got, _ = orc.nll_loss(logp, t, w, reduction=red)
        ref = float(F.nll_loss(lt, tt, weight=wt, reduction=red))
        assert abs(got - ref) <= 3000 * 2 * U64 * abs(ref), (red, got, ref)
    got, _ = orc.nll_loss(logp, t, None, reduction="mean")
    assert abs(got - float(F.nll_loss(lt, tt, reduction="mean"))) <= 3000 * 2 * U64 * got


def pin_nll_all_ignored(orc):
    """Every sample ignored: sum 0, total weight 0, mean 0/0 = NaN, and every
    per-sample loss 0."""
    logp = np.full((5, 4), -1.0, np.float32)
    t = np.full(5, 3, np.int64)
    s, tw = orc.nll_loss(logp, t, ignore_index=3, reduction="sum")
    assert s == 0.0 and tw == 0.0
    mean, _ = orc.nll_loss(logp, t, ignore_index=3, reduction="mean")
    assert math.isnan(mean)
    none, _ = orc.nll_loss(logp, t, ignore_index=3, reduction="none")
    assert np.all(none == 0.0)


def pin_nll_invariants(orc):
    """Doubling every weight (exact in binary32 and binary64) leaves the mean
    bit for bit and doubles the sum and the total weight exactly; permuting
    the samples leaves the sum within rounding."""
    logp, t, w = synth.nll_inputs(999, 21, 9)
    s1, tw1 = orc.nll_loss(logp, t, w, reduction="sum")
    m1, _ = orc.nll_loss(logp, t, w, reduction="mean")
    s2, tw2 = orc.nll_loss(logp, t, 2 * w, reduction="sum")
    m2, _ = orc.nll_loss(logp, t, 2 * w, reduction="mean")
    assert s2 == 2 * s1 and tw2 == 2 * tw1 and m2 == m1
    perm = np.random.default_rng(5).permutation(t.size)
    s3, _ = orc.nll_loss(logp[perm], t[perm], w, reduction="sum")
    assert abs(s3 - s1) <= 999 * 2 * U64 * s1


def pin_nll_rejects_bad_targets(orc):
    """A target outside [0, C) that is not ignore_index is an argument error
    (the first sample, so a faulty bound reads in bounds)."""
    logp, t, w = synth.nll_inputs(10, 6, 11, ignore_frac=0.0)
    for bad in (6, -2, 1 << 40):
        tb = t.copy()
        tb[0] = bad
        try:
            orc.nll_loss(logp, tb, w)
        except ValueError:
            continue
        raise AssertionError("target %d accepted" % bad)


NLL_PINS = [
    pin_nll_uniform_closed_form, pin_nll_hand_worked, pin_nll_exact_rational, pin_nll_torch,
    pin_nll_all_ignored, pin_nll_invariants, pin_nll_rejects_bad_targets,
]
