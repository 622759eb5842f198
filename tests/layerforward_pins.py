"""Pins for the FP64 oracle of the Fig. 9-shaped tile kernel
(oracle/layerforward_oracle.c; arXiv 2207.00257, Sec. IV-A and IV-B).

Per tile of 16 rows: p[y][x] = hidden[j][x] * input[j], a halving tree over
y, every row written back (row y then holds the sum of p over rows
y .. y + L(y) - 1, L(y) the largest power of two dividing y, 16 for y = 0)
and the 16 column sums written to output. The pins check closed forms
(all-ones and one-hot tiles), an independent matrix-vector product for the
column sums, block sums over the tree's row ranges computed another way,
and argument errors.
"""
from __future__ import annotations

import numpy as np

U64 = 2.0 ** -53
SPAN = [16] + [y & -y for y in range(1, 16)]  # largest power of two dividing y


def pin_lf_all_ones(orc):
    """All ones: every column sum is 16 and row y holds L(y)."""
    h = np.ones((64, 16), np.float32)
    nh, out = orc.layerforward(h, np.ones(64, np.float32))
    assert np.all(out == 16.0)
    for y in range(16):
        assert np.all(nh[y::16] == SPAN[y]), y


def pin_lf_one_hot(orc):
    """input one-hot at row k of each tile: the column sums are hidden's row
    k, and row y holds hidden row k when k lies in [y, y + L(y)), else 0."""
    rng = np.random.default_rng(31)
    h = rng.uniform(0.5, 1.5, size=(48, 16)).astype(np.float32)
    for k in (0, 5, 15):
        v = np.zeros(48, np.float32)
        v[k::16] = 1.0
        nh, out = orc.layerforward(h, v)
        assert np.array_equal(out.reshape(3, 16), h[k::16].astype(np.float64))
        for y in range(16):
            want = h[k::16].astype(np.float64) if y <= k < y + SPAN[y] else np.zeros((3, 16))
            assert np.array_equal(nh[y::16], want), (k, y)


def pin_lf_matvec(orc):
    """Column sums against an independent matrix-vector product per tile
    (numpy's binary64 dot)."""
    rng = np.random.default_rng(32)
    h = rng.uniform(0.5, 1.5, size=(16 * 50, 16)).astype(np.float32)
    v = rng.uniform(0.5, 1.5, size=16 * 50).astype(np.float32)
    _, out = orc.layerforward(h, v)
    ref = np.einsum("byx,by->bx", h.reshape(50, 16, 16).astype(np.float64), v.reshape(50, 16).astype(np.float64))
    assert np.all(np.abs(out.reshape(50, 16) - ref) <= 20 * U64 * ref)


def pin_lf_tree_rows(orc):
    """Every row after the tree against prefix-sum differences over its
    power-of-two row range (a different evaluation of the same sums)."""
    rng = np.random.default_rng(33)
    h = rng.uniform(0.5, 1.5, size=(16 * 20, 16)).astype(np.float32)
    v = rng.uniform(0.5, 1.5, size=16 * 20).astype(np.float32)
    nh, _ = orc.layerforward(h, v)
    p = (h.astype(np.float64) * v.astype(np.float64)[:, None]).reshape(20, 16, 16)
    csum = np.concatenate([np.zeros((20, 1, 16)), np.cumsum(p, axis=1)], axis=1)
    for y in range(16):
        ref = csum[:, y + SPAN[y], :] - csum[:, y, :]
        assert np.all(np.abs(nh.reshape(20, 16, 16)[:, y, :] - ref) <= 40 * U64 * ref), y


def pin_lf_rejects_bad_rows(orc):
    """R must be a multiple of 16 (whole tiles)."""
    try:
        orc.layerforward(np.ones((20, 16), np.float32), np.ones(20, np.float32))
    except ValueError:
        return
    raise AssertionError("20 rows accepted")


LAYERFORWARD_PINS = [pin_lf_all_ones, pin_lf_one_hot, pin_lf_matvec, pin_lf_tree_rows, pin_lf_rejects_bad_rows]
