"""The FP64 row-softmax / log-sum-exp oracle against its pins (closed forms,
a 50-digit evaluation of the definition, scipy, invariants)."""
import numpy as np
import pytest

import oracle
from softmax_pins import SOFTMAX_PINS


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(oracle.build())


@pytest.mark.parametrize("pin", SOFTMAX_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_rejects_bad_arguments(orc):
    with pytest.raises(ValueError):
        orc.softmax_batched(np.ones(4, np.float32), np.array([0, 3, 2], np.int64))
    with pytest.raises(ValueError):
        orc.softmax_batched(np.ones(4, np.float32), np.array([0, 5], np.int64))
    with pytest.raises(TypeError):
        orc.softmax_batched(np.ones(4, np.float64), np.array([0, 4], np.int64))
