"""The FP64 forward NLL-loss oracle against its pins (closed form, a case
worked by hand, exact rationals, torch in float64, invariants)."""
import numpy as np
import pytest

import oracle
from nll_pins import NLL_PINS


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(oracle.build())


@pytest.mark.parametrize("pin", NLL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_rejects_bad_arguments(orc):
    with pytest.raises(ValueError):
        orc.nll_loss(np.zeros(4, np.float32), np.zeros(4, np.int64))          # logp not [N, C]
    with pytest.raises(ValueError):
        orc.nll_loss(np.zeros((4, 3), np.float32), np.zeros(3, np.int64))     # target length
    with pytest.raises(ValueError):
        orc.nll_loss(np.zeros((4, 3), np.float32), np.zeros(4, np.int64), np.ones(2, np.float32))
