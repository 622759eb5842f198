"""The FP64 oracle of the Fig. 9-shaped tile kernel against its pins."""
import pytest

import oracle
from layerforward_pins import LAYERFORWARD_PINS


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(oracle.build())


@pytest.mark.parametrize("pin", LAYERFORWARD_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)
