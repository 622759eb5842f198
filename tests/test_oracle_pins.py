"""The FP64 oracle against its pins (closed forms, exact rationals, brute
force, invariants, metamorphic relations, library decoders)."""
import pytest

import oracle
from oracle_pins import ALL_PINS


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(oracle.build())


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_rejects_bad_arguments(orc):
    import numpy as np

    with pytest.raises(ValueError):
        orc.normalize_batched(np.ones(4, np.float32), np.array([0, 3, 2], np.int64))
    with pytest.raises(ValueError):
        orc.normalize_batched(np.ones(4, np.float32), np.array([0, 5], np.int64))
    with pytest.raises(ValueError):
        orc.normalize_perblock(np.ones(4, np.float32), 0)
    with pytest.raises(TypeError):
        orc.normalize(np.ones(4, np.float64))
