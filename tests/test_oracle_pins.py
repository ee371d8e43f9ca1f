"""The FP64 oracle against its pins (CPU only)."""
import warnings

import pytest

import oracle as O
import pins


@pytest.fixture(scope="module")
def orc():
    return O.get()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        pin(orc)
