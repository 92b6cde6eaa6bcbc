"""The FP64 oracle against facts fixed by the paper and by mathematics (CPU only)."""
import pytest

import oracle
from tests import pins


@pytest.mark.parametrize("pin", pins.PINS, ids=lambda p: p.__name__[4:])
def test_pin(pin):
    pin(oracle.default())
