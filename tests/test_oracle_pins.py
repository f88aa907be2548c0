"""The CPU oracle against facts fixed by the paper and by the mathematics."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(O, pin):
    pin(O)
