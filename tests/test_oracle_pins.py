"""The FP64 oracle against closed forms, invariants and an independent
set-based statement of the Barnes-Hut walk (CPU only)."""
import pytest

import _pins


@pytest.mark.parametrize("pin", _pins.ALL_PINS, ids=lambda f: f.__name__[4:])
def test_pin(pin):
    pin()
