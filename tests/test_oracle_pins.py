"""The oracles against their pins (CPU only)."""
import pytest

import oracle
from tests import pins, pins_pi


def setup_module(module):
    oracle.build()


@pytest.mark.parametrize("pin", pins.ALL_PINS + pins_pi.PI_PINS + pins_pi.OTHER_PINS,
                         ids=lambda f: f.__name__)
def test_pin(pin):
    pin()
