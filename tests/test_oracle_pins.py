"""The oracle against its pins (CPU only)."""
import pytest

import oracle
from tests import pins


def setup_module(module):
    oracle.build()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()
