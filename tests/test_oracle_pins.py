"""The CPU oracle against its pins (brute force, libraries, invariants, hand cases)."""
import pytest

from oracle import binning_oracle
from tests import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(binning_oracle)
