"""The oracle against facts that do not come from the oracle (see
``oracle_pins``)."""
import pytest

from oracle import oracle as O
from tests.oracle_pins import PINS


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(O)
