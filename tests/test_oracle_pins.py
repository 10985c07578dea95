"""The FP64 oracle against closed forms, limits, invariants, brute force and
independent library routines (no GPU)."""
import pytest

from tests import oracle_pins as P

PINS = P.ALL_PINS


@pytest.mark.parametrize("pin", PINS, ids=[f.__name__ for f in PINS])
def test_pin(pin):
    pin()
