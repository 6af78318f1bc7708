"""The FP64 oracle against its pins (CPU only): values printed in the paper,
closed forms, SymPy derivatives, invariants and brute force."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle  # noqa: E402
import oracle_pins  # noqa: E402


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=[p.__name__ for p in oracle_pins.ALL_PINS])
def test_pin(pin):
    pin(oracle)
