"""The CPU oracle against its pins (brute force, independent Split, closed forms, invariants,
the paper's Example 1, exact arithmetic). CPU only."""
import pytest

import oracle
from oracle_pins import ALL_PINS


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin):
    pin()
