"""The float64 surrogate reference (oracle/nn.py) against its pins (tests/oracle_nn_pins.py):
numpy's correlation, adjoint identities, central finite differences, torch autograd with the
bfloat16 rounding points, closed forms, float32 bit rounding and a hand-computed feature table.
CPU only."""
import pytest

from oracle import nn
from oracle_nn_pins import ALL_NN_PINS


@pytest.mark.parametrize("pin", ALL_NN_PINS, ids=[p.__name__ for p in ALL_NN_PINS])
def test_reference_passes_pin(pin):
    pin(nn)
