"""The CPU oracle against its pins (closed forms, exact arithmetic, LAPACK/BLAS
libraries, textbook fixtures, finite differences).  CPU only."""
import pytest

import oracle
from tests.oracle_pins import ALL_PINS


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_oracle_pin(pin, lib):
    pin(lib)
