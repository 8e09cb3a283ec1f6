"""The CPU oracle against its pins (closed forms, exact bounds, textbook
compaction and range, brute force).  CPU only."""
import pytest

import oracle as O
from pins import PINS


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(pin):
    pin(O.lib())
