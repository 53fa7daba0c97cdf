"""The CPU oracle against its pins (values fixed by the paper and by
mathematics, see tests/pins.py)."""

import pytest

import oracle
import pins


@pytest.mark.parametrize("pin", pins.ALL, ids=lambda f: f.__name__)
def test_pin(pin):
    ok, detail = pin(oracle)
    assert ok, detail
