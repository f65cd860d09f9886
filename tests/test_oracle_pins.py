"""The CPU oracle against what the paper and the mathematics fix.

Each pin (tests/pins.py) compares the oracle with a closed form, a library
integrator, an exact discrete identity or a symmetry; none compares the oracle
with itself or with the HIP library.
"""
import pytest

from . import pins


@pytest.mark.parametrize("name", list(pins.ALL_PINS))
def test_pin(name):
    ok, info = pins.ALL_PINS[name]()
    assert ok, f"{name}: {info}"
