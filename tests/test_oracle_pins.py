"""CPU pins of the oracle (no GPU): see tests/oracle_pins.py."""
import pytest

from tests import oracle_pins


@pytest.mark.parametrize("check", oracle_pins.ALL, ids=lambda c: c.__name__)
def test_oracle_pin(check):
    fails = check()
    assert not fails, "\n".join(fails[:20])
