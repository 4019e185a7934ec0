"""The oracle against its pins (CPU only)."""
import pytest

import oracle
import pins


@pytest.mark.parametrize("pin", pins.PINS, ids=[p.__name__ for p in pins.PINS])
def test_oracle_pin(pin):
    pin(oracle.load())


def test_range_error():
    hits = pins.make_hits([(0, 0, 0), (256, 3, 1)])
    with pytest.raises(oracle.OracleRangeError):
        oracle.cluster(hits, 256, 256, 10)
    hits = pins.make_hits([(0, 300, 0)])
    with pytest.raises(oracle.OracleRangeError):
        oracle.cluster(hits, 448, 299, 10)
