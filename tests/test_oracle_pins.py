"""The CPU oracle against its pins (closed forms, brute force, cKDTree, invariants)."""
import pytest

import oracle_pins


@pytest.mark.parametrize("name", sorted(oracle_pins.PINS))
def test_pin(name):
    oracle_pins.PINS[name]()


def test_ckdtree_c1_all_tiles():
    """All 16,777,216 pixel centres of the 10k-point, zoom-4 workload."""
    oracle_pins.pin_ckdtree(n_tiles=256)
