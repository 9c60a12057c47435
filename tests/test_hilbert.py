"""Pins for the test-side Hilbert index used to check the GPU's sort order."""
import numpy as np

from helpers import hilbert_np


def test_order2_sequence():
    # The order-2 Hilbert curve visits the 4x4 grid in this (x, y) order.
    seq = [(0, 0), (1, 0), (1, 1), (0, 1), (0, 2), (0, 3), (1, 3), (1, 2),
           (2, 2), (2, 3), (3, 3), (3, 2), (3, 1), (2, 1), (2, 0), (3, 0)]
    x = np.array([p[1] for p in seq])   # this convention: first coordinate is the row
    y = np.array([p[0] for p in seq])
    d = hilbert_np(x, y, 2)
    assert sorted(d.tolist()) == list(range(16))
    # consecutive indices are grid neighbours, start at a corner
    order = np.argsort(d)
    pts = np.stack([x[order], y[order]], 1)
    assert (np.abs(np.diff(pts, axis=0)).sum(1) == 1).all()


def test_bijective_and_adjacent_order5():
    n = 32
    gx, gy = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    d = hilbert_np(gx.ravel(), gy.ravel(), 5)
    assert np.array_equal(np.sort(d), np.arange(n * n, dtype=np.uint64))
    order = np.argsort(d)
    pts = np.stack([gx.ravel()[order], gy.ravel()[order]], 1)
    assert (np.abs(np.diff(pts, axis=0)).sum(1) == 1).all()
    # quadrant structure: the first quarter of the curve stays in one quadrant
    q = pts[: n * n // 4]
    assert (q.max(0) < n // 2).all()


def test_large_order_is_monotone_refinement():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 1 << 20, 1000)
    y = rng.integers(0, 1 << 20, 1000)
    d20 = hilbert_np(x, y, 20)
    d10 = hilbert_np(x >> 10, y >> 10, 10)
    assert np.array_equal(d20 >> np.uint64(20), d10)    # a coarser curve is a prefix
