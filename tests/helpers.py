"""Shared test helpers: mask unpacking and parity comparison."""
from __future__ import annotations

import numpy as np

AMBIGUOUS_LIMIT = 1e-6   # ambiguous pixels allowed, as a fraction of all pixels


def unpack_masks(masks) -> np.ndarray:
    """(n, 8192) uint8 packed masks -> (n, 256, 256) uint8 0/1, [tile][row][col].
    Column i of a row is bit (i & 7), least significant first, of byte i >> 3."""
    m = np.asarray(masks, dtype=np.uint8).reshape(-1, 256, 32)
    return np.unpackbits(m, axis=-1, bitorder="little").reshape(-1, 256, 256)


def parity(gpu_bits: np.ndarray, tri: np.ndarray):
    """(mismatches on non-ambiguous pixels, ambiguous pixels, lit pixels)."""
    amb = tri == 2
    want = tri == 1
    mism = (gpu_bits.astype(bool) != want) & ~amb
    return int(mism.sum()), int(amb.sum()), int(want.sum())


def hilbert_np(x: np.ndarray, y: np.ndarray, bits: int) -> np.ndarray:
    """Hilbert index on a 2^bits grid (vectorised, uint64); written from the
    curve's recursive definition, independently of the GPU build."""
    x = x.astype(np.uint64).copy()
    y = y.astype(np.uint64).copy()
    d = np.zeros_like(x)
    full = np.uint64((1 << bits) - 1)
    for b in range(bits - 1, -1, -1):
        s = np.uint64(1 << b)
        rx = (x & s) > 0
        ry = (y & s) > 0
        quad = np.where(rx, np.where(ry, 2, 3), np.where(ry, 1, 0)).astype(np.uint64)
        d += quad * s * s
        flip = rx & ~ry
        x = np.where(flip, full - x, x)
        y = np.where(flip, full - y, y)
        swap = ~ry
        x, y = np.where(swap, y, x), np.where(swap, x, y)
    return d
