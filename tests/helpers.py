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


def input_fingerprint(rows_strided: np.ndarray, n_rows: int, tiles: np.ndarray, r: np.ndarray) -> str:
    """SHA-256 of a generated workload: every 1000th object row (rows 0, 1000,
    ...; passed in, so that a chunked generator can assemble them), the object
    count and the requests.  Ties a stored oracle result to the inputs it was
    computed from."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.int64(n_rows).tobytes())
    h.update(np.ascontiguousarray(rows_strided, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(tiles, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(r, dtype=np.float64).tobytes())
    return h.hexdigest()


def stratified_sample(tiles: np.ndarray, per_zoom: int, seed: int, zmin: int = 0) -> np.ndarray:
    """Request indices: per_zoom drawn at random at every zoom >= zmin present."""
    rng = np.random.default_rng(seed)
    out = []
    for z in np.unique(tiles[:, 0]):
        if z < zmin:
            continue
        idx = np.nonzero(tiles[:, 0] == z)[0]
        out.append(np.sort(rng.permutation(idx)[:per_zoom]))
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)
