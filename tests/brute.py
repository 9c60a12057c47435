"""Brute force for tiny inputs: every object against every pixel (numpy).

Independent of the oracle's index and of its C code: it pins the oracle's
culling and addressing.  Distances follow the definition of the mask (the
distance from the pixel centre to the nearest point or closed segment, in
world pixels of the tile's zoom).
"""
from __future__ import annotations

import math

import numpy as np

BAND = 1e-6


def merc01(lonlat: np.ndarray) -> np.ndarray:
    """Own Web-Mercator (atanh form), used only by the brute force."""
    ll = np.asarray(lonlat, dtype=np.float64).reshape(-1, 2)
    lat = np.clip(ll[:, 1], -85.0511287798066, 85.0511287798066)
    X = (ll[:, 0] + 180.0) / 360.0
    Y = 0.5 - np.arctanh(np.sin(np.radians(lat))) / (2.0 * math.pi)
    return np.stack([X, Y], axis=1)


def objects_merc01(objects: np.ndarray, kind: int) -> np.ndarray:
    if kind == 0:
        return merc01(objects)
    o = np.asarray(objects, dtype=np.float64).reshape(-1, 4)
    a = merc01(o[:, 0:2])
    b = merc01(o[:, 2:4])
    return np.concatenate([a, b], axis=1)


def brute_distance(objs: np.ndarray, kind: int, z: int, x: int, y: int,
                   chunk: int = 64, off: tuple = (0.0, 0.0)) -> np.ndarray:
    """D (256,256) [row j][column i] at the pixel centres shifted by ``off``
    (px, e.g. an anti-aliasing sub-sample); objs are normalised Mercator."""
    S = 256.0 * 2.0 ** z
    cols = np.arange(256, dtype=np.float64) + 0.5
    PX = np.tile(cols + off[0], 256)[:, None]          # column i of pixel p
    PY = np.repeat(cols + off[1], 256)[:, None]        # row j of pixel p
    best = np.full((65536, 1), np.inf)
    if kind == 0:
        o = np.asarray(objs, dtype=np.float64).reshape(-1, 2)
        for s in range(0, o.shape[0], chunk):
            u = o[s:s + chunk, 0] * S - 256.0 * x
            v = o[s:s + chunk, 1] * S - 256.0 * y
            d2 = (PX - u[None, :]) ** 2 + (PY - v[None, :]) ** 2
            best = np.minimum(best, d2.min(axis=1, keepdims=True))
    else:
        o = np.asarray(objs, dtype=np.float64).reshape(-1, 4)
        for s in range(0, o.shape[0], chunk):
            ax = o[s:s + chunk, 0] * S - 256.0 * x
            ay = o[s:s + chunk, 1] * S - 256.0 * y
            bx = o[s:s + chunk, 2] * S - 256.0 * x
            by = o[s:s + chunk, 3] * S - 256.0 * y
            dx, dy = bx - ax, by - ay
            l2 = dx * dx + dy * dy
            safe = np.where(l2 > 0, l2, 1.0)
            t = ((PX - ax) * dx + (PY - ay) * dy) / safe
            t = np.where(l2 > 0, np.clip(t, 0.0, 1.0), 0.0)
            ex = PX - (ax + t * dx)
            ey = PY - (ay + t * dy)
            best = np.minimum(best, (ex * ex + ey * ey).min(axis=1, keepdims=True))
    return np.sqrt(best).reshape(256, 256)


def tri_state(D: np.ndarray, r: float) -> np.ndarray:
    return np.where(D < r - BAND, 1, np.where(D > r + BAND, 0, 2)).astype(np.uint8)


def near_band_edge(D: np.ndarray, r: float, tol: float = 1e-9) -> np.ndarray:
    """Pixels whose classification could flip under last-bit rounding."""
    return (np.abs(D - (r - BAND)) <= tol) | (np.abs(D - (r + BAND)) <= tol) | (np.abs(D - r) <= tol)


def brute_fill(edges: np.ndarray, first, z: int, x: int, y: int):
    """Polygon fill by brute force: for every polygon, the parity of its edges
    crossed by a ray from each pixel centre towards -x (half-open in y), then
    OR over polygons.  Returns (inside (256,256) bool, distance (256,256) from
    each centre to the nearest edge, px).  edges: normalised Mercator (n, 4)."""
    S = 256.0 * 2.0 ** z
    e = np.asarray(edges, dtype=np.float64).reshape(-1, 4)
    ax, ay = e[:, 0] * S - 256.0 * x, e[:, 1] * S - 256.0 * y
    bx, by = e[:, 2] * S - 256.0 * x, e[:, 3] * S - 256.0 * y
    c = np.arange(256, dtype=np.float64) + 0.5
    CX, CY = np.meshgrid(c, c)                       # [row j][column i]
    inside = np.zeros((256, 256), dtype=bool)
    dist = np.full((256, 256), np.inf)
    for p in range(len(first) - 1):
        par = np.zeros((256, 256), dtype=bool)
        for q in range(first[p], first[p + 1]):
            cross = (ay[q] > CY) != (by[q] > CY)
            if cross.any():
                with np.errstate(divide="ignore", invalid="ignore"):
                    xc = ax[q] + (CY - ay[q]) * (bx[q] - ax[q]) / (by[q] - ay[q])
                par ^= cross & (xc < CX)
            dx, dy = bx[q] - ax[q], by[q] - ay[q]
            l2 = dx * dx + dy * dy
            t = np.clip(((CX - ax[q]) * dx + (CY - ay[q]) * dy) / l2, 0.0, 1.0) if l2 > 0 else 0.0
            dist = np.minimum(dist, np.hypot(CX - (ax[q] + t * dx), CY - (ay[q] + t * dy)))
        inside |= par
    return inside, dist
