"""Writes the oracle's masks for zoom-stratified samples of the two largest
workloads, which tests/test_gpu_fullsize.py compares with the GPU path:

  fullsize_c4.npz  2e8 star-polygon edges, 4,096 requests at zooms 2-20:
                   27 requests per zoom (513 tiles); the oracle indexes every
                   edge.
  fullsize_c3.npz  1e9 clustered points, 10,000 requests at zooms 0-18:
                   27 requests per zoom at zooms >= ZMIN_C3; each tile is
                   rendered by an oracle index over the points of the zoom-8
                   cells it covers and of the cells around them, which holds
                   every point within a cell's width (>= 256 px at zoom >= 8,
                   >= 1.4 degrees) of the tile.  Below ZMIN_C3 a tile holds up
                   to 270M points, beyond a host index here.

Each file holds the sampled request indices, their tiles and radii, the
oracle's lit bits (tri-state 1) and ambiguous bits (tri-state 2), packed
least significant bit first in the masks' layout, and a fingerprint of the
generated inputs (helpers.input_fingerprint) that the test recomputes.

  fullsize_c4_aa.npz  the 2e8 edges' anti-aliased values (oracle, exact mode)
                   for 4 requests per zoom (76 tiles).
  fullsize_c4_fill.npz  the fill masks of their 1,961,254 polygons for 27
                   requests per zoom (513 tiles), the oracle over all polygons.
  fullsize_c3_aa.npz  the 1e9 points' anti-aliased values (oracle, exact mode)
                   for 4 requests per zoom at zooms >= ZMIN_C3 (64 tiles).

Calls only the oracle and the seeded generators.  Usage:
    python tests/golden/make_fullsize_parity.py [c4] [c3] [c4aa] [c4fill] [c3aa]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import hvgen  # noqa: E402
import oracle  # noqa: E402
from helpers import input_fingerprint, stratified_sample  # noqa: E402

PER_ZOOM = 27
PER_ZOOM_AA = 4
ZMIN_C3 = 3
SEED = 4040
T0 = time.time()


def log(msg):
    print(f"[{time.time() - T0:7.1f}s] {msg}", flush=True)


def save(path, idx, tiles, r, tri, fp, note):
    np.savez_compressed(path, idx=idx, tiles=tiles[idx], r=r[idx],
                        lit=np.packbits(tri == 1, axis=-1, bitorder="little"),
                        amb=np.packbits(tri == 2, axis=-1, bitorder="little"),
                        fingerprint=np.array(fp), note=np.array(note))
    log(f"wrote {path}: {len(idx)} tiles, {int((tri == 1).sum())} lit, {int((tri == 2).sum())} ambiguous")


def render_all(ix, tiles, r, idx, step=32):
    tri = np.empty((len(idx), 256, 256), dtype=np.uint8)
    for s in range(0, len(idx), step):
        sel = idx[s:s + step]
        tri[s:s + len(sel)] = ix.render(tiles[sel], r[sel], want_bit=False)["tri"]
        log(f"rendered {s + len(sel)}/{len(idx)}")
    return tri


def c4():
    edges = hvgen.gen_c4_edges()
    tiles, r = hvgen.c4_requests(edges, n=4096)
    fp = input_fingerprint(edges[::1000], edges.shape[0], tiles, r)
    idx = stratified_sample(tiles, PER_ZOOM, SEED)
    log(f"c4: {edges.shape[0]} edges, {len(idx)} sampled requests; building the oracle index")
    ix = oracle.OracleIndex(edges, oracle.POLYGON_EDGES)
    del edges
    tri = render_all(ix, tiles, r, idx)
    save(os.path.join(HERE, "fullsize_c4.npz"), idx, tiles, r, tri, fp,
         f"{PER_ZOOM} requests per zoom (seed {SEED}); oracle over all edges")


def c4aa():
    """Anti-aliased values (Algorithm 1's 0-4, the oracle's exact mode) of 4
    requests per zoom of the 2e8 edges: per pixel the value, the number of
    its sub-samples within 1e-6 px of r (ambiguous) and the number certainly
    within r."""
    edges = hvgen.gen_c4_edges()
    tiles, r = hvgen.c4_requests(edges, n=4096)
    fp = input_fingerprint(edges[::1000], edges.shape[0], tiles, r)
    idx = stratified_sample(tiles, PER_ZOOM_AA, SEED + 1)
    log(f"c4aa: {edges.shape[0]} edges, {len(idx)} sampled requests; building the oracle index")
    ix = oracle.OracleIndex(edges, oracle.POLYGON_EDGES)
    del edges
    val = np.empty((len(idx), 256, 256), dtype=np.uint8)
    amb = np.empty_like(val)
    sure = np.empty_like(val)
    for s in range(0, len(idx), 8):
        sel = idx[s:s + 8]
        o = ix.render_aa(tiles[sel], r[sel])
        val[s:s + len(sel)], amb[s:s + len(sel)], sure[s:s + len(sel)] = o["val"], o["amb"], o["sure"]
        log(f"c4aa: rendered {s + len(sel)}/{len(idx)}")
    path = os.path.join(HERE, "fullsize_c4_aa.npz")
    np.savez_compressed(path, idx=idx, tiles=tiles[idx], r=r[idx], val=val, amb=amb, sure=sure,
                        fingerprint=np.array(fp),
                        note=np.array(f"{PER_ZOOM_AA} requests per zoom (seed {SEED + 1}); oracle (exact mode) "
                                      "over all edges"))
    log(f"wrote {path}: {len(idx)} tiles, {int((val > 0).sum())} nonzero, {int(amb.sum())} ambiguous sub-samples")


def c4fill():
    """Fill masks (Algorithm 2) of the 2e8 edges' polygons for 27 requests
    per zoom, by an oracle over all 1,961,254 polygons."""
    edges = hvgen.gen_c4_edges()
    first = hvgen.c4_polygon_first(edges)
    tiles, r = hvgen.c4_requests(edges, n=4096)
    fp = input_fingerprint(edges[::1000], edges.shape[0], tiles, r)
    idx = stratified_sample(tiles, PER_ZOOM, SEED + 2)
    log(f"c4fill: {len(first) - 1} polygons, {len(idx)} sampled requests; building the oracle")
    P = oracle.OraclePolygons(edges, first)
    del edges
    tri = np.empty((len(idx), 256, 256), dtype=np.uint8)
    for s in range(0, len(idx), 8):
        sel = idx[s:s + 8]
        tri[s:s + len(sel)] = P.render(tiles[sel])["tri"]
        log(f"c4fill: rendered {s + len(sel)}/{len(idx)}")
    save(os.path.join(HERE, "fullsize_c4_fill.npz"), idx, tiles, r, tri, fp,
         f"{PER_ZOOM} requests per zoom (seed {SEED + 2}); fill oracle over all polygons")


def _cell_of(pts):
    """Zoom-8 cell (row-major, 256 x 256) of each point: chooses which points a
    tile's host index holds (own projection; the oracle projects them itself)."""
    lat = np.clip(pts[:, 1], -85.0511287798066, 85.0511287798066)
    cx = np.minimum(((pts[:, 0] + 180.0) / 360.0 * 256).astype(np.int32), 255)
    cy = np.minimum(((0.5 - np.arctanh(np.sin(np.radians(lat))) / (2 * np.pi)) * 256).astype(np.int32), 255)
    return (np.clip(cy, 0, 255) * 256 + np.clip(cx, 0, 255)).astype(np.uint16)


def _c3_points_by_cell():
    """The 1e9 points sorted by zoom-8 cell, with the cells' start offsets."""
    n = 1_000_000_000
    tiles, r = hvgen.c3_requests(10_000)
    pts = hvgen.gen_c3_points(n)
    fp = input_fingerprint(pts[::1000], n, tiles, r)
    log(f"c3: {n} points generated; sorting by zoom-8 cell")
    cells = np.empty(n, dtype=np.uint16)
    for s in range(0, n, 10_000_000):
        cells[s:s + 10_000_000] = _cell_of(pts[s:s + 10_000_000])
    start = np.zeros(65537, dtype=np.int64)
    start[1:] = np.cumsum(np.bincount(cells, minlength=65536))
    order = np.argsort(cells, kind="stable")
    del cells
    pts = pts[order]
    del order
    return pts, start, tiles, r, fp


def _c3_near(pts, start, tile):
    """The points of the zoom-8 cells a tile covers and of the cells around them."""
    z, x, y = (int(v) for v in tile)
    if z >= 8:
        x0 = x1 = x >> (z - 8)
        y0 = y1 = y >> (z - 8)
    else:
        x0, x1 = x << (8 - z), ((x + 1) << (8 - z)) - 1
        y0, y1 = y << (8 - z), ((y + 1) << (8 - z)) - 1
    xa, xb = max(0, x0 - 1), min(255, x1 + 1)
    return np.concatenate([pts[start[cy * 256 + xa]:start[cy * 256 + xb + 1]]
                           for cy in range(max(0, y0 - 1), min(255, y1 + 1) + 1)])


def c3():
    pts, start, tiles, r, fp = _c3_points_by_cell()
    idx = stratified_sample(tiles, PER_ZOOM, SEED, zmin=ZMIN_C3)
    tri = np.empty((len(idx), 256, 256), dtype=np.uint8)
    for k, t in enumerate(idx):
        z = int(tiles[t, 0])
        sub = _c3_near(pts, start, tiles[t])
        if len(sub) == 0:
            tri[k] = 0
            continue
        tri[k] = oracle.OracleIndex(sub, oracle.POINTS).render(tiles[t:t + 1], r[t:t + 1], want_bit=False)["tri"][0]
        if k % 20 == 0 or z <= 5:
            log(f"c3: tile {k + 1}/{len(idx)} z{z}: {len(sub)} points near")
    save(os.path.join(HERE, "fullsize_c3.npz"), idx, tiles, r, tri, fp,
         f"{PER_ZOOM} requests per zoom at zooms >= {ZMIN_C3} (seed {SEED}); each tile against an oracle index "
         "over the points of the zoom-8 cells it covers and the cells around them")


def c3aa():
    """Anti-aliased values (oracle, exact mode) of 4 requests per zoom of the
    1e9 points at zooms >= ZMIN_C3, each tile against an oracle index over the
    points near it (the margin, a zoom-8 cell, exceeds r + 1/4 px)."""
    pts, start, tiles, r, fp = _c3_points_by_cell()
    idx = stratified_sample(tiles, PER_ZOOM_AA, SEED + 3, zmin=ZMIN_C3)
    val = np.zeros((len(idx), 256, 256), dtype=np.uint8)
    amb = np.zeros_like(val)
    sure = np.zeros_like(val)
    for k, t in enumerate(idx):
        sub = _c3_near(pts, start, tiles[t])
        if len(sub):
            o = oracle.OracleIndex(sub, oracle.POINTS).render_aa(tiles[t:t + 1], r[t:t + 1])
            val[k], amb[k], sure[k] = o["val"][0], o["amb"][0], o["sure"][0]
        log(f"c3aa: tile {k + 1}/{len(idx)} z{int(tiles[t, 0])}: {len(sub)} points near")
    path = os.path.join(HERE, "fullsize_c3_aa.npz")
    np.savez_compressed(path, idx=idx, tiles=tiles[idx], r=r[idx], val=val, amb=amb, sure=sure,
                        fingerprint=np.array(fp),
                        note=np.array(f"{PER_ZOOM_AA} requests per zoom at zooms >= {ZMIN_C3} (seed {SEED + 3}); "
                                      "oracle (exact mode) over the points near each tile"))
    log(f"wrote {path}: {len(idx)} tiles, {int((val > 0).sum())} nonzero, {int(amb.sum())} ambiguous sub-samples")


if __name__ == "__main__":
    for key in sys.argv[1:] or ["c4", "c3"]:
        {"c4": c4, "c3": c3, "c4aa": c4aa, "c4fill": c4fill, "c3aa": c3aa}[key]()
