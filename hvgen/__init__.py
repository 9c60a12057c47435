"""Seeded synthetic workloads for the per-pixel tile-mask engine.

The paper measures on OpenStreetMap and OpenCelliD extracts (its Table 5.2)
that are not available here.  These generators stand in for them with
planet-scale point, linestring and polygon-edge sets of the same kinds, and
with random tile requests over a band of zooms as in its Experiments 2 and 3.

This module is shared by the CPU oracle's tests and by the GPU path's tests
and benchmark.  It produces inputs only: longitude/latitude arrays in
degrees, tile lists and radii.  It computes nothing the method computes (no
projection of objects, no distance, no index); the one exception is the
request sampler ``_tile_of_anchor``, which picks *which* tile to ask for from
an anchor location and therefore never decides what a mask should contain.

Every generator uses numpy's PCG64 ``default_rng``; chunked generators use
``SeedSequence(seed).spawn(k)`` so that each chunk is reproducible alone.

Object layouts (all float64, array-of-structures):
  points            (n, 2): lon, lat
  segments / edges  (n, 4): lon0, lat0, lon1, lat1
Tile lists are int32 (n, 3): z, x, y in the XYZ scheme (y = 0 at the north).
"""
from __future__ import annotations

import math

import numpy as np

LON_LO, LON_HI = -180.0, 180.0
LAT_LO, LAT_HI = -85.0, 85.0

KIND_POINTS = 0
KIND_SEGMENTS = 1
KIND_POLYGON_EDGES = 2


def _fold(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Reflect values into [lo, hi] (a reflecting random walk's position)."""
    w = hi - lo
    y = np.mod(x - lo, 2.0 * w)
    y = np.where(y > w, 2.0 * w - y, y)
    return lo + y


def _tile_of_anchor(lon: np.ndarray, lat: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Request sampling only: the XYZ tile that contains an anchor location.

    Used to draw density-proportional tile requests.  It decides which tiles
    are requested, never what their masks hold (both the oracle and the GPU
    path project the objects themselves).
    """
    n = 2.0 ** z.astype(np.float64)
    fx = (lon + 180.0) / 360.0
    phi = np.radians(np.clip(lat, -85.0511287798066, 85.0511287798066))
    fy = 0.5 - np.arcsinh(np.tan(phi)) / (2.0 * math.pi)
    tx = np.clip(np.floor(fx * n), 0, n - 1).astype(np.int64)
    ty = np.clip(np.floor(fy * n), 0, n - 1).astype(np.int64)
    return np.stack([z.astype(np.int64), tx, ty], axis=1).astype(np.int32)


def all_tiles(z: int) -> np.ndarray:
    """All 4^z tiles of zoom z, row-major in y, then x."""
    n = 1 << z
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([np.full(n * n, z), x.ravel(), y.ravel()], axis=1).astype(np.int32)


# ---------------------------------------------------------------- config 1
def gen_c1_points(seed: int = 0, n: int = 10_000) -> np.ndarray:
    """Uniform points: lon U[-180,180), then lat U[-85,85)."""
    rng = np.random.default_rng(seed)
    lon = rng.uniform(-180.0, 180.0, n)
    lat = rng.uniform(-85.0, 85.0, n)
    return np.ascontiguousarray(np.stack([lon, lat], axis=1))


def c1_requests():
    """All 256 tiles at zoom 4 with point radius 2 px."""
    return all_tiles(4), 2.0


# ---------------------------------------------------------------- config 2
def gen_c2_segments(seed: int = 2, n_segments: int = 10_000_000,
                    n_centres: int = 64, centre_sigma: float = 2.0) -> np.ndarray:
    """Random-walk polylines split into segments.

    64 mixture centres (lon U[-180,180), lat U[-80,80]); each polyline picks a
    centre, starts at centre + N(0, 2 deg) per axis, has m ~ U{2..50}
    vertices, log-normal step length (median 0.01 deg, sigma 1 in log space)
    and uniform heading.  Positions reflect at +-180 / +-85 deg.  Polylines
    are generated until exactly ``n_segments`` segments exist (the last one is
    truncated).
    """
    rng = np.random.default_rng(seed)
    c_lon = rng.uniform(-180.0, 180.0, n_centres)
    c_lat = rng.uniform(-80.0, 80.0, n_centres)
    p_max = n_segments // 20 + 64
    m = rng.integers(2, 51, p_max)                       # vertices per polyline
    nseg = m - 1
    cum = np.cumsum(nseg)
    p = int(np.searchsorted(cum, n_segments)) + 1        # polylines used
    if cum[-1] < n_segments:
        raise RuntimeError("polyline budget too small")
    nseg = nseg[:p].copy()
    nseg[-1] -= int(cum[p - 1] - n_segments)             # truncate the last
    k = rng.integers(0, n_centres, p)
    s_lon = c_lon[k] + rng.normal(0.0, centre_sigma, p)
    s_lat = c_lat[k] + rng.normal(0.0, centre_sigma, p)
    step = rng.lognormal(math.log(0.01), 1.0, n_segments)
    head = rng.uniform(0.0, 2.0 * math.pi, n_segments)
    d_lon = step * np.cos(head)
    d_lat = step * np.sin(head)
    # segmented prefix sums: offset of each step from its polyline's start
    first = np.concatenate([[0], np.cumsum(nseg)[:-1]])
    owner = np.repeat(np.arange(p), nseg)
    cl = np.cumsum(d_lon)
    ca = np.cumsum(d_lat)
    base_l = np.concatenate([[0.0], cl])[first]
    base_a = np.concatenate([[0.0], ca])[first]
    end_l = cl - base_l[owner]
    end_a = ca - base_a[owner]
    beg_l = end_l - d_lon
    beg_a = end_a - d_lat
    out = np.empty((n_segments, 4), dtype=np.float64)
    out[:, 0] = _fold(s_lon[owner] + beg_l, LON_LO, LON_HI)
    out[:, 1] = _fold(s_lat[owner] + beg_a, LAT_LO, LAT_HI)
    out[:, 2] = _fold(s_lon[owner] + end_l, LON_LO, LON_HI)
    out[:, 3] = _fold(s_lat[owner] + end_a, LAT_LO, LAT_HI)
    return out


def c2_requests():
    """All 4096 tiles at zoom 6; line width 1 px -> half-width 0.5 px."""
    return all_tiles(6), 0.5


# ---------------------------------------------------------------- config 3
C3_HOTSPOTS = 1000


def _c3_hotspots(seed: int):
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss.spawn(1)[0])
    lon = rng.uniform(-180.0, 180.0, C3_HOTSPOTS)
    lat = rng.uniform(-80.0, 80.0, C3_HOTSPOTS)
    sig = 10.0 ** rng.uniform(-2.0, 0.0, C3_HOTSPOTS)
    return lon, lat, sig


def _c3_draw(rng, m, hot):
    lon_h, lat_h, sig = hot
    is_hot = rng.random(m) < 0.9
    k = rng.integers(0, C3_HOTSPOTS, m)
    g = rng.normal(0.0, 1.0, (m, 2))
    u_lon = rng.uniform(-180.0, 180.0, m)
    u_lat = rng.uniform(-85.0, 85.0, m)
    lon = np.where(is_hot, _fold(lon_h[k] + sig[k] * g[:, 0], LON_LO, LON_HI), u_lon)
    lat = np.where(is_hot, _fold(lat_h[k] + sig[k] * g[:, 1], LAT_LO, LAT_HI), u_lat)
    return np.ascontiguousarray(np.stack([lon, lat], axis=1))


def gen_c3_chunk(chunk: int, chunk_size: int = 10_000_000, seed: int = 3,
                 n_chunks: int = 100) -> np.ndarray:
    """One chunk of the clustered GPS-like point set.

    1000 hotspots (centre lon U[-180,180), lat U[-80,80]; sigma = 10^U[-2,0]
    deg); 90% of points from a hotspot (isotropic Gaussian, reflected), 10%
    uniform over [-180,180) x [-85,85).
    """
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(1 + n_chunks)
    rng = np.random.default_rng(children[1 + chunk])
    return _c3_draw(rng, chunk_size, _c3_hotspots(seed))


def _workers(jobs: int) -> int:
    import os
    return max(1, min(jobs, 16, len(os.sched_getaffinity(0))))


def gen_c3_points(n: int, seed: int = 3, chunk_size: int = 10_000_000, workers: int | None = None,
                  progress=None) -> np.ndarray:
    """The clustered point set, chunk by chunk.  Chunks are independent, so
    large sets are filled by a thread pool (numpy's generators and array
    arithmetic release the GIL) straight into one array; ``progress(done,
    total)`` is called as chunks finish."""
    n_chunks = max(1, -(-n // chunk_size))
    spawn = max(100, n_chunks)
    if n_chunks == 1:
        return gen_c3_chunk(0, chunk_size, seed, spawn)[:n].copy()
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty((n, 2), dtype=np.float64)

    def fill(chunk):
        lo = chunk * chunk_size
        m = min(chunk_size, n - lo)
        out[lo:lo + m] = gen_c3_chunk(chunk, chunk_size, seed, spawn)[:m]

    with ThreadPoolExecutor(workers or _workers(n_chunks)) as ex:
        for k, _ in enumerate(ex.map(fill, range(n_chunks))):
            if progress:
                progress(k + 1, n_chunks)
    return out


def c3_requests(n: int = 10_000, seed: int = 30, data_seed: int = 3, zmax: int = 18):
    """Density-proportional tiles: z ~ U{0..18}, anchor drawn from the point
    distribution, r ~ U[1,3] px.  Returns (tiles int32 (n,3), r float64 (n,))."""
    rng = np.random.default_rng(seed)
    z = rng.integers(0, zmax + 1, n)
    anc = _c3_draw(rng, n, _c3_hotspots(data_seed))
    r = rng.uniform(1.0, 3.0, n)
    return _tile_of_anchor(anc[:, 0], anc[:, 1], z), r


# ---------------------------------------------------------------- config 4
def _c4_chunk(args) -> np.ndarray:
    """Polygons of one chunk until it holds at least `target` edges."""
    seed, chunk, n_chunks, target, n_centres, centre_sigma, batch_polygons = args
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(1 + n_chunks)
    crng = np.random.default_rng(kids[0])
    c_lon = crng.uniform(-180.0, 180.0, n_centres)
    c_lat = crng.uniform(-80.0, 80.0, n_centres)
    rng = np.random.default_rng(kids[1 + chunk])
    parts = []
    total = 0
    while total < target:
        k = rng.integers(4, 201, batch_polygons)
        cum = np.cumsum(k)
        p = min(batch_polygons, int(np.searchsorted(cum, target - total)) + 1)
        k = k[:p]
        ci = rng.integers(0, n_centres, p)
        px = c_lon[ci] + rng.normal(0.0, centre_sigma, p)
        py = c_lat[ci] + rng.normal(0.0, centre_sigma, p)
        rho = rng.lognormal(math.log(0.05), 1.0, p)
        nv = int(k.sum())
        owner = np.repeat(np.arange(p), k)
        ang = rng.uniform(0.0, 2.0 * math.pi, nv)
        order = np.lexsort((ang, owner))
        ang = ang[order]
        rad = rho[owner] * rng.uniform(0.5, 1.0, nv)
        vx = _fold(px[owner] + rad * np.cos(ang), LON_LO, LON_HI)
        vy = _fold(py[owner] + rad * np.sin(ang), LAT_LO, LAT_HI)
        first = np.concatenate([[0], np.cumsum(k)[:-1]])
        nxt = np.arange(nv) + 1
        nxt[first + k - 1] = first                        # closing edge
        e = np.empty((nv, 4), dtype=np.float64)
        e[:, 0] = vx
        e[:, 1] = vy
        e[:, 2] = vx[nxt]
        e[:, 3] = vy[nxt]
        parts.append(e)
        total += nv
    return np.concatenate(parts, axis=0)


def gen_c4_edges(seed: int = 4, min_edges: int = 200_000_000, n_centres: int = 256,
                 centre_sigma: float = 2.0, batch_polygons: int = 200_000, chunk_edges: int = 10_000_000,
                 workers: int | None = None) -> np.ndarray:
    """Star-shaped random polygons split into edges (closing edge included).

    Polygon centre = one of 256 mixture centres + N(0, 2 deg); k ~ U{4..200}
    vertices at sorted uniform angles; base radius log-normal (median 0.05
    deg, sigma 1); vertex radius = base * U[0.5, 1].  The set is made of
    independent chunks of about chunk_edges edges (generated in parallel for
    large sets), each run until it holds its share; the total is at least
    ``min_edges``.
    """
    n_chunks = max(1, -(-min_edges // chunk_edges))
    share = -(-min_edges // n_chunks)
    jobs = [(seed, c, n_chunks, share, n_centres, centre_sigma, batch_polygons) for c in range(n_chunks)]
    if n_chunks == 1:
        return _c4_chunk(jobs[0])
    from multiprocessing import get_context
    with get_context("fork").Pool(workers or _workers(n_chunks)) as pool:
        parts = pool.map(_c4_chunk, jobs)
    return np.concatenate(parts, axis=0)


def c4_polygon_first(edges: np.ndarray) -> np.ndarray:
    """Polygon offsets of a c4 edge set (npoly + 1 entries): polygons are
    emitted whole, their edges consecutive, so a new polygon starts where an
    edge does not begin at the previous edge's end.  Checks that every
    polygon closes."""
    e = np.asarray(edges, dtype=np.float64).reshape(-1, 4)
    brk = np.nonzero(np.any(e[1:, 0:2] != e[:-1, 2:4], axis=1))[0] + 1
    first = np.concatenate([[0], brk, [e.shape[0]]]).astype(np.int64)
    closes = np.all(e[first[1:] - 1, 2:4] == e[first[:-1], 0:2], axis=1)
    if not closes.all() or np.any(np.diff(first) < 3):
        raise ValueError("edges do not form closed polygons of three or more edges")
    return first


def c4_requests(edges: np.ndarray, n: int = 4096, seed: int = 40, zlo: int = 2, zhi: int = 20):
    """Mixed requests: z ~ U{2..20}, anchor = a random vertex, width
    w ~ U{1..5} px -> half-width r = w/2.  Returns (tiles, r)."""
    rng = np.random.default_rng(seed)
    z = rng.integers(zlo, zhi + 1, n)
    idx = rng.integers(0, edges.shape[0], n)
    w = rng.integers(1, 6, n)
    return _tile_of_anchor(edges[idx, 0], edges[idx, 1], z), w.astype(np.float64) / 2.0


# ---------------------------------------------------------------- config 5
def c5_arrivals(rate: float, seed: int = 5, max_requests: int = 20_000,
                max_seconds: float = 10.0, c2_objects: np.ndarray | None = None,
                c3_anchor_seed: int = 3, zmax: int = 20):
    """Poisson request stream over two resident datasets.

    Returns a dict of arrays: t (arrival time, s), dataset (0 = linestrings,
    1 = points), tiles (n,3) and r (half-width or radius, px).  Linestring
    requests take w ~ U{1..5} -> r = w/2; point requests r ~ U[1,3].
    Anchors are a random segment start (linestrings) or a draw from the point
    distribution (points).
    """
    rng = np.random.default_rng([seed, int(rate)])
    gaps = rng.exponential(1.0 / rate, max_requests)
    t = np.cumsum(gaps)
    n = int(np.searchsorted(t, max_seconds))
    n = max(1, min(n, max_requests))
    t = t[:n]
    ds = (rng.random(n) < 0.5).astype(np.int32)
    z = rng.integers(0, zmax + 1, n)
    w = rng.integers(1, 6, n).astype(np.float64) / 2.0
    rp = rng.uniform(1.0, 3.0, n)
    r = np.where(ds == 0, w, rp)
    if c2_objects is None:
        raise ValueError("c2_objects required for linestring anchors")
    i2 = rng.integers(0, c2_objects.shape[0], n)
    anc3 = _c3_draw(rng, n, _c3_hotspots(c3_anchor_seed))
    alon = np.where(ds == 0, c2_objects[i2, 0], anc3[:, 0])
    alat = np.where(ds == 0, c2_objects[i2, 1], anc3[:, 1])
    return {"t": t, "dataset": ds, "tiles": _tile_of_anchor(alon, alat, z), "r": r}
