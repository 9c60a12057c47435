"""Polygon filling (SIBF, Algorithm 2) on the GPU against the oracle, through
the C ABI.  Bar: every pixel the oracle does not flag (centre within 1e-6 px
of an edge of a polygon that could hold it) matches bit-exactly."""
import math

import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import log
from helpers import unpack_masks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "needs a GPU"
    return t


@pytest.fixture(scope="module")
def hv():
    from paper_2005_12489_amd import hv as m
    return m


def build_polys(hv, torch, edges, first, merc01=False):
    t = torch.from_numpy(np.ascontiguousarray(edges, dtype=np.float64)).cuda()
    h = hv.hv_polygon_index_build(t, first, flags=hv.HV_INPUT_MERC01 if merc01 else 0)
    del t
    return h


def fill(hv, torch, h, tiles, launch=None):
    tiles = np.asarray(tiles).reshape(-1, 3)
    out = torch.empty((max(1, len(tiles)), 8192), dtype=torch.uint8, device="cuda")
    out.fill_(0x3C)     # masks must be fully overwritten
    hv.hv_render_fill(h, tiles, out, launch)
    torch.cuda.synchronize()
    return unpack_masks(out[:len(tiles)].cpu().numpy())


def check(got, tri, what):
    clean = tri != 2
    bad = int((got[clean] != tri[clean]).sum())
    log(f"{what}: pixels={got.size} filled={int(got.sum())} ambiguous={int((~clean).sum())} mismatches={bad}")
    assert bad == 0, f"{what}: {bad} pixels differ from the oracle"


def _ring_px(z, x, y, pts):
    S = 256.0 * 2 ** z
    X = (256.0 * x + np.array([p[0] for p in pts])) / S
    Y = (256.0 * y + np.array([p[1] for p in pts])) / S
    return np.stack([X, Y, np.roll(X, -1), np.roll(Y, -1)], 1)


def _group(rings_per_poly, z, x, y):
    edges, first = [], [0]
    for rings in rings_per_poly:
        for ring in rings:
            edges.append(_ring_px(z, x, y, ring))
        first.append(first[-1] + sum(len(r) for r in rings))
    return np.concatenate(edges), np.array(first, dtype=np.int64)


def _box(u0, v0, u1, v1):
    return [(u0, v0), (u1, v0), (u1, v1), (u0, v1)]


def test_fill_closed_forms(hv, torch):
    z, x, y = 9, 300, 200
    polys = [[_box(10.25, 30.25, 20.75, 40.75), _box(13.25, 33.25, 16.75, 36.75)],       # square with a hole
             [_box(100.25, 30.25, 140.75, 60.75)], [_box(110.25, 40.25, 120.75, 50.75)],  # nested, separate
             [[(100.0, 100.0), (137.0, 100.0), (100.0, 137.0)]],                           # right triangle
             [[(50.5, 160.0), (70.5, 180.5), (50.5, 201.0), (30.5, 180.5)]],              # vertices on centre lines
             [_box(-40.0, 220.0, 40.0, 300.0)]]                                            # across the tile's corner
    e, f = _group(polys, z, x, y)
    log("fill closed forms")
    h = build_polys(hv, torch, e, f, merc01=True)
    tiles = [(z, x, y), (z, x - 1, y), (z, x - 1, y + 1), (z, x, y + 1), (z - 1, x // 2, y // 2)]
    ref = oracle.OraclePolygons(e, f, merc01=True).render(tiles)["tri"]
    got = fill(hv, torch, h, tiles)
    check(got, ref, "fill closed forms")
    assert int(got[0, 30:41, 10:21].sum()) == 121 - 16 and got[0, 45, 115] == 1
    hv.hv_free(h)


def test_fill_random_rings_holes_overlaps(hv, torch):
    """Random simple rings (stars), some with a star hole, overlapping, at
    several zooms; region 32 and 64 agree."""
    rng = np.random.default_rng(71)
    for z, x, y in ((3, 2, 3), (10, 600, 400), (16, 40000, 30000)):
        polys = []
        for _ in range(40):
            c = rng.uniform(-60, 316, 2)
            rho = rng.uniform(4.0, 120.0)
            k = int(rng.integers(4, 60))
            ang = np.sort(rng.uniform(0, 2 * math.pi, k))
            rad = rho * rng.uniform(0.5, 1.0, k)
            outer = [(c[0] + rad[q] * math.cos(ang[q]), c[1] + rad[q] * math.sin(ang[q])) for q in range(k)]
            rings = [outer]
            if rng.random() < 0.4:
                rings.append([(c[0] + 0.3 * rad[q] * math.cos(ang[q]), c[1] + 0.3 * rad[q] * math.sin(ang[q]))
                              for q in range(k)][::-1])
            polys.append(rings)
        e, f = _group(polys, z, x, y)
        h = build_polys(hv, torch, e, f, merc01=True)
        tiles = [(z, x + dx, y + dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
        log(f"fill random rings z={z}")
        ref = oracle.OraclePolygons(e, f, merc01=True).render(tiles)["tri"]
        got = fill(hv, torch, h, tiles)
        check(got, ref, f"fill random rings z={z}")
        assert np.array_equal(fill(hv, torch, h, tiles, dict(region=64, waves_per_wg=4, cand_cap=256)), got)
        assert np.array_equal(fill(hv, torch, h, tiles, dict(region=32, waves_per_wg=2, cand_cap=128)), got)
        assert np.array_equal(fill(hv, torch, h, tiles, dict(region=32, waves_per_wg=1, cand_cap=128,
                                                              cull_nodes=2)), got)
        hv.hv_free(h)


def test_fill_large_polygons_across_tiles(hv, torch):
    """Rings of 1000 vertices spanning many tiles: tiles deep inside fill
    completely, tiles on the boundary partly, tiles outside stay empty."""
    rng = np.random.default_rng(73)
    polys = []
    for cx, cy, rho in ((10.0, 45.0, 8.0), (-60.0, -20.0, 15.0)):
        k = 1000
        ang = np.sort(rng.uniform(0, 2 * math.pi, k))
        rad = rho * rng.uniform(0.8, 1.0, k)
        lon = cx + rad * np.cos(ang)
        lat = cy + 0.7 * rad * np.sin(ang)
        polys.append(np.stack([lon, lat, np.roll(lon, -1), np.roll(lat, -1)], 1))
    e = np.concatenate(polys)
    f = np.array([0, 1000, 2000], dtype=np.int64)
    h = build_polys(hv, torch, e, f)
    X, Y = oracle.project(np.array([[10.0, 45.0], [-60.0, -20.0], [19.5, 45.0], [120.0, 0.0]]))
    tiles = [(z, int(X[q] * 2 ** z), int(Y[q] * 2 ** z)) for z in (2, 5, 8, 12) for q in range(4)]
    log("fill large polygons")
    ref = oracle.OraclePolygons(e, f).render(tiles)["tri"]
    got = fill(hv, torch, h, tiles)
    check(got, ref, "fill large polygons")
    deep = [k for k, t in enumerate(tiles) if t[0] == 12 and k % 4 in (0, 1)]
    assert all(got[k].all() for k in deep), "tiles deep inside are full"
    assert not got[[k for k, t in enumerate(tiles) if k % 4 == 3]].any(), "tiles far outside are empty"
    hv.hv_free(h)


def test_fill_many_edge_rings_both_ray_sides(hv, torch):
    """Rings of 20,000 and 5,000 vertices (an outer ring and its hole) that
    span many regions of a tile: regions in a polygon's left half cast rays to
    -x, those in its right half to +x (the nearer box side, as Algorithm 2
    does per pixel); both must give the oracle's parity, next to a small
    polygon in the hole and a long thin one across the tile."""
    rng = np.random.default_rng(79)
    z, x, y = 10, 300, 400

    def ring(cx, cy, rho, k, wiggle):
        ang = np.linspace(0.0, 2 * math.pi, k, endpoint=False)
        rad = rho * (1.0 + wiggle * rng.uniform(-1.0, 1.0, k))
        return list(zip(cx + rad * np.cos(ang), cy + 0.8 * rad * np.sin(ang)))

    outer = ring(128.3, 131.7, 110.0, 20_000, 0.02)
    hole = ring(120.1, 125.4, 45.0, 5_000, 0.05)
    small = ring(118.6, 127.2, 9.0, 12, 0.1)
    thin = [(2.2, 60.3), (250.7, 64.9), (250.7, 66.1), (2.2, 61.8)]
    e, f = _group([[outer, hole], [small], [thin]], z, x, y)
    h = build_polys(hv, torch, e, f, merc01=True)
    tiles = [(z, x, y), (z, x + 1, y), (z, x, y + 1), (z + 1, 2 * x, 2 * y), (z + 1, 2 * x + 1, 2 * y + 1),
             (z - 1, x // 2, y // 2)]
    log("fill many-edge rings")
    ref = oracle.OraclePolygons(e, f, merc01=True).render(tiles)["tri"]
    for L in (None, dict(region=64, waves_per_wg=4, cand_cap=256), dict(region=32, waves_per_wg=1, cand_cap=64)):
        got = fill(hv, torch, h, tiles, L)
        check(got, ref, f"fill many-edge rings {L}")
    assert got[0].sum() > 20000 and got[0, 128, 124] == 1 and got[0, 128, 110] == 0, "ring, hole, small polygon"
    hv.hv_free(h)


def test_fill_star_polygons_mixed_zooms(hv, torch):
    edges = hvgen.gen_c4_edges(min_edges=300_000, batch_polygons=4000)
    first = hvgen.c4_polygon_first(edges)
    tiles, _ = hvgen.c4_requests(edges, n=160, seed=47)
    log(f"fill c4 star polygons: {len(first) - 1} polygons, {len(tiles)} tiles")
    h = build_polys(hv, torch, edges, first)
    info = hv.hv_index_info(h)
    assert info["kind"] == hv.HV_POLYGONS and info["n"] == len(first) - 1
    ref = oracle.OraclePolygons(edges, first).render(tiles)["tri"]
    got = fill(hv, torch, h, tiles)
    check(got, ref, "fill c4 star polygons")
    hv.hv_free(h)


def test_fill_degenerate_geometry(hv, torch):
    """Degenerate rings placed on pixel-centre lines (tile-local px, centres
    at k + 0.5): zero-length edges, collinear vertices, edges along row and
    column centre lines, a bow-tie, two polygons sharing an edge, a hole
    touching its outer ring, a sliver thinner than 1e-9 px along a row line,
    and an 8000-edge ring spanning many edge chunks."""
    z, x, y = 12, 1500, 1700
    box = _box
    polys = [
        [[(10.5, 10.5), (10.5, 10.5), (20.5, 10.5), (25.5, 10.5), (30.5, 10.5), (30.5, 20.5), (10.5, 20.5)]],
        [box(40.0, 40.5, 60.0, 50.5)],                                        # top and bottom edges on row lines
        [box(70.5, 40.0, 80.5, 60.0)],                                        # left and right edges on column lines
        [[(100.0, 100.0), (120.0, 120.0), (120.0, 100.0), (100.0, 120.0)]],   # bow-tie
        [box(140.0, 100.0, 150.0, 110.0)], [box(150.0, 100.0, 160.0, 110.0)],  # shared edge x = 150
        [box(10.0, 140.0, 40.0, 170.0), [(10.0, 140.0), (20.0, 150.0), (30.0, 140.0)]],  # hole touching the ring
        [[(60.0, 150.5 - 1e-10), (90.0, 150.5 - 1e-10), (90.0, 150.5 + 1e-10), (60.0, 150.5 + 1e-10)]],  # sliver
    ]
    k = 8000
    ang = np.linspace(0.0, 2.0 * math.pi, k, endpoint=False)
    rad = 60.0 + 25.0 * np.sin(7.0 * ang)
    polys.append([[(190.0 + rad[q] * math.cos(ang[q]) * 0.8, 200.0 + rad[q] * math.sin(ang[q]) * 0.8) for q in range(k)]])
    e, f = _group(polys, z, x, y)
    h = build_polys(hv, torch, e, f, merc01=True)
    tiles = [(z, x, y), (z, x + 1, y), (z, x, y + 1), (z - 1, x // 2, y // 2), (z + 1, 2 * x, 2 * y)]
    log("fill degenerate geometry")
    ref = oracle.OraclePolygons(e, f, merc01=True).render(tiles)["tri"]
    got = fill(hv, torch, h, tiles)
    check(got, ref, "fill degenerate geometry")
    for L in (dict(region=64, waves_per_wg=4, cand_cap=256), dict(region=32, waves_per_wg=1, cand_cap=128, cull_nodes=1)):
        assert np.array_equal(fill(hv, torch, h, tiles, L), got), L
    hv.hv_free(h)


def test_fill_empty_index_and_far_tiles(hv, torch):
    e = hv.hv_polygon_index_build(None, [0])
    got = fill(hv, torch, e, [(0, 0, 0), (7, 3, 100)])
    assert not got.any()
    hv.hv_free(e)
