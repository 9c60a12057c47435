"""GPU masks against the CPU oracle, through the C ABI.

Bar: every pixel the oracle does not flag as ambiguous matches bit-exactly;
ambiguous pixels (|D - r| <= 1e-6 px) stay below 1e-6 of all pixels on the
synthetic workloads (closed-form cases with exact ties are compared on the
oracle's inclusive bit instead).
"""
import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import build, log, render, render_mixed
from helpers import AMBIGUOUS_LIMIT, parity, unpack_masks
from brute import merc01

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


def _assert_parity(bits, tri, what):
    mism, amb, lit = parity(bits, tri)
    px = tri.size
    log(f"{what}: pixels={px} lit={lit} ambiguous={amb} mismatches={mism}")
    assert mism == 0, f"{what}: {mism} non-ambiguous mismatches"
    assert amb <= AMBIGUOUS_LIMIT * px + 1e-9 or amb == 0, f"{what}: {amb} ambiguous pixels"


def test_c1_points_all_tiles(hv, torch):
    """10k uniform points, all 256 tiles of zoom 4, r = 2 px (full workload)."""
    pts = hvgen.gen_c1_points()
    tiles, r = hvgen.c1_requests()
    log("c1 build+render")
    h = build(hv, torch, pts, hv.HV_POINTS)
    bits = render(hv, torch, h, tiles, r)
    hv.hv_free(h)
    tri = oracle.OracleIndex(pts, oracle.POINTS).render(tiles, r)["tri"]
    _assert_parity(bits, tri, "c1")


def test_c2_linestrings_reduced(hv, torch):
    """The linestring recipe at 300k segments: dense and empty z6 tiles, plus z3 and z9."""
    segs = hvgen.gen_c2_segments(n_segments=300_000)
    m = merc01(segs[:, :2])
    rng = np.random.default_rng(21)
    t6 = np.unique(np.floor(m[rng.integers(0, len(m), 60)] * 64).astype(np.int32), axis=0)
    tiles6 = np.concatenate([np.column_stack([np.full(len(t6), 6), t6]),
                             hvgen.all_tiles(6)[rng.integers(0, 4096, 40)]])
    tiles3 = hvgen.all_tiles(3)
    t9 = np.floor(m[rng.integers(0, len(m), 40)] * 512).astype(np.int32)
    tiles9 = np.column_stack([np.full(len(t9), 9), t9])
    log("c2-reduced build")
    h = build(hv, torch, segs, hv.HV_SEGMENTS)
    ix = oracle.OracleIndex(segs, oracle.SEGMENTS)
    for tiles, r in ((tiles6, 0.5), (tiles3, 0.5), (tiles9, 1.5), (tiles6, 2.5)):
        log(f"c2-reduced render z={tiles[0, 0]} r={r} n={len(tiles)}")
        bits = render(hv, torch, h, tiles, r)
        _assert_parity(bits, ix.render(tiles, r)["tri"], f"c2-reduced z{tiles[0, 0]} r{r}")
    hv.hv_free(h)


def test_c2_linestrings_full_all_tiles(hv, torch):
    """Full 10M-segment workload: all 4096 z6 tiles in one graph-captured
    batcher launch (the benchmark's launch) and in one plain render, both
    checked against the oracle on every tile; the ambiguous pixels are
    counted over all 268M pixels."""
    segs = hvgen.gen_c2_segments()
    tiles, r = hvgen.c2_requests()
    log("c2-full build")
    h = build(hv, torch, segs, hv.HV_SEGMENTS)
    log("c2-full render 4096 tiles: batcher and plain call")
    reqs = hv.requests(h, tiles, r)
    levels = hv.hv_index_info(h)["levels"]
    b = hv.hv_batcher_create(len(tiles), max_indexes=1, max_levels=levels)
    out = torch.empty((len(tiles), 8192), dtype=torch.uint8, device="cuda")
    out.fill_(0x5A)
    hv.hv_batcher_run(b, reqs, out)
    torch.cuda.synchronize()
    hv.hv_batcher_free(b)
    bits = unpack_masks(out.cpu().numpy())
    del out
    plain = render(hv, torch, h, tiles, r)
    hv.hv_free(h)
    assert np.array_equal(bits, plain), "batcher and plain call differ"
    del plain
    log("c2-full oracle on all 4096 tiles")
    tri = oracle.OracleIndex(segs, oracle.SEGMENTS).render(tiles, r, want_bit=False)["tri"]
    _assert_parity(bits, tri, "c2-full")
    assert bits.sum() > 0


def test_points_mixed_zooms_and_radii(hv, torch):
    """The clustered-point recipe at 200k points; density-proportional tiles
    at zooms 0..18 with r ~ U[1,3]."""
    pts = hvgen.gen_c3_points(200_000)
    tiles, rs = hvgen.c3_requests(n=160)
    rs = np.round(rs * 4) / 4            # a few distinct radii -> fewer calls
    log("c3-reduced build")
    h = build(hv, torch, pts, hv.HV_POINTS)
    bits = render_mixed(hv, torch, h, tiles, rs)
    hv.hv_free(h)
    tri = oracle.OracleIndex(pts, oracle.POINTS).render(tiles, rs)["tri"]
    _assert_parity(bits, tri, "c3-reduced")


def test_polygon_edges_mixed(hv, torch):
    """The star-polygon recipe at ~150k edges; zooms 2..20, widths 1..5 px."""
    edges = hvgen.gen_c4_edges(min_edges=150_000, batch_polygons=5000)
    tiles, rs = hvgen.c4_requests(edges, n=160)
    log("c4-reduced build")
    h = build(hv, torch, edges, hv.HV_POLYGON_EDGES)
    bits = render_mixed(hv, torch, h, tiles, rs)
    hv.hv_free(h)
    tri = oracle.OracleIndex(edges, oracle.POLYGON_EDGES).render(tiles, rs)["tri"]
    _assert_parity(bits, tri, "c4-reduced")


@pytest.mark.parametrize("kind", [0, 1])
def test_seams_and_zoom_extremes(hv, torch, kind):
    """Objects straddling tile seams, at zooms 0, 7, 15, 20 and 22."""
    rng = np.random.default_rng(30 + kind)
    for z in (0, 7, 15, 20, 22):
        n = 1 << z
        x, y = (0, 0) if z == 0 else (int(rng.integers(1, n - 1)), int(rng.integers(1, n - 1)))
        S = 256.0 * 2.0 ** z
        u = rng.uniform(-12, 268, (300, 2))
        A = (np.array([256.0 * x, 256.0 * y]) + u) / S
        if kind == 0:
            objs = A
        else:
            B = (np.array([256.0 * x, 256.0 * y]) + u + rng.normal(0, 8, (300, 2))) / S
            B[:5] = A[:5]
            objs = np.concatenate([A, B], 1)
        objs = np.clip(objs, 0.0, 1.0)
        tiles = [(z, x, y)] if z == 0 else [(z, x, y), (z, x - 1, y), (z, x + 1, y), (z, x, y - 1), (z, x, y + 1)]
        flags = hv.HV_INPUT_MERC01 | (hv.HV_POINTS if kind == 0 else hv.HV_SEGMENTS)
        log(f"seams kind={kind} z={z}")
        h = build(hv, torch, objs, flags)
        ix = oracle.OracleIndex(objs, oracle.POINTS if kind == 0 else oracle.SEGMENTS, merc01=True)
        for r in (0.5, 1.0, 2.5, 64.0):
            bits = render(hv, torch, h, tiles, r)
            out = ix.render(tiles, r)
            mism, amb, _ = parity(bits, out["tri"])
            assert mism == 0, (z, r, mism)
        hv.hv_free(h)


def test_exact_ties_match_inclusive_bit(hv, torch):
    """Points on pixel centres and segments through centres / along pixel
    edges: exact distance ties; the GPU's d^2 <= r^2 must equal D <= r."""
    z, x, y = 10, 300, 400
    S = 256.0 * 2 ** z
    pts = np.array([[(256.0 * x + 100.5) / S, (256.0 * y + 50.5) / S],
                    [(256.0 * x + 10.0) / S, (256.0 * y + 200.0) / S],
                    [(256.0 * x + 0.5) / S, (256.0 * y + 128.5) / S]])
    h = build(hv, torch, pts, hv.HV_POINTS | hv.HV_INPUT_MERC01)
    ix = oracle.OracleIndex(pts, oracle.POINTS, merc01=True)
    tiles = [(z, x, y), (z, x - 1, y)]
    for r in (1.0, 2.0, 3.0, 5.0):
        log(f"ties points r={r}")
        assert np.array_equal(render(hv, torch, h, tiles, r), ix.render(tiles, r)["bit"]), r
    hv.hv_free(h)

    def seg(u0, v0, u1, v1):
        return [(256.0 * x + u0) / S, (256.0 * y + v0) / S, (256.0 * x + u1) / S, (256.0 * y + v1) / S]
    segs = np.array([seg(20.5, 77.5, 60.5, 77.5), seg(77.5, 20.5, 77.5, 60.5), seg(100.5, 140, 150.5, 140),
                     seg(10.5, 10.5, 30.5, 30.5), seg(200.5, 200.5, 200.5, 200.5)])
    h = build(hv, torch, segs, hv.HV_SEGMENTS | hv.HV_INPUT_MERC01)
    ix = oracle.OracleIndex(segs, oracle.SEGMENTS, merc01=True)
    for r in (0.5, 1.0, 2.0):
        log(f"ties segments r={r}")
        assert np.array_equal(render(hv, torch, h, [(z, x, y)], r), ix.render([(z, x, y)], r)["bit"]), r
    hv.hv_free(h)


def test_empty_and_tiny_indexes(hv, torch):
    h = hv.hv_index_build(None, hv.HV_POINTS, 0)
    log("empty index render")
    bits = render(hv, torch, h, [(0, 0, 0), (5, 3, 7)], 3.0)
    assert bits.sum() == 0
    hv.hv_free(h)
    for n in (1, 2, 15, 16, 17, 257):
        rng = np.random.default_rng(n)
        objs = np.column_stack([rng.uniform(10, 11, n), rng.uniform(45, 46, n)])
        log(f"tiny index n={n}")
        h = build(hv, torch, objs, hv.HV_POINTS)
        m = merc01(objs[:1])[0]
        tiles = [(z, int(m[0] * 2 ** z), int(m[1] * 2 ** z)) for z in (0, 4, 8, 12)]
        bits = render(hv, torch, h, tiles, 1.5)
        tri = oracle.OracleIndex(objs, oracle.POINTS).render(tiles, 1.5)["tri"]
        assert parity(bits, tri)[0] == 0, n
        hv.hv_free(h)


def test_duplicates_and_clamped_latitudes(hv, torch):
    """Identical objects (Hilbert ties) and latitudes beyond the Mercator limit."""
    rng = np.random.default_rng(40)
    base = np.column_stack([rng.uniform(-180, 180, 50), rng.uniform(84, 90, 50)])
    objs = np.concatenate([base] * 40 + [base[:, ::1] * [1, -1]])
    log("duplicates / clamped latitudes")
    h = build(hv, torch, objs, hv.HV_POINTS)
    tiles = np.concatenate([hvgen.all_tiles(2), [(5, k, 0) for k in range(0, 32, 3)], [(5, k, 31) for k in range(1, 32, 5)]])
    bits = render(hv, torch, h, tiles, 2.0)
    hv.hv_free(h)
    tri = oracle.OracleIndex(objs, oracle.POINTS).render(tiles, 2.0)["tri"]
    assert parity(bits, tri)[0] == 0
    assert bits.sum() > 0


def test_invalid_coordinates_rejected(hv, torch):
    for bad in ([[np.nan, 0.0]], [[181.0, 0.0]], [[0.0, 90.5]], [[0.0, -np.inf]]):
        t = torch.tensor(np.array(bad * 20, dtype=np.float64)).cuda()
        log(f"invalid coordinates {bad}")
        with pytest.raises(hv.HvError, match="non-finite|lon|lat") as e:
            hv.hv_index_build(t, hv.HV_POINTS)
        assert e.value.code == hv.HV_EINVAL


@pytest.mark.parametrize("kind", [0, 1])
def test_dense_low_zoom_accepts(hv, torch, kind):
    """Tree nodes far smaller than a pixel (dense clusters at zooms 0-6):
    containment accepts and skipping of fully lit ranges decide most pixels;
    every mode must still equal the oracle."""
    rng = np.random.default_rng(50 + kind)
    n = 400_000
    c = np.array([[12.0, 41.0], [-70.0, -20.0], [100.0, 30.0]])
    k = rng.integers(0, 3, n)
    a = c[k] + rng.normal(0, [[0.3], [1.5], [4.0]][0][0], (n, 2)) * np.array([1.0, 1.0])
    a = np.clip(a, [-179.9, -84.9], [179.9, 84.9])
    objs = a if kind == 0 else np.concatenate([a, np.clip(a + rng.normal(0, 0.01, (n, 2)), [-179.9, -84.9],
                                                          [179.9, 84.9])], 1)
    m = merc01(c)
    tiles = [(0, 0, 0)]
    for z in (2, 4, 6):
        for q in m:
            tiles.append((z, int(q[0] * 2 ** z), int(q[1] * 2 ** z)))
    tiles = np.array(tiles)
    log(f"dense low zoom kind={kind}")
    h = build(hv, torch, objs, kind)
    ix = oracle.OracleIndex(objs, kind)
    for r in (0.5, 1.0, 2.5):
        tri = ix.render(tiles, r)["tri"]
        ref = render(hv, torch, h, tiles, r)
        _assert_parity(ref, tri, f"dense kind={kind} r={r}")
        for L in (dict(region=64, waves_per_wg=4, cand_cap=256), dict(region=0, block=16, waves_per_wg=2),
                  dict(region=32, waves_per_wg=2, objs_per_lane=2, cand_cap=256)):
            assert np.array_equal(render(hv, torch, h, tiles, r, launch=L), ref), (r, L)
    hv.hv_free(h)


@pytest.mark.parametrize("kind", [0, 1])
def test_edge_accepts_small_clusters(hv, torch, kind):
    """Clusters whose bounding boxes are about as wide as the radius, so that
    edge accepts (a pixel within r of both ends of one side of a node box)
    decide many pixels at the very edge of what they may claim."""
    rng = np.random.default_rng(60 + kind)
    z0 = 5
    nclu = 3000
    per = 16 * rng.integers(1, 17, nclu)
    clon = rng.uniform(0.0, 45.0, nclu)
    clat = rng.uniform(22.0, 55.0, nclu)
    deg_px = 360.0 / (256 * 2 ** z0)
    ex = rng.uniform(0.05, 6.0, nclu) * deg_px
    ey = rng.uniform(0.05, 6.0, nclu) * deg_px * np.cos(np.radians(clat))
    idx = np.repeat(np.arange(nclu), per)
    m = len(idx)
    lon = clon[idx] + (rng.random(m) - 0.5) * ex[idx]
    lat = clat[idx] + (rng.random(m) - 0.5) * ey[idx]
    if kind == 0:
        objs = np.stack([lon, lat], 1)
    else:
        lon2 = clon[idx] + (rng.random(m) - 0.5) * ex[idx]
        lat2 = clat[idx] + (rng.random(m) - 0.5) * ey[idx]
        objs = np.stack([lon, lat, lon2, lat2], 1)
    anchors = merc01(np.stack([clon[:40], clat[:40]], 1))
    tiles = sorted({(z, int(q[0] * 2 ** z), int(q[1] * 2 ** z)) for z in range(3, 9) for q in anchors})
    tiles = np.array(tiles)
    log(f"edge accepts kind={kind} objects={m} tiles={len(tiles)}")
    h = build(hv, torch, objs, kind)
    ix = oracle.OracleIndex(objs, kind)
    for r in (0.5, 1.0, 1.7, 3.0):
        tri = ix.render(tiles, r)["tri"]
        ref = render(hv, torch, h, tiles, r)
        _assert_parity(ref, tri, f"edge accepts kind={kind} r={r}")
        for L in (dict(region=64, waves_per_wg=4, cand_cap=256), dict(region=0, block=16, waves_per_wg=2),
                  dict(region=32, waves_per_wg=2, objs_per_lane=2, cand_cap=256)):
            assert np.array_equal(render(hv, torch, h, tiles, r, launch=L), ref), (r, L)
    hv.hv_free(h)
