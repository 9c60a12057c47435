"""The full-size workloads in the launch the benchmark times (the graph-
captured batcher, default shape): 1e9 clustered points with 10,000 requests
at zooms 0-18, and 2e8 polygon edges with 4,096 requests at zooms 2-20, as
distance masks and as polygon fills (hv_render_fill, default shape).

At this size the oracle cannot index everything on the host, so it checks
sampled tiles at zoom >= 10 over the objects whose bounding box comes within
4 px of them (a superset of every object that can reach the tile), and
properties that hold at any size cover every tile: the masks of the whole
set are the OR of the masks of its two halves, and a point's own pixel is
lit for r >= sqrt(2)/2."""
import math

import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import log
from helpers import AMBIGUOUS_LIMIT, parity, unpack_masks

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


def _build(hv, torch, objs, kind):
    t = torch.from_numpy(objs).cuda()
    torch.cuda.synchronize()
    h = hv.hv_index_build(t, kind)
    del t
    torch.cuda.empty_cache()
    return h


def _batched(hv, torch, hs, tiles, r):
    """All requests through one graph-captured batcher run (default shape)."""
    n = len(tiles)
    reqs = hv.requests(np.broadcast_to(np.asarray(hs, dtype=np.uint64), (n,)), tiles, r)
    levels = max(hv.hv_index_info(int(h))["levels"] for h in np.atleast_1d(hs))
    b = hv.hv_batcher_create(n, max_indexes=1, max_levels=levels)
    out = torch.empty((n, 8192), dtype=torch.uint8, device="cuda")
    out.fill_(0x5A)
    hv.hv_batcher_run(b, reqs, out)
    torch.cuda.synchronize()
    hv.hv_batcher_free(b)
    return out.cpu().numpy()


def _lonlat_box(z, x, y, margin_px):
    """lon/lat bounds of tile (z, x, y) grown by margin_px pixels (exact
    inverse of the Mercator projection at the grown edges)."""
    S = 256.0 * 2 ** z
    u0, u1 = (256.0 * x - margin_px) / S, (256.0 * (x + 1) + margin_px) / S
    v0, v1 = (256.0 * y - margin_px) / S, (256.0 * (y + 1) + margin_px) / S
    lon0, lon1 = u0 * 360.0 - 180.0, u1 * 360.0 - 180.0
    lat = lambda v: math.degrees(math.atan(math.sinh(math.pi * (1.0 - 2.0 * v))))
    return lon0, lon1, lat(min(v1, 1.0)), lat(max(v0, 0.0))


def _deep_sample(tiles, k, zmin=10):
    deep = np.nonzero(tiles[:, 0] >= zmin)[0]
    return deep[np.linspace(0, len(deep) - 1, k).astype(int)]


def _check_sample(packed, objs, kind, tiles, r, pick, what):
    for t in pick:
        z, x, y = (int(v) for v in tiles[t])
        lon0, lon1, lat0, lat1 = _lonlat_box(z, x, y, 4.0 + float(np.max(r)))
        if kind == oracle.POINTS:
            sel = (objs[:, 0] >= lon0) & (objs[:, 0] <= lon1) & (objs[:, 1] >= lat0) & (objs[:, 1] <= lat1)
        else:
            lo_x = np.minimum(objs[:, 0], objs[:, 2])
            hi_x = np.maximum(objs[:, 0], objs[:, 2])
            lo_y = np.minimum(objs[:, 1], objs[:, 3])
            hi_y = np.maximum(objs[:, 1], objs[:, 3])
            sel = (hi_x >= lon0) & (lo_x <= lon1) & (hi_y >= lat0) & (lo_y <= lat1)
        sub = objs[sel]
        got = unpack_masks(packed[t:t + 1])
        if sub.shape[0] == 0:
            assert not got.any(), (what, t)
            continue
        tri = oracle.OracleIndex(sub, kind).render(tiles[t:t + 1], float(np.asarray(r)[t]))["tri"]
        mism, amb, lit = parity(got, tri)
        log(f"{what} tile {tuple(tiles[t])}: objects near={sub.shape[0]} lit={lit} ambiguous={amb} mismatches={mism}")
        assert mism == 0, (what, tuple(tiles[t]))
        assert amb <= AMBIGUOUS_LIMIT * 65536 + 1e-9 or amb <= 2, (what, tuple(tiles[t]), amb)


def test_c3_full_size(hv, torch):
    n = 1_000_000_000
    log("c3 full size: generate 1e9 points")
    pts = hvgen.gen_c3_points(n)
    tiles, r = hvgen.c3_requests(10_000)
    h = _build(hv, torch, pts, hv.HV_POINTS)
    log("c3 full size: render 10000 requests")
    full = _batched(hv, torch, h, tiles, r)
    hv.hv_free(h)
    # union over two halves, every tile
    log("c3 full size: halves")
    ha = _build(hv, torch, pts[: n // 2], hv.HV_POINTS)
    a = _batched(hv, torch, ha, tiles, r)
    hv.hv_free(ha)
    hb = _build(hv, torch, pts[n // 2:], hv.HV_POINTS)
    b = _batched(hv, torch, hb, tiles, r)
    hv.hv_free(hb)
    assert np.array_equal(full, a | b), "whole set = OR of its halves"
    # own pixel of sampled points (r >= 1 > sqrt(2)/2)
    rng = np.random.default_rng(91)
    idx = rng.integers(0, n, 512)
    X, Y = oracle.project(pts[idx])
    z = rng.integers(0, 19, 512)
    own = np.stack([z, (X * 2.0 ** z).astype(np.int64), (Y * 2.0 ** z).astype(np.int64)], 1)
    h = _build(hv, torch, pts, hv.HV_POINTS)
    m = unpack_masks(_batched(hv, torch, h, own, np.full(512, 1.0)))
    hv.hv_free(h)
    S = 256.0 * 2.0 ** z
    i = np.minimum((X * S - 256.0 * own[:, 1]).astype(np.int64), 255)
    j = np.minimum((Y * S - 256.0 * own[:, 2]).astype(np.int64), 255)
    assert m[np.arange(512), j, i].all(), "a point's own pixel is lit"
    pick = _deep_sample(tiles, 6)
    log(f"c3 full size: oracle on {len(pick)} sampled tiles")
    _check_sample(full, pts, oracle.POINTS, tiles, r, pick, "c3-full")


def test_c4_full_size(hv, torch):
    log("c4 full size: generate 2e8 edges")
    edges = hvgen.gen_c4_edges()
    tiles, r = hvgen.c4_requests(edges, n=4096)
    h = _build(hv, torch, edges, hv.HV_POLYGON_EDGES)
    log("c4 full size: render 4096 requests")
    full = _batched(hv, torch, h, tiles, r)
    hv.hv_free(h)
    n = edges.shape[0]
    log("c4 full size: halves")
    ha = _build(hv, torch, edges[: n // 2], hv.HV_POLYGON_EDGES)
    a = _batched(hv, torch, ha, tiles, r)
    hv.hv_free(ha)
    hb = _build(hv, torch, edges[n // 2:], hv.HV_POLYGON_EDGES)
    b = _batched(hv, torch, hb, tiles, r)
    hv.hv_free(hb)
    assert np.array_equal(full, a | b), "whole set = OR of its halves"
    pick = _deep_sample(tiles, 6)
    log(f"c4 full size: oracle on {len(pick)} sampled tiles")
    _check_sample(full, edges, oracle.POLYGON_EDGES, tiles, r, pick, "c4-full")


def _check_fill_sample(packed, edges, first, tiles, pick, what):
    """Oracle fill of sampled tiles over the polygons whose bounding box meets
    the tile grown by 4 px (a superset of every polygon that can hold one of
    its pixel centres)."""
    lo_x = np.minimum.reduceat(np.minimum(edges[:, 0], edges[:, 2]), first[:-1])
    hi_x = np.maximum.reduceat(np.maximum(edges[:, 0], edges[:, 2]), first[:-1])
    lo_y = np.minimum.reduceat(np.minimum(edges[:, 1], edges[:, 3]), first[:-1])
    hi_y = np.maximum.reduceat(np.maximum(edges[:, 1], edges[:, 3]), first[:-1])
    for t in pick:
        z, x, y = (int(v) for v in tiles[t])
        lon0, lon1, lat0, lat1 = _lonlat_box(z, x, y, 4.0)
        sel = np.nonzero((hi_x >= lon0) & (lo_x <= lon1) & (hi_y >= lat0) & (lo_y <= lat1))[0]
        got = unpack_masks(packed[t:t + 1])
        if len(sel) == 0:
            assert not got.any(), (what, t)
            continue
        sub = np.concatenate([edges[first[p]:first[p + 1]] for p in sel])
        sub_first = np.concatenate([[0], np.cumsum(first[sel + 1] - first[sel])])
        tri = oracle.OraclePolygons(sub, sub_first).render(tiles[t:t + 1])["tri"]
        clean = tri != 2
        bad = int((got[clean] != tri[clean]).sum())
        log(f"{what} tile {tuple(tiles[t])}: polygons near={len(sel)} filled={int(got.sum())} "
            f"ambiguous={int((~clean).sum())} mismatches={bad}")
        assert bad == 0, (what, tuple(tiles[t]))


def _fill(hv, torch, edges, first, tiles):
    d = torch.from_numpy(edges).cuda()
    torch.cuda.synchronize()
    h = hv.hv_polygon_index_build(d, first)
    del d
    torch.cuda.empty_cache()
    out = torch.empty((len(tiles), 8192), dtype=torch.uint8, device="cuda")
    out.fill_(0x77)
    hv.hv_render_fill(h, hv.tiles_array(tiles), out, None)
    torch.cuda.synchronize()
    hv.hv_free(h)
    res = out.cpu().numpy()
    del out
    torch.cuda.empty_cache()
    return res


def test_c4_fill_full_size(hv, torch):
    log("c4 fill full size: generate 2e8 edges")
    edges = hvgen.gen_c4_edges()
    first = hvgen.c4_polygon_first(edges)
    tiles, _ = hvgen.c4_requests(edges, n=4096)
    log(f"c4 fill full size: {len(first) - 1} polygons, 4096 requests")
    full = _fill(hv, torch, edges, first, tiles)
    # the fill of a set of polygons is the OR of the fills of any split of it
    log("c4 fill full size: halves")
    half = (len(first) - 1) // 2
    a = _fill(hv, torch, edges[: first[half]], first[: half + 1], tiles)
    b = _fill(hv, torch, edges[first[half]:], first[half:] - first[half], tiles)
    assert np.array_equal(full, a | b), "whole set = OR of its halves"
    assert full.any() and not full.all()
    # deep tiles, and two at zoom 4-5 where regions hold thousands of polygons
    low = np.nonzero((tiles[:, 0] >= 4) & (tiles[:, 0] <= 5))[0][:2]
    pick = np.concatenate([_deep_sample(tiles, 6, zmin=8), low])
    log(f"c4 fill full size: oracle on {len(pick)} sampled tiles")
    _check_fill_sample(full, edges, first, tiles, pick, "c4-fill-full")
