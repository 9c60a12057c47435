"""The full-size workloads in the launch the benchmark times (the graph-
captured batcher; for the 2e8 edges the autotuned shape, as bench.py picks
it): 1e9 clustered points with 10,000 requests at zooms 0-18, and 2e8 polygon
edges with 4,096 requests at zooms 2-20, as distance masks and as polygon
fills (hv_render_fill, default shape).

The oracle's masks for zoom-stratified samples of both -- 27 requests per
zoom: all of zooms 2-20 for the edges, zooms 3-18 for the points -- are
stored in tests/golden/fullsize_*.npz by tests/golden/make_fullsize_parity.py
(which calls only the oracle and the generators), with a fingerprint of the
inputs that is checked here first.  Every sampled pixel the oracle does not
flag as ambiguous must match, and the ambiguous pixels, counted over the
whole sample, must stay below 1e-6 of the pixels checked.  Properties that
hold at any size cover every tile: the masks of the whole set are the OR of
the masks of its two halves, and a point's own pixel is lit for r >=
sqrt(2)/2."""
import math
import os

import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import log
from helpers import AMBIGUOUS_LIMIT, input_fingerprint, parity, unpack_masks

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _batched(hv, torch, hs, tiles, r, launch=None):
    """All requests through one graph-captured batcher run (default shape, or
    the given launch)."""
    n = len(tiles)
    reqs = hv.requests(np.broadcast_to(np.asarray(hs, dtype=np.uint64), (n,)), tiles, r)
    levels = max(hv.hv_index_info(int(h))["levels"] for h in np.atleast_1d(hs))
    b = hv.hv_batcher_create(n, max_indexes=1, max_levels=levels, launch=launch)
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


def _check_golden(packed, name, objs, tiles, r, what):
    """The GPU masks of the stored sample against the oracle's stored masks."""
    g = np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz"))
    fp = input_fingerprint(objs[::1000], objs.shape[0], tiles, r)
    assert str(g["fingerprint"]) == fp, f"{what}: the inputs differ from those the stored oracle masks were made from"
    idx = g["idx"]
    assert np.array_equal(g["tiles"], tiles[idx]) and np.array_equal(g["r"], r[idx])
    lit = np.unpackbits(g["lit"], axis=-1, bitorder="little").astype(bool)
    amb = np.unpackbits(g["amb"], axis=-1, bitorder="little").astype(bool)
    tri = np.where(amb, 2, np.where(lit, 1, 0)).astype(np.uint8)
    got = unpack_masks(packed[idx])
    mism_per = ((got.astype(bool) != lit) & ~amb).reshape(len(idx), -1).sum(1)
    n_amb = int(amb.sum())
    for z in np.unique(tiles[idx, 0]):
        sel = tiles[idx, 0] == z
        log(f"{what} z{z}: {int(sel.sum())} tiles, lit={int(lit[sel].sum())} ambiguous={int(amb[sel].sum())} "
            f"mismatches={int(mism_per[sel].sum())}")
    bad = idx[mism_per > 0]
    assert len(bad) == 0, f"{what}: non-ambiguous mismatches in requests {bad[:10].tolist()}"
    px = tri.size
    log(f"{what}: {len(idx)} sampled tiles, {px} pixels, {n_amb} ambiguous ({n_amb / px:.2e})")
    assert n_amb <= AMBIGUOUS_LIMIT * px, f"{what}: {n_amb} ambiguous pixels over {px}"


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
    log("c3 full size: stored oracle masks of 27 requests per zoom at zooms 3-18")
    _check_golden(full, "c3", pts, tiles, r, "c3-full")


def test_c4_full_size(hv, torch):
    log("c4 full size: generate 2e8 edges")
    edges = hvgen.gen_c4_edges()
    tiles, r = hvgen.c4_requests(edges, n=4096)
    h = _build(hv, torch, edges, hv.HV_POLYGON_EDGES)
    log("c4 full size: autotune, then render 4096 requests in the tuned shape")
    reqs = hv.requests(h, tiles, r)
    scratch = torch.empty((len(tiles), 8192), dtype=torch.uint8, device="cuda")
    launch, _ = hv.hv_autotune(reqs, scratch)
    del scratch
    log(f"c4 full size: tuned launch {launch}")
    full = _batched(hv, torch, h, tiles, r, launch)
    assert np.array_equal(full, _batched(hv, torch, h, tiles, r)), "tuned and default shapes differ"
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
    log("c4 full size: stored oracle masks of 27 requests per zoom at zooms 2-20")
    _check_golden(full, "c4", edges, tiles, r, "c4-full")


def _aa_golden(hv, torch, name, objs, kind, tiles, r, what):
    """Anti-aliased values (0-4) of all requests, rendered in one launch in the
    autotuned shape, as bench.py times them, against the oracle's exact mode
    on the stored sample: equal wherever no sub-sample is within 1e-6 px of r,
    and otherwise within the bracket the ambiguous sub-samples allow."""
    g = np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz"))
    fp = input_fingerprint(objs[::1000], objs.shape[0], tiles, r)
    assert str(g["fingerprint"]) == fp, f"{what}: the inputs differ from those the stored oracle values were made from"
    idx = g["idx"]
    assert np.array_equal(g["tiles"], tiles[idx]) and np.array_equal(g["r"], r[idx])
    h = _build(hv, torch, objs, kind)
    reqs = hv.requests(h, tiles, r)
    scratch = torch.empty((len(tiles), 8192), dtype=torch.uint8, device="cuda")
    launch, _ = hv.hv_autotune(reqs, scratch)
    del scratch
    log(f"{what}: tuned launch {launch}")
    out = torch.empty((len(tiles), hv.HV_AA_BYTES), dtype=torch.uint8, device="cuda")
    out.fill_(0xA5)   # every value must be written
    hv.hv_render_batch_aa(reqs, out, launch)
    torch.cuda.synchronize()
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy().reshape(-1, 256, 256)
    del out
    torch.cuda.empty_cache()
    hv.hv_free(h)
    val, amb, sure = g["val"], g["amb"], g["sure"]
    clean = amb == 0
    assert got.max() <= 4
    bad = (got != val) & clean
    in_bracket = (got >= sure) & (got <= sure + amb)
    for z in np.unique(tiles[idx, 0]):
        sel = tiles[idx, 0] == z
        log(f"{what} z{z}: {int(sel.sum())} tiles, nonzero={int((val[sel] > 0).sum())} "
            f"ambiguous sub-samples={int(amb[sel].sum())} mismatches={int(bad[sel].sum())}")
    assert not bad.any(), f"{what}: {int(bad.sum())} values differ from the oracle"
    assert in_bracket[~clean].all(), f"{what}: a value outside its ambiguity bracket"
    n_amb = int(amb.sum())
    log(f"{what}: {len(idx)} sampled tiles, {4 * got.size} sub-samples, {n_amb} ambiguous")
    assert n_amb <= AMBIGUOUS_LIMIT * 4 * got.size, f"{what}: {n_amb} ambiguous sub-samples"


def test_c4_full_size_aa(hv, torch):
    """The 2e8 edges' 4,096 requests, anti-aliased, against 4 stored oracle
    requests per zoom at zooms 2-20."""
    log("c4 aa full size: generate 2e8 edges")
    edges = hvgen.gen_c4_edges()
    tiles, r = hvgen.c4_requests(edges, n=4096)
    _aa_golden(hv, torch, "c4_aa", edges, hv.HV_POLYGON_EDGES, tiles, r, "c4 aa")


def test_c3_full_size_aa(hv, torch):
    """The 1e9 points' 10,000 requests, anti-aliased, against 4 stored oracle
    requests per zoom at zooms 3-18."""
    log("c3 aa full size: generate 1e9 points")
    pts = hvgen.gen_c3_points(1_000_000_000)
    tiles, r = hvgen.c3_requests(10_000)
    _aa_golden(hv, torch, "c3_aa", pts, hv.HV_POINTS, tiles, r, "c3 aa")


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
    tiles, r = hvgen.c4_requests(edges, n=4096)
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
    log("c4 fill full size: stored oracle masks of 27 requests per zoom at zooms 2-20")
    _check_golden(full, "c4_fill", edges, tiles, r, "c4-fill-full")
