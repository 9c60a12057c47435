"""Batches of heterogeneous requests (mixed datasets, zooms, styles) in one
launch; the graph-captured batcher; the autotuner.  Each request's mask must
be the same alone and in the mix, and match the oracle."""
import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import build, log, render
from helpers import parity, unpack_masks

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


@pytest.fixture(scope="module")
def world(hv, torch):
    """Three resident indexes and a mixed request stream over them."""
    segs = hvgen.gen_c2_segments(n_segments=300_000)
    pts = hvgen.gen_c3_points(200_000)
    edges = hvgen.gen_c4_edges(min_edges=120_000, batch_polygons=4000)
    log("batch world: build 3 indexes")
    hs = [build(hv, torch, segs, hv.HV_SEGMENTS), build(hv, torch, pts, hv.HV_POINTS),
          build(hv, torch, edges, hv.HV_POLYGON_EDGES)]
    objs = [segs, pts, edges]
    kinds = [oracle.SEGMENTS, oracle.POINTS, oracle.POLYGON_EDGES]
    rng = np.random.default_rng(77)
    t2 = hvgen.c5_arrivals(2000.0, c2_objects=segs, max_requests=150, seed=8)
    t3, r3 = hvgen.c3_requests(n=100, seed=31)
    t4, r4 = hvgen.c4_requests(edges, n=100, seed=41)
    ds = np.concatenate([np.zeros(150, int), np.ones(100, int), np.full(100, 2)])
    tiles = np.concatenate([t2["tiles"], t3, t4])
    r = np.concatenate([np.round(t2["r"] * 2) / 2, np.round(r3 * 2) / 2, r4])
    perm = rng.permutation(len(ds))
    yield dict(hs=hs, objs=objs, kinds=kinds, ds=ds[perm], tiles=tiles[perm], r=r[perm])
    for h in hs:
        hv.hv_free(h)


def _batch(hv, torch, w, sel=None, launch=None):
    sel = np.arange(len(w["ds"])) if sel is None else sel
    reqs = hv.requests(np.array(w["hs"], dtype=np.uint64)[w["ds"][sel]], w["tiles"][sel], w["r"][sel])
    out = torch.empty((len(sel), 8192), dtype=torch.uint8, device="cuda")
    out.fill_(0x5A)
    hv.hv_render_batch(reqs, out, launch)
    torch.cuda.synchronize()
    return unpack_masks(out.cpu().numpy()), reqs


def test_mixed_batch_alone_vs_mix_and_oracle(hv, torch, world):
    w = world
    log(f"mixed batch of {len(w['ds'])} requests")
    mix, _ = _batch(hv, torch, w)
    for k in range(len(w["ds"])):
        alone = render(hv, torch, w["hs"][w["ds"][k]], w["tiles"][k:k + 1], float(w["r"][k]))
        assert np.array_equal(alone[0], mix[k]), k
    for d in range(3):
        sel = np.nonzero(w["ds"] == d)[0]
        tri = oracle.OracleIndex(w["objs"][d], w["kinds"][d]).render(w["tiles"][sel], w["r"][sel])["tri"]
        mism, amb, lit = parity(mix[sel], tri)
        log(f"dataset {d}: {len(sel)} requests, lit={lit} ambiguous={amb} mismatches={mism}")
        assert mism == 0


def test_mixed_batch_every_mode_identical(hv, torch, world):
    ref, _ = _batch(hv, torch, world)
    for L in (dict(region=64, waves_per_wg=4, cand_cap=256), dict(region=0, block=16, waves_per_wg=2),
              dict(region=0, block=8, waves_per_wg=4), dict(region=32, waves_per_wg=2, objs_per_lane=2,
                                                             cand_cap=256)):
        log(f"mixed batch shape {L}")
        got, _ = _batch(hv, torch, world, launch=L)
        assert np.array_equal(got, ref), L


def test_batcher_graph_replays(hv, torch, world):
    """A captured graph replayed with different batches, eager work and
    synchronisation in between; every replay equals the eager batch."""
    w = world
    b = hv.hv_batcher_create(512, max_indexes=4, max_levels=12)
    try:
        rng = np.random.default_rng(5)
        for rep in range(5):
            n = [350, 120, 350, 1, 200][rep]
            sel = rng.choice(len(w["ds"]), n, replace=False)
            reqs = hv.requests(np.array(w["hs"], dtype=np.uint64)[w["ds"][sel]], w["tiles"][sel], w["r"][sel])
            out = torch.empty((n, 8192), dtype=torch.uint8, device="cuda")
            out.fill_(0xC3)
            log(f"batcher replay {rep} n={n}")
            hv.hv_batcher_run(b, reqs, out)
            lat = hv.hv_batcher_latency(b, n)
            got = unpack_masks(out.cpu().numpy())
            eager, _ = _batch(hv, torch, w, sel)
            assert np.array_equal(got, eager), rep
            assert np.all(lat >= 0) and np.all(np.isfinite(lat)) and lat.max() < 1e6
            # eager work in between replays
            torch.cuda.synchronize()
            x = torch.randn(1 << 20, device="cuda")
            float(x.sum())
        # two runs in flight back to back on the stream
        sel = np.arange(64)
        reqs = hv.requests(np.array(w["hs"], dtype=np.uint64)[w["ds"][sel]], w["tiles"][sel], w["r"][sel])
        o1 = torch.empty((64, 8192), dtype=torch.uint8, device="cuda")
        o2 = torch.empty((64, 8192), dtype=torch.uint8, device="cuda")
        hv.hv_batcher_run(b, reqs, o1)
        hv.hv_batcher_run(b, reqs, o2)
        torch.cuda.synchronize()
        assert torch.equal(o1, o2)
        with pytest.raises(hv.HvError, match="max_requests"):
            hv.hv_batcher_run(b, hv.requests(w["hs"][0], np.zeros((513, 3), int), 1.0), o1)
    finally:
        hv.hv_batcher_free(b)


def test_batcher_switches_default_shape_by_size(hv, torch, world):
    """A default batcher holds one graph per size class of the default shape
    (4 waves per region below 1024 requests, 2 below 4096, 1 beyond); runs
    that cross the classes in turn equal one fixed explicit shape."""
    w = world
    b = hv.hv_batcher_create(4500, max_indexes=3, max_levels=12)
    rng = np.random.default_rng(12)
    fixed = dict(region=32, waves_per_wg=1, objs_per_lane=2, cand_cap=128)
    try:
        for n in (4500, 300, 2000, 1023, 1024, 4096, 4095, 1):
            sel = rng.integers(0, len(w["ds"]), n)
            reqs = hv.requests(np.array(w["hs"], dtype=np.uint64)[w["ds"][sel]], w["tiles"][sel], w["r"][sel])
            out = torch.empty((n, 8192), dtype=torch.uint8, device="cuda")
            out.fill_(0x69)
            log(f"default batcher n={n}")
            hv.hv_batcher_run(b, reqs, out)
            torch.cuda.synchronize()
            ref, _ = _batch(hv, torch, w, sel, launch=fixed)
            assert np.array_equal(unpack_masks(out.cpu().numpy()), ref), n
    finally:
        hv.hv_batcher_free(b)


def test_autotune_caches_a_valid_shape(hv, torch, world):
    w = world
    _, reqs = _batch(hv, torch, w)
    scratch = torch.empty((len(reqs), 8192), dtype=torch.uint8, device="cuda")
    log("autotune")
    best, ms = hv.hv_autotune(reqs, scratch)
    assert ms > 0 and best in [hv.hv_tuned_launch(reqs)]
    ref, _ = _batch(hv, torch, w, launch=dict(region=32, waves_per_wg=1, cand_cap=64))
    tuned, _ = _batch(hv, torch, w)           # launch=None -> the cached shape
    assert np.array_equal(tuned, ref)
