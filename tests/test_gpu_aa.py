"""Anti-aliased output (Algorithm 1's value 0-4 per pixel) on the GPU against
the oracle's exact mode, through the C ABI.

Bar: a pixel none of whose four sub-samples the oracle flags as ambiguous
(within 1e-6 px of r) has exactly the oracle's value; a pixel with a sub-samples
flagged has a value in [sure, sure + a], sure = its sub-samples certainly
within r.  Algorithm 1 as printed (the oracle's paper mode) never counts more.
"""
import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import build, log

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


def render_aa(hv, torch, hs, tiles, r, launch=None):
    tiles = np.asarray(tiles).reshape(-1, 3)
    hs = np.broadcast_to(np.asarray(hs, dtype=np.uint64), (tiles.shape[0],))
    reqs = hv.requests(hs, tiles, np.broadcast_to(np.asarray(r, dtype=np.float64), (tiles.shape[0],)))
    out = torch.empty((max(1, tiles.shape[0]), hv.HV_AA_BYTES), dtype=torch.uint8, device="cuda")
    out.fill_(0xA5)   # every value must be written
    hv.hv_render_batch_aa(reqs, out, launch)
    torch.cuda.synchronize()
    return out[:tiles.shape[0]].cpu().numpy().reshape(-1, 256, 256)


def check_aa(got, ref, what, paper=None):
    val, amb, sure = ref["val"], ref["amb"], ref["sure"]
    assert got.max() <= 4, what
    clean = amb == 0
    bad = int((got[clean] != val[clean]).sum())
    lo_ok = np.all(got[~clean] >= sure[~clean]) and np.all(got[~clean] <= sure[~clean] + amb[~clean])
    n_amb = int(amb.sum())
    log(f"{what}: pixels={got.size} nonzero={int((got > 0).sum())} ambiguous sub-samples={n_amb} "
        f"mismatches={bad}")
    assert bad == 0, f"{what}: {bad} values differ from the oracle"
    assert lo_ok, f"{what}: a value outside its ambiguity bracket"
    assert n_amb <= 1e-6 * 4 * got.size + 1e-9 or n_amb <= 4, f"{what}: {n_amb} ambiguous sub-samples"
    if paper is not None:
        ok = (paper["amb"] == 0) & clean
        assert np.all(paper["val"][ok] <= got[ok]), f"{what}: printed step counted more"
        log(f"{what}: Algorithm 1 as printed differs on {int((paper['val'][ok] != got[ok]).sum())} pixels")


def test_aa_points_c1_all_tiles(hv, torch):
    pts = hvgen.gen_c1_points()
    tiles, r = hvgen.c1_requests()
    log("aa c1")
    h = build(hv, torch, pts, hv.HV_POINTS)
    ix = oracle.OracleIndex(pts, oracle.POINTS)
    got = render_aa(hv, torch, h, tiles, r)
    check_aa(got, ix.render_aa(tiles, r), "aa c1", paper=ix.render_aa(tiles, r, mode="paper"))
    for L in (dict(region=64, waves_per_wg=4, cand_cap=256), dict(region=0, block=16, waves_per_wg=2),
              dict(region=32, waves_per_wg=1, objs_per_lane=2, cand_cap=128),
              dict(region=32, waves_per_wg=1, objs_per_lane=2, cand_cap=64, grid_wgs=1 << 20),
              dict(region=32, waves_per_wg=2, objs_per_lane=4, cand_cap=512, grid_wgs=7)):
        assert np.array_equal(render_aa(hv, torch, h, tiles, r, launch=L), got), L
    hv.hv_free(h)


@pytest.mark.parametrize("r", [0.5, 1.5])
def test_aa_linestrings(hv, torch, r):
    segs = hvgen.gen_c2_segments(n_segments=300_000)
    all6 = hvgen.all_tiles(6)
    rng = np.random.default_rng(61)
    tiles = all6[rng.choice(len(all6), 96, replace=False)]
    log(f"aa linestrings r={r}")
    h = build(hv, torch, segs, hv.HV_SEGMENTS)
    ix = oracle.OracleIndex(segs, oracle.SEGMENTS)
    got = render_aa(hv, torch, h, tiles, r)
    check_aa(got, ix.render_aa(tiles, r), f"aa linestrings r={r}", paper=ix.render_aa(tiles, r, mode="paper"))
    hv.hv_free(h)


def test_aa_points_mixed_zooms_and_radii(hv, torch):
    pts = hvgen.gen_c3_points(300_000)
    tiles, rr = hvgen.c3_requests(n=120, seed=33)
    log("aa clustered points, zooms 0-18")
    h = build(hv, torch, pts, hv.HV_POINTS)
    ix = oracle.OracleIndex(pts, oracle.POINTS)
    ref = ix.render_aa(tiles, rr)
    # the default split (zooms 0-1 as child tiles here), every request as
    # child tiles, and none
    for split in (0, -2, -1):
        L = {"region": 32, "objs_per_lane": 2, "aa_split": split}
        got = render_aa(hv, torch, h, tiles, rr, launch=L)
        check_aa(got, ref, f"aa clustered points, aa_split {split}")
        # the timing entry point renders the same values, with positive times
        out = torch.zeros((len(tiles), hv.HV_AA_BYTES), dtype=torch.uint8, device="cuda")
        ms = hv.hv_time_aa(hv.requests(h, tiles, rr), out, L, reps=2)
        torch.cuda.synchronize()
        assert ms[0] > 0 and ms[1] > 0, ms
        assert np.array_equal(out.cpu().numpy().reshape(-1, 256, 256), got), split
    hv.hv_free(h)


def test_aa_mixed_batch_and_extremes(hv, torch):
    segs = hvgen.gen_c2_segments(n_segments=100_000)
    pts = hvgen.gen_c1_points(n=5000)
    hs = [build(hv, torch, segs, hv.HV_SEGMENTS), build(hv, torch, pts, hv.HV_POINTS)]
    ixs = [oracle.OracleIndex(segs, oracle.SEGMENTS), oracle.OracleIndex(pts, oracle.POINTS)]
    # a point's own tile at z = 21 and z = 22 (the deepest zoom), tiny and large radii
    X, Y = oracle.project(pts[:1])
    deep = (21, int(X[0] * 2 ** 21), int(Y[0] * 2 ** 21))
    deepest = (22, int(X[0] * 2 ** 22), int(Y[0] * 2 ** 22))
    cases = [(1, (0, 0, 0), 0.1), (1, (0, 0, 0), 64.0), (1, deep, 0.3), (1, deep, 3.0), (0, (3, 4, 3), 2.5),
             (0, (5, 9, 12), 0.5), (1, (4, 7, 6), 1.0), (0, (0, 0, 0), 0.5), (1, deepest, 0.36),
             (1, deepest, 2.0)]
    ds = np.array([c[0] for c in cases])
    tiles = np.array([c[1] for c in cases])
    rs = np.array([c[2] for c in cases])
    log("aa mixed batch over two indexes")
    refs = [ixs[d].render_aa(tiles[ds == d], rs[ds == d]) for d in (0, 1)]
    # with aa_split -2, the zoom-22 and r = 64 requests stay in one pass; the
    # last launch renders child tiles one wavefront per pixel block
    for L in ({"region": 32, "objs_per_lane": 2}, {"region": 32, "objs_per_lane": 2, "aa_split": -2},
              {"region": 32, "aa_split": -1}, {"aa_split": 1}):
        split = L.get("aa_split", 0)
        got = render_aa(hv, torch, np.array(hs, dtype=np.uint64)[ds], tiles, rs, launch=L)
        for d in (0, 1):
            check_aa(got[ds == d], refs[d], f"aa mixed dataset {d}, aa_split {split}")
    for h in hs:
        hv.hv_free(h)


def test_aa_c2_full_size_all_tiles(hv, torch):
    """The full 10M-segment workload, anti-aliased: all 4096 zoom-6 tiles in one
    call (one pass: 10M segments are below the default split at zoom 6),
    each against the oracle's exact mode; the ambiguous sub-samples are
    counted over all 1.07e9 of them."""
    segs = hvgen.gen_c2_segments()
    tiles, r = hvgen.c2_requests()
    log("aa c2-full build")
    h = build(hv, torch, segs, hv.HV_SEGMENTS)
    log("aa c2-full render 4096 tiles")
    got = render_aa(hv, torch, h, tiles, r)
    hv.hv_free(h)
    log("aa c2-full oracle on all 4096 tiles")
    ref = oracle.OracleIndex(segs, oracle.SEGMENTS).render_aa(tiles, r)
    del segs
    check_aa(got, ref, "aa c2-full")
    assert (got > 0).sum() > 0
