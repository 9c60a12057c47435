"""GPU index structure, determinism and launch-shape invariance, through the C ABI."""
import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import build, log, render
from helpers import hilbert_np, parity

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


@pytest.mark.parametrize("kind,n", [(0, 100_000), (1, 250_000), (0, 37), (1, 16)])
def test_structure(hv, torch, kind, n):
    """Sorted order is a stable sort by Hilbert key of the box centre; every
    object lies in its leaf box; every child box lies in its parent's; the
    root is the data's bounding box; projection agrees with the oracle's."""
    objs = hvgen.gen_c1_points(seed=5, n=n) if kind == 0 else hvgen.gen_c2_segments(seed=6, n_segments=n)
    log(f"structure kind={kind} n={n}")
    h = build(hv, torch, objs, kind)
    info = hv.hv_index_info(h)
    order = hv.hv_index_read(h, hv.HV_READ_ORDER).astype(np.int64)
    P = hv.hv_index_read(h, hv.HV_READ_OBJECTS)
    assert np.array_equal(np.sort(order), np.arange(n))
    # projection: against the oracle's, a few ulp
    w = 2 if kind == 0 else 4
    ox, oy = oracle.project(objs.reshape(-1, 2))
    O = np.stack([ox, oy], 1).reshape(-1, w)[order]
    assert np.max(np.abs(P - O)) <= 4e-16
    # keys from the GPU's own projected coordinates
    bits = info["key_bits"]
    if kind == 0:
        cx, cy = P[:, 0], P[:, 1]
    else:
        cx = 0.5 * (np.minimum(P[:, 0], P[:, 2]) + np.maximum(P[:, 0], P[:, 2]))
        cy = 0.5 * (np.minimum(P[:, 1], P[:, 3]) + np.maximum(P[:, 1], P[:, 3]))
    s = 2.0 ** bits
    qx = np.clip(np.floor(cx * s), 0, s - 1)
    qy = np.clip(np.floor(cy * s), 0, s - 1)
    key = hilbert_np(qx, qy, bits)
    assert np.all(key[1:] >= key[:-1]), "not sorted by Hilbert key"
    tie = key[1:] == key[:-1]
    assert np.all(order[1:][tie] > order[:-1][tie]), "equal keys out of input order"
    # boxes
    L, F = info["leaf_size"], info["fanout"]
    leaves = hv.hv_index_read(h, hv.HV_READ_NODES, 0)
    owner = np.arange(n) // L
    xs = P[:, 0::2]
    ys = P[:, 1::2]
    assert np.array_equal(leaves[:, 0], np.minimum.reduceat(xs.min(1), np.arange(0, n, L)))
    assert np.all(xs.min(1) >= leaves[owner, 0]) and np.all(xs.max(1) <= leaves[owner, 2])
    assert np.all(ys.min(1) >= leaves[owner, 1]) and np.all(ys.max(1) <= leaves[owner, 3])
    prev = leaves
    for lvl in range(1, info["levels"]):
        cur = hv.hv_index_read(h, hv.HV_READ_NODES, lvl)
        par = np.arange(len(prev)) // F
        assert np.all(prev[:, 0] >= cur[par, 0]) and np.all(prev[:, 1] >= cur[par, 1])
        assert np.all(prev[:, 2] <= cur[par, 2]) and np.all(prev[:, 3] <= cur[par, 3])
        assert np.array_equal(cur[:, 0], np.minimum.reduceat(prev[:, 0], np.arange(0, len(prev), F)))
        prev = cur
    assert len(prev) == 1
    root = prev[0]
    assert np.array_equal(root, [xs.min(), ys.min(), xs.max(), ys.max()])
    assert np.array_equal(root, info["root"])
    hv.hv_free(h)


def test_deterministic_and_permutation_invariant(hv, torch):
    segs = hvgen.gen_c2_segments(seed=7, n_segments=200_000)
    tiles = hvgen.all_tiles(5)
    log("determinism")
    h1 = build(hv, torch, segs, hv.HV_SEGMENTS)
    h2 = build(hv, torch, segs, hv.HV_SEGMENTS)
    perm = np.random.default_rng(1).permutation(len(segs))
    h3 = build(hv, torch, segs[perm], hv.HV_SEGMENTS)
    a = render(hv, torch, h1, tiles, 1.0)
    b = render(hv, torch, h2, tiles, 1.0)
    c = render(hv, torch, h3, tiles, 1.0)
    assert np.array_equal(hv.hv_index_read(h1, hv.HV_READ_OBJECTS), hv.hv_index_read(h2, hv.HV_READ_OBJECTS))
    assert np.array_equal(a, b)
    # a different input order can change the layout only where keys tie, never the masks
    tri = oracle.OracleIndex(segs, oracle.SEGMENTS).render(tiles, 1.0)["tri"]
    assert parity(a, tri)[0] == 0 and parity(c, tri)[0] == 0
    assert np.array_equal(a[tri != 2], c[tri != 2])
    for h in (h1, h2, h3):
        hv.hv_free(h)


SHAPES = [dict(block=b, cand_cap=c, waves_per_wg=w, grid_wgs=g)
          for b in (8, 16, 32) for c in (64, 128, 512) for w in (1, 2, 4) for g in (0, 7)
          if not (c == 512 and w == 4)]
SHAPES += [dict(region=rs, cand_cap=64 * w * o, waves_per_wg=w, objs_per_lane=o)
           for rs in (32, 64) for w in (1, 2, 4) for o in (1, 2, 4)]
SHAPES += [dict(region=rs, cand_cap=512, waves_per_wg=w, objs_per_lane=o, grid_wgs=7)
           for rs in (32, 64) for w, o in ((1, 1), (2, 4))]
# queues below a leaf step's objects: they take them 64 * waves at a time
SHAPES += [dict(region=rs, cand_cap=c * w, waves_per_wg=w, objs_per_lane=o, grid_wgs=g)
           for rs, c, w, o, g in ((32, 64, 1, 2, 0), (32, 64, 1, 2, 1 << 20), (32, 96, 1, 2, 0), (32, 64, 2, 4, 0),
                                  (32, 160, 1, 4, 7), (64, 64, 4, 2, 0))]
# cull depth: from the root alone to a deep frontier
SHAPES += [dict(region=32, cand_cap=128, waves_per_wg=1, objs_per_lane=2, cull_nodes=c) for c in (1, 3, 16, 64, 255)]
SHAPES += [dict(block=16, cand_cap=64, waves_per_wg=2, cull_nodes=c) for c in (1, 40)]


def test_launch_shapes_identical(hv, torch):
    """Every launch shape (block size, LDS candidate capacity -- 64 forces a
    flush after every leaf step, less than a step's objects flushes within
    it --, waves per workgroup, persistent grid
    size, including a 7-workgroup grid that makes each wave loop over many
    blocks, and the cull depth of the per-tile pass) gives bit-identical
    masks."""
    segs = hvgen.gen_c2_segments(seed=8, n_segments=400_000)
    pts = hvgen.gen_c3_points(300_000)
    edges = hvgen.gen_c4_edges(seed=12, min_edges=60_000, batch_polygons=2000)
    rng = np.random.default_rng(9)
    t12, _ = hvgen.c4_requests(edges, n=24, seed=13, zlo=11, zhi=14)
    cases = ((segs, hv.HV_SEGMENTS, hvgen.all_tiles(4), 1.5),
             (pts, hv.HV_POINTS, np.concatenate([hvgen.all_tiles(3), hvgen.all_tiles(7)[rng.integers(0, 16384, 64)]]), 2.0),
             # large pixel ranges: wide points and long edges at high zoom
             (pts[:20000], hv.HV_POINTS, hvgen.all_tiles(3), 40.0),
             (edges, hv.HV_POLYGON_EDGES, t12, 2.5))
    for objs, kind, tiles, r in cases:
        h = build(hv, torch, objs, kind)
        ref = None
        for s in SHAPES:
            log(f"shape kind={kind} {s}")
            bits = render(hv, torch, h, tiles, r, launch=s)
            if ref is None:
                ref = bits
            assert np.array_equal(bits, ref), s
        one = render(hv, torch, h, tiles[:12], r, one_per_call=True)
        assert np.array_equal(one, ref[:12])
        hv.hv_free(h)


def test_side_stream(hv, torch):
    pts = hvgen.gen_c1_points()
    tiles, r = hvgen.c1_requests()
    h = build(hv, torch, pts, hv.HV_POINTS)
    ref = render(hv, torch, h, tiles, r)
    s = torch.cuda.Stream()
    log("side stream")
    with torch.cuda.stream(s):
        out = torch.empty((len(tiles), 8192), dtype=torch.uint8, device="cuda")
        hv.hv_render_tiles(h, tiles, r, out)
    s.synchronize()
    from helpers import unpack_masks
    assert np.array_equal(unpack_masks(out.cpu().numpy()), ref)
    hv.hv_free(h)
