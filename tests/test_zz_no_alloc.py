"""hv_render_batch_noalloc (static device scratch, no allocation) against
hv_render_batch, the entry point it varies, through the C ABI.

Two no-allocation calls in a row on the same stream, the second with a
smaller batch, each compared byte for byte with hv_render_batch on the same
requests (the masks are bits, so equality is the bar); the scratch keeps the
first call's contents, so the second also shows that nothing of them leaks
into a later, smaller batch.  A batch over the static limit is rejected on
the host before any device work."""
import numpy as np
import pytest

import hvgen
from gpu_common import build, log

pytestmark = pytest.mark.gpu


def _mixed(rng, n, pts, segs, hp, hs, hv):
    """n requests over two indexes: zooms 0-14, radii 0.5-3 px, tiles drawn
    around random objects (so most of them hold data)."""
    ds = rng.integers(0, 2, n)
    z = rng.integers(0, 15, n)
    ip = rng.integers(0, len(pts), n)
    isg = rng.integers(0, len(segs), n)
    lon = np.where(ds == 0, pts[ip, 0], segs[isg, 0])
    lat = np.where(ds == 0, pts[ip, 1], segs[isg, 1])
    tiles = hvgen._tile_of_anchor(lon, lat, z)
    r = np.where(ds == 0, rng.uniform(1.0, 3.0, n), rng.integers(1, 6, n) / 2.0)
    return hv.requests(np.where(ds == 0, hp, hs).astype(np.uint64), tiles, r)


def test_noalloc_equals_render_batch_twice():
    import torch

    from paper_2005_12489_amd import hv
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    pts = hvgen.gen_c1_points(seed=11, n=50_000)
    segs = hvgen.gen_c2_segments(seed=12, n_segments=300_000)
    hp = build(hv, torch, pts, hv.HV_POINTS)
    hs = build(hv, torch, segs, hv.HV_SEGMENTS)
    rng = np.random.default_rng(2026)
    try:
        for n in (3000, 257):
            reqs = _mixed(rng, n, pts, segs, hp, hs, hv)
            want = torch.empty((n, hv.HV_MASK_BYTES), dtype=torch.uint8, device="cuda")
            got = torch.empty_like(want)
            want.fill_(0xA5)
            got.fill_(0x5A)
            log(f"noalloc: {n} requests, hv_render_batch")
            hv.hv_render_batch(reqs, want)
            torch.cuda.synchronize()
            log(f"noalloc: {n} requests, hv_render_batch_noalloc")
            hv.hv_render_batch_noalloc(reqs, got)
            torch.cuda.synchronize()
            a, b = want.cpu().numpy(), got.cpu().numpy()
            lit = int(np.unpackbits(a).sum())
            log(f"noalloc: {n} requests, {lit} lit pixels, {int((a != b).sum())} bytes differ")
            assert lit > 0
            assert np.array_equal(a, b), f"{n} requests: masks differ"
        # over the static limit: rejected before any device work, output untouched
        big = _mixed(rng, hv.HV_NOALLOC_MAX_REQUESTS + 1, pts, segs, hp, hs, hv)
        with pytest.raises(hv.HvError, match="HV_NOALLOC_MAX_REQUESTS"):
            hv.hv_render_batch_noalloc(big, got)
    finally:
        hv.hv_free(hp)
        hv.hv_free(hs)
