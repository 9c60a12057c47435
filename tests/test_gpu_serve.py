"""Serving on the GPU: Poisson arrivals over two resident indexes, admitted
and batched as they arrive on two streams.  Each served mask must equal the
same request rendered alone, and the oracle."""
import numpy as np
import pytest

import hvgen
import oracle
from gpu_common import build, log
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


def test_served_equals_alone_and_oracle(hv, torch):
    from paper_2005_12489_amd import serve
    segs = hvgen.gen_c2_segments(n_segments=300_000)
    pts = hvgen.gen_c3_points(300_000)
    log("serve: build two indexes")
    h2, h3 = build(hv, torch, segs, hv.HV_SEGMENTS), build(hv, torch, pts, hv.HV_POINTS)
    arr = hvgen.c5_arrivals(20000.0, c2_objects=segs, max_requests=3000, zmax=14)
    ds = arr["dataset"]
    reqs = hv.requests(np.where(ds == 0, h2, h3).astype(np.uint64), arr["tiles"], arr["r"])
    ex = serve.GpuExecutor(reqs, streams=2, max_batch=512, max_indexes=2, max_levels=12, keep_masks=True)
    log("serve: 3000 requests at 20k req/s")
    st = serve.serve(arr["t"], serve.Scheduler(max_batch=512), ex)
    ex.close()
    log(f"serve: batches={st['batches']} mean={st['mean_batch']:.1f} p50={st['p50_ms']:.3f} ms "
        f"p99={st['p99_ms']:.3f} ms tiles/s={st['tiles_per_s']:.0f}")
    assert st["batches"] > 1 and np.all(np.isfinite(st["latency_s"]))
    served = unpack_masks(ex.masks)
    alone = torch.empty((1, 8192), dtype=torch.uint8, device="cuda")
    for k in range(len(reqs)):
        hv.hv_render_batch(reqs[k:k + 1], alone)
        torch.cuda.synchronize()
        assert np.array_equal(unpack_masks(alone.cpu().numpy())[0], served[k]), k
    for d, objs, kind in ((0, segs, oracle.SEGMENTS), (1, pts, oracle.POINTS)):
        sel = np.nonzero(ds == d)[0][:150]
        tri = oracle.OracleIndex(objs, kind).render(arr["tiles"][sel], arr["r"][sel])["tri"]
        assert parity(served[sel], tri)[0] == 0, d
    hv.hv_free(h2)
    hv.hv_free(h3)


def test_served_with_parse_rules_and_cache_equals_alone(hv, torch):
    """Parse rules, result pool and joined duplicates change only which
    requests make tasks: every served mask still equals the request rendered
    alone."""
    from paper_2005_12489_amd import serve
    segs = hvgen.gen_c2_segments(n_segments=200_000)
    pts = hvgen.gen_c3_points(200_000)
    rng = np.random.default_rng(9)
    small = np.stack([rng.uniform(10.0, 12.0, 2000), rng.uniform(40.0, 42.0, 2000)], 1)
    hs = [build(hv, torch, segs, hv.HV_SEGMENTS), build(hv, torch, pts, hv.HV_POINTS),
          build(hv, torch, small, hv.HV_POINTS)]
    arr = hvgen.c5_arrivals(20000.0, c2_objects=segs, max_requests=3000, zmax=8)
    n = len(arr["t"])
    ds = arr["dataset"].copy()
    ds[::10] = 2                        # a tenth go to the small set: mostly outside its box
    req = {"dataset": ds, "tiles": arr["tiles"], "r": arr["r"]}
    reqs = hv.requests(np.array(hs, dtype=np.uint64)[ds], arr["tiles"], arr["r"])
    parser = serve.RequestParser([hv.hv_index_info(h)["root"] for h in hs])
    cache = serve.ResultCache(cap_bytes=64 << 20, ttl_s=60.0)
    ex = serve.GpuExecutor(reqs, streams=2, max_batch=512, max_indexes=3, max_levels=12, keep_masks=True,
                           return_masks=True)
    log(f"serve with parse rules and cache: {n} requests")
    st = serve.serve(arr["t"], serve.Scheduler(max_batch=512), ex, requests=req, parser=parser, cache=cache)
    ex.close()
    log(f"tasks={st['tasks']} hits={st['cache_hits']} joined={st['joined']} empty={st['empty']} "
        f"p50={st['p50_ms']:.3f} ms p99={st['p99_ms']:.3f} ms")
    assert st["cache_hits"] > 0 and st["empty"] > 0 and st["tasks"] < n
    assert st["tasks"] + st["cache_hits"] + st["joined"] + st["empty"] + st["rejected"] == n
    served = unpack_masks(ex.masks)
    alone = torch.empty((n, 8192), dtype=torch.uint8, device="cuda")
    hv.hv_render_batch(reqs, alone)
    torch.cuda.synchronize()
    ref = unpack_masks(alone.cpu().numpy())
    for k in range(n):
        assert np.array_equal(ref[k], served[k]), (k, int(st["status"][k]))
    # and the oracle, on every request answered without a task of its own
    # (empty tiles, pool hits, joined duplicates) and on a sample of the rest
    status = st["status"]
    keys = [(int(ds[i]), *map(int, arr["tiles"][i]), float(arr["r"][i])) for i in range(n)]
    first = {}
    for i, k in enumerate(keys):
        first.setdefault(k, i)
    repeat = np.array([first[k] != i for i, k in enumerate(keys)])
    pick = np.nonzero((status == serve.EMPTY) | repeat)[0]
    pick = np.concatenate([pick, np.nonzero((status == serve.TASK) & ~repeat)[0][:200]])
    log(f"serve with parse rules and cache: oracle on {len(pick)} served masks "
        f"({int((status == serve.EMPTY).sum())} empty, {int(repeat.sum())} repeats)")
    objs = [(segs, oracle.SEGMENTS), (pts, oracle.POINTS), (small, oracle.POINTS)]
    total_amb = 0
    for d, (o, kind) in enumerate(objs):
        sel = pick[ds[pick] == d]
        if len(sel) == 0:
            continue
        tri = oracle.OracleIndex(o, kind).render(arr["tiles"][sel], arr["r"][sel])["tri"]
        mism, amb, _ = parity(served[sel], tri)
        total_amb += amb
        assert mism == 0, d
    assert total_amb <= 1e-6 * 65536 * len(pick) + 1
    for h in hs:
        hv.hv_free(h)


def test_memory_budget_binds_before_slots(hv, torch):
    """Admission by device memory: the budget admits 48 requests' bytes (the
    library's own count per request) while thousands of slots are free, so
    a burst of 2,500 requests runs at most 48 at a time; every served mask
    still equals the request rendered alone."""
    from paper_2005_12489_amd import serve
    segs = hvgen.gen_c2_segments(n_segments=300_000)
    pts = hvgen.gen_c3_points(300_000)
    h2, h3 = build(hv, torch, segs, hv.HV_SEGMENTS), build(hv, torch, pts, hv.HV_POINTS)
    arr = hvgen.c5_arrivals(50000.0, c2_objects=segs, max_requests=2500, zmax=14)
    reqs = hv.requests(np.where(arr["dataset"] == 0, h2, h3).astype(np.uint64), arr["tiles"], arr["r"])
    per = serve.request_bytes(h2, arr["tiles"][0], 1.0)
    budget = 48 * per
    ex = serve.GpuExecutor(reqs, streams=2, max_batch=512, max_indexes=2, max_levels=12, keep_masks=True,
                           mem_budget=budget)
    assert ex.max_batch == 48
    sch = serve.Scheduler(max_batch=512, max_inflight=16384, mem_budget=budget)
    log(f"serve under a memory budget of {budget} bytes: {len(reqs)} requests arriving at once")
    st = serve.serve(np.zeros(len(reqs)), sch, ex)       # one burst: the queue always holds more than fits
    ex.close()
    log(f"peak in flight {sch.peak_inflight}, peak bytes {sch.peak_mem}, batches {st['batches']}, "
        f"p99 {st['p99_ms']:.3f} ms")
    assert sch.peak_mem <= budget and sch.peak_inflight <= 48 and sch.peak_inflight < sch.max_inflight
    assert sch.peak_inflight == 48, "a burst fills the budget"
    assert sch.inflight == 0 and sch.mem_used == 0
    served = unpack_masks(ex.masks)
    alone = torch.empty((1, 8192), dtype=torch.uint8, device="cuda")
    for k in range(len(reqs)):
        hv.hv_render_batch(reqs[k:k + 1], alone)
        torch.cuda.synchronize()
        assert np.array_equal(unpack_masks(alone.cpu().numpy())[0], served[k]), k
    hv.hv_free(h2)
    hv.hv_free(h3)
