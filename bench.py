"""Tile-mask throughput on one MI355X.  Prints one JSON line.

One step renders every request of the workload in one batched launch: a
HIP graph [copy the staged requests -> tile-frontier kernel -> query kernel]
replayed by hv_batcher, with the index already resident in HBM.

Workloads (--workload):
  c4 (default)  >= 2e8 star-polygon edges; 4,096 mixed requests per launch at
                zooms 2-20, widths 1-5 px, against one launch per tile.
  c1            10,000 uniform points; all 256 tiles of zoom 4; radius 2 px.
  c2            10,000,000 linestring segments (random-walk polylines,
                64-centre mixture); all 4,096 tiles of zoom 6; width 1 px.
  c3            1e9 clustered points; 10,000 density-proportional tiles at
                zooms 0-18, radius 1-3 px.
  c4fill        the c4 polygons filled (Algorithm 2) over the c4 requests.
  c5            serving: the c2 and c3 indexes resident; Poisson arrivals at
                1k-50k requests/s over both, zooms 0-20, mixed styles;
                continuous batching on two streams against one launch per
                request (20,000 requests or 10 s per rate).

Reported beside the batched figure: per-request latency p50/p99 inside a
batch (device completion stamps), the same requests as one plain
hv_render_batch call, and as one launch per request (p50/p99 of each
launch); the index build time; the query kernel against its roofline
(algorithmic bytes and flops per launch from the oracle's work counters,
the bound being whichever takes longer at peak, and HBM traffic from
committed rocprofv3 counters taken in the same launch shape while the query
source is unchanged); and the CPU oracle timed on a bounded sample of the
workload, on all host cores and on one thread.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import hvgen  # noqa: E402

METRIC = "256×256 tiles/sec at 1 GPU + p50/p99 tile latency; batched vs per-tile launch"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
WORK_FILE = os.path.join(ROOT, "tests", "golden", "algorithmic_work.json")
COUNTERS_GLOB = os.path.join(ROOT, "profiles", "counters_query*.json")
QUERY_SOURCE = os.path.join(ROOT, "paper_2005_12489_amd", "csrc", "hv_query.hip")

WORKLOADS = {
    "c1": dict(name="points-10k-z4-all256-r2", kind=0),
    "c2": dict(name="linestrings-10M-z6-all4096-w1", kind=1),
    "c3": dict(name="points-1e9-clustered-10000tiles-z0-18-r1-3", kind=0),
    "c4": dict(name="polygon-edges-2e8-4096mixed-z2-20-w1-5", kind=2),
    "c5": dict(name="serving-linestrings-10M+points-1e9-poisson-1k-50k", kind=-1),
    "c4fill": dict(name="polygon-fill-2e8edges-4096mixed-z2-20", kind=-2),
}
RATES = (1000.0, 2000.0, 5000.0, 10000.0, 20000.0, 50000.0)


_T0 = time.perf_counter()


def stage(msg: str) -> None:
    """Progress line on stderr (long runs must keep writing)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def _gen_progress(done: int, total: int) -> None:
    if done == total or done % 10 == 0:
        stage(f"generated chunk {done}/{total}")


def make_workload(key: str, scale: float = 1.0):
    """(objects, tiles (n,3), r (n,), config dict)."""
    if key == "c1":
        objs = hvgen.gen_c1_points()
        tiles, r = hvgen.c1_requests()
        cfg = {"n_points": int(objs.shape[0]), "zoom": 4, "tiles": int(len(tiles)), "r_px": r}
        return objs, tiles, np.full(len(tiles), r), cfg
    if key == "c2":
        objs = hvgen.gen_c2_segments()
        tiles, r = hvgen.c2_requests()
        cfg = {"n_segments": int(objs.shape[0]), "zoom": 6, "tiles": int(len(tiles)), "r_px": r,
               "line_width_px": 2 * r}
        return objs, tiles, np.full(len(tiles), r), cfg
    if key == "c3":
        n = int(1_000_000_000 * scale)
        objs = hvgen.gen_c3_points(n, progress=_gen_progress)
        tiles, r = hvgen.c3_requests(10_000)
        cfg = {"n_points": n, "zooms": "0-18", "tiles": int(len(tiles)), "r_px": "U[1,3]"}
        return objs, tiles, r, cfg
    if key == "c4":
        objs = hvgen.gen_c4_edges(min_edges=int(200_000_000 * scale))
        tiles, r = hvgen.c4_requests(objs, n=4096)
        cfg = {"n_edges": int(objs.shape[0]), "zooms": "2-20", "requests_per_launch": int(len(tiles)),
               "line_width_px": "U{1..5}"}
        return objs, tiles, r, cfg
    raise KeyError(key)


def query_kernel_name(launch, aa: bool = False) -> str:
    """Name of the query kernel a launch shape runs (as profilers show it);
    aa: the anti-aliased kernel, always in region mode (region 32 when the
    shape names none)."""
    if not launch:
        return f"k_query_region<32, 2, {int(aa)}>"   # the default shape, whatever its waves per workgroup
    L = launch
    region = L.get("region", 0) or (32 if aa else 0)
    if region:
        return f"k_query_region<{region}, {L.get('objs_per_lane', 1) or 1}, {int(aa)}>"
    return f"k_query<{L.get('block', 16) or 16}>"


def fill_kernel_name(launch) -> str:
    """Name of the fill kernel a launch shape runs (filling is region mode
    only; region 32 by default)."""
    return f"k_fill_region<{(launch or {}).get('region', 32) or 32}>"


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def source_hash() -> str:
    return hashlib.sha256(open(QUERY_SOURCE, "rb").read()).hexdigest()


def launch_key(launch) -> dict:
    """A launch shape with every field spelled out (None = the default)."""
    fields = ("block", "cand_cap", "waves_per_wg", "grid_wgs", "region", "objs_per_lane", "cull_nodes")
    return None if launch is None else {k: int(launch.get(k, 0) or 0) for k in fields}


def committed_traffic(workload: str, kernel: str, launch):
    """HBM bytes per launch of the query kernel from committed rocprofv3
    counters (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter
    reads for a plain copy of known size), used only when they were taken on
    this workload, with this kernel, in this exact launch shape and with the
    query source as it is now."""
    import glob
    want = launch_key(launch)
    for path in sorted(glob.glob(COUNTERS_GLOB)):
        c = json.load(open(path))
        for e in c.get("runs", [c]):
            if (e.get("workload") == workload and e.get("kernel") == kernel and e.get("launch") == want
                    and e.get("query_source_sha256") == source_hash()):
                return e["hbm_bytes_per_launch"], os.path.relpath(path, ROOT)
    return None, None


def algorithmic_work(workload: str, zooms=None):
    """Algorithmic bytes and flops of one launch of a workload from the
    oracle's counters (tests/golden/algorithmic_work.json).  A workload too
    large for the oracle to count whole has an entry counted on a per-zoom
    sample and extrapolated per zoom ("<workload>/zooms-A-B-extrapolated");
    its requests at zooms the entry does not cover (`zooms`: the zoom of each
    request) add their output bytes (8192 per mask, or the entry's
    mask_bytes) and nothing else, so the figure is a lower bound, and the
    record says so."""
    if not os.path.exists(WORK_FILE):
        return None
    data = json.load(open(WORK_FILE))
    if workload in data:
        return dict(data[workload])
    keys = [k for k in data if k.startswith(workload + "/zooms-") and data[k].get("extrapolated")]
    if not keys or zooms is None:
        return None
    e = data[keys[0]]
    zs = np.asarray(zooms)
    covered = np.isin(zs, [int(z) for z in e["per_zoom"]])
    assert int(covered.sum()) == e["tiles"], "extrapolated counts do not match this batch's zoom mix"
    rest = int((~covered).sum())
    return {"alg_bytes": e["alg_bytes"] + e.get("mask_bytes", 8192) * rest, "alg_flops": e["alg_flops"],
            "alg_bytes_upper_bound": e.get("alg_bytes_upper_bound", False),
            "extrapolated": f"{keys[0]}: {e['tiles']} requests at zooms {min(map(int, e['per_zoom']))}-"
                            f"{max(map(int, e['per_zoom']))} extrapolated per zoom from the oracle's counts on a "
                            f"sample of them; the {rest} other requests count their mask bytes only (a lower "
                            f"bound, so achieved and frac are lower bounds)"}


def roofline_record(workload: str, launch, frontier_ms: float, query_ms: float, zooms=None, kernel=None):
    """The query kernel against its roofline.  Algorithmic work per launch
    comes from the oracle's counters (algorithmic_work): bytes = masks + the
    objects unlit pixels need, flops = the exact distance tests those pixels
    need plus one witness per lit pixel.  The roofline time is max(bytes /
    8 TB/s, flops / 78.6 TFLOP/s); the larger term names the bound ("hbm" or
    "alu": FP64 vector arithmetic), and the other side is reported beside
    it.  `kernel` names the measured kernel (default: the query kernel of
    the launch shape)."""
    work = algorithmic_work(workload, zooms)
    if not work:
        return None
    kname = kernel or query_kernel_name(launch)
    sec = query_ms * 1e-3
    gbs = work["alg_bytes"] / sec / 1e9
    tfl = work["alg_flops"] / sec / 1e12
    t_bytes = work["alg_bytes"] / (HBM_PEAK_GBS * 1e9)
    t_flops = work["alg_flops"] / (FP64_PEAK_TFLOPS * 1e12)
    traffic, src = committed_traffic(workload, kname, launch)
    rec = {"kernel": kname, "kernel_ms": query_ms, "frontier_kernel_ms": frontier_ms,
           "alg_bytes_per_launch": work["alg_bytes"], "alg_flops_per_launch": work["alg_flops"],
           "roofline_ms": max(t_bytes, t_flops) * 1e3, "traffic": traffic, "traffic_source": src,
           "traffic_gbs": traffic / sec / 1e9 if traffic else None}
    if work.get("extrapolated"):
        rec["alg_extrapolated"] = work["extrapolated"]
    if work.get("alg_bytes_upper_bound"):
        rec["alg_bytes_note"] = "an upper bound: an object needed by two of a tile's four child tiles counts twice"
    if t_flops > t_bytes:
        rec.update({"bound": "alu", "achieved": tfl, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tfl / FP64_PEAK_TFLOPS, "hbm_achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS})
    else:
        rec.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "fp64_tflops": tfl, "fp64_frac": tfl / FP64_PEAK_TFLOPS})
    order = ("bound", "achieved", "peak", "unit", "frac", "traffic")
    return {**{k: rec[k] for k in order}, **{k: v for k, v in rec.items() if k not in order}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _near_first_vertex(objs, tiles, pick):
    """Indices of the objects whose first vertex lies in a zoom-8 cell that a
    picked tile covers, or in one of the cells around it (1.4 degrees).  Own
    projection of the first vertex: this only chooses which objects the
    timing sample's index holds."""
    lon = objs[:, 0]
    lat = np.clip(objs[:, 1], -85.0511287798066, 85.0511287798066)
    cx = np.minimum(((lon + 180.0) / 360.0 * 256).astype(np.int32), 255)
    cy = np.minimum(((0.5 - np.arctanh(np.sin(np.radians(lat))) / (2 * np.pi)) * 256).astype(np.int32), 255)
    need = np.zeros((256, 256), dtype=bool)
    for t in pick:
        z, x, y = (int(v) for v in tiles[t])
        if z >= 8:
            x0 = x1 = x >> (z - 8)
            y0 = y1 = y >> (z - 8)
        else:
            x0, x1 = x << (8 - z), ((x + 1) << (8 - z)) - 1
            y0, y1 = y << (8 - z), ((y + 1) << (8 - z)) - 1
        need[max(0, y0 - 1):min(255, y1 + 1) + 1, max(0, x0 - 1):min(255, x1 + 1) + 1] = True
    return np.nonzero(need[cy, cx])[0]


def cpu_baseline(objs, kind, tiles, r, seconds: float, zmin: int = 0):
    """The oracle (as it stands) timed on a bounded sample of the requests,
    on all host cores and on one thread, index build untimed.

    Sets of up to 5e7 objects: the oracle indexes all of them and renders
    requests drawn at random.  Larger sets: the sample is stratified by zoom,
    the same number of requests at every zoom the workload draws (its zooms
    are uniform, so the sample has the workload's zoom mix), and the oracle
    indexes the objects whose first vertex lies within one zoom-8 cell of a
    sampled tile.  zmin > 0 leaves out the zooms below it (tiles that hold
    too much of a very large set for a host index built inside a bench)."""
    import oracle
    threads = oracle.default_threads()
    rng = np.random.default_rng(12345)
    zs = np.unique(tiles[:, 0])
    zs = zs[zs >= zmin]
    whole = objs.shape[0] <= 50_000_000
    if whole:
        order = rng.permutation(len(tiles))
        note = f"requests drawn at random (seed 12345) from the {len(tiles)}; index over all {objs.shape[0]} objects"
    else:
        per = 5
        order = np.concatenate([rng.permutation(np.nonzero(tiles[:, 0] == z)[0])[:per] for z in zs])
        order = order[rng.permutation(len(order))]
        stage(f"oracle baseline: selecting the objects near {len(order)} sampled requests")
        keep = _near_first_vertex(objs, tiles, order)
        objs = objs[keep]
        mix = "the workload's zoom mix" if zmin <= tiles[:, 0].min() else f"zooms below {zmin} left out"
        note = (f"{per} requests per zoom (zooms {zs.min()}-{zs.max()}, seed 12345; {mix}); "
                f"index over the {objs.shape[0]} objects whose first vertex lies within one zoom-8 cell of them")
    stage(f"oracle baseline: building the oracle index over {objs.shape[0]} objects")
    ix = oracle.OracleIndex(objs, kind)

    def timed(nthreads, budget, chunk):
        done, t0 = 0, time.perf_counter()
        while done < len(order) and time.perf_counter() - t0 < budget:
            sel = order[done:done + chunk]
            ix.render(tiles[sel], r[sel], nthreads=nthreads, want_bit=False)
            done += len(sel)
        return done, time.perf_counter() - t0

    stage(f"oracle baseline: rendering on {threads} threads")
    n_all, t_all = timed(threads, seconds, max(threads, 8) if len(order) > 512 else len(order))
    stage(f"oracle baseline: {n_all} requests in {t_all:.1f} s; one thread")
    per_zoom = {}
    if not whole or len(zs) > 1:
        # one thread, request by request, so that the time per zoom is known
        t1 = 0.0
        n1 = 0
        for t in order:
            c0 = time.perf_counter()
            ix.render(tiles[t:t + 1], r[t:t + 1], nthreads=1, want_bit=False)
            dt = time.perf_counter() - c0
            t1 += dt
            n1 += 1
            z = int(tiles[t, 0])
            e = per_zoom.setdefault(str(z), [0, 0.0])
            e[0] += 1
            e[1] += dt
            if t1 > seconds:
                break
        per_zoom = {z: {"requests": v[0], "ms_per_tile_1thread": v[1] / v[0] * 1e3} for z, v in per_zoom.items()}
    else:
        n1, t1 = timed(1, seconds / 2, 8)
    return {"value": n_all / t_all, "unit": "tiles/s", "cores": threads, "kind": "oracle",
            "value_1thread": n1 / t1, "cpu_model": cpu_model(),
            "sample": f"{n_all} of the {len(order)} sampled requests on {threads} threads ({t_all:.1f} s) and "
                      f"{n1} on one thread ({t1:.1f} s); {note}; index build untimed",
            "per_zoom_1thread": per_zoom or None}


def serve_bench(args, hv, torch):
    """Serving sweep over request rates: continuous batching vs one launch per request."""
    from paper_2005_12489_amd import serve
    segs = hvgen.gen_c2_segments()
    n3 = int(1_000_000_000 * args.scale)
    pts = hvgen.gen_c3_points(n3, progress=_gen_progress)
    hs = []
    for objs, kind in ((segs, hv.HV_SEGMENTS), (pts, hv.HV_POINTS)):
        d = torch.from_numpy(objs).cuda()
        torch.cuda.synchronize()
        hs.append(hv.hv_index_build(d, kind))
        del d
        torch.cuda.empty_cache()
        stage(f"index built over {objs.shape[0]} objects")
    levels = max(hv.hv_index_info(h)["levels"] for h in hs)
    roots = [hv.hv_index_info(h)["root"] for h in hs]
    del pts
    rows = []
    for rate in RATES:
        arr = hvgen.c5_arrivals(rate, c2_objects=segs)
        reqs = hv.requests(np.where(arr["dataset"] == 0, hs[0], hs[1]).astype(np.uint64), arr["tiles"], arr["r"])
        row = {"rate": rate, "requests": len(reqs)}
        keyed = {"dataset": arr["dataset"], "tiles": arr["tiles"], "r": arr["r"]}
        for mode, mb in (("batched", 4096), ("per_request", 1), ("batched_cached", 4096)):
            cached = mode == "batched_cached"
            ex = serve.GpuExecutor(reqs, streams=2, max_batch=mb, max_indexes=2, max_levels=levels,
                                   return_masks=cached)
            warm = np.arange(min(64, len(reqs)))
            serve.serve(np.zeros(len(warm)), serve.Scheduler(max_batch=mb), _Subset(ex, warm))
            extra = {}
            if cached:
                extra = {"requests": keyed, "parser": serve.RequestParser(roots),
                         "cache": serve.ResultCache(cap_bytes=1 << 30, ttl_s=60.0)}
            st = serve.serve(arr["t"], serve.Scheduler(max_batch=mb), ex, **extra)
            ex.close()
            keys = ("tiles_per_s", "p50_ms", "p99_ms", "max_ms", "batches", "mean_batch")
            if cached:
                keys += ("tasks", "cache_hits", "joined", "empty", "rejected")
            row[mode] = {k: st[k] for k in keys}
            stage(f"rate {rate:g}/s {mode}: {st['tiles_per_s']:.0f} tiles/s p99 {st['p99_ms']:.2f} ms")
        print(json.dumps({"serving_rate": rate, **row}), file=sys.stderr, flush=True)
        rows.append(row)
    for h in hs:
        hv.hv_free(h)
    top = rows[-1]
    rec = {
        "metric": METRIC, "value": top["batched"]["tiles_per_s"], "unit": "tiles/s", "n_gpus": 1,
        "steps": len(rows), "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["c5"]["name"], "n_segments": int(segs.shape[0]), "n_points": n3,
                   "rates_per_s": list(RATES), "streams": 2, "max_batch": 4096},
        "serving": rows,
        "note": "value = served tiles/s at the highest offered rate without the result pool; latency = "
                "completion (masks on the host) - scheduled arrival; batched_cached adds the parse rules, "
                "the result pool (1 GiB, 60 s) and joining of duplicate requests",
    }
    print(json.dumps(rec))


def fill_bench(args, hv, torch):
    """Polygon filling (SIBF) of the c4 polygons over the c4 requests."""
    import oracle
    stage("workload c4fill: generating")
    edges = hvgen.gen_c4_edges(min_edges=int(200_000_000 * args.scale))
    first = hvgen.c4_polygon_first(edges)
    tiles, _ = hvgen.c4_requests(edges, n=4096)
    n = len(tiles)
    d = torch.from_numpy(edges).cuda()
    torch.cuda.synchronize()
    h = hv.hv_polygon_index_build(d, first)
    del d
    torch.cuda.empty_cache()
    info = hv.hv_index_info(h)
    stage(f"polygon index: {len(first) - 1} polygons, {edges.shape[0]} edges, {info['build_ms']:.1f} ms")
    launch = json.loads(args.launch) if args.launch else None
    out = torch.empty((n, hv.HV_MASK_BYTES), dtype=torch.uint8, device="cuda")
    t4 = hv.tiles_array(tiles)
    for _ in range(args.warmup):
        hv.hv_render_fill(h, t4, out, launch)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        hv.hv_render_fill(h, t4, out, launch)
        evs[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in evs]
    value = n * args.steps / wall
    stage(f"timed {args.steps} steps: {wall / args.steps * 1e3:.3f} ms/step")
    # the fill kernel alone, HIP events on the stream it runs on
    frontier_ms, fill_ms = hv.hv_time_fill(h, t4, out, launch, reps=max(args.steps, 3))
    roofline = roofline_record(WORKLOADS["c4fill"]["name"], launch, frontier_ms, fill_ms,
                               kernel=fill_kernel_name(launch))
    per_tile = None
    if not args.no_per_tile:
        pe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        torch.cuda.synchronize()
        q0 = time.perf_counter()
        for k in range(n):
            pe[k][0].record()
            hv.hv_render_fill(h, t4[k:k + 1], out[k], launch)
            pe[k][1].record()
        torch.cuda.synchronize()
        lat = [a.elapsed_time(b) for a, b in pe]
        per_tile = {"tiles_per_s": n / (time.perf_counter() - q0), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                    "launches": n}
    cpu = None
    if not args.no_cpu_baseline:
        # the polygons near 64 requests at zoom >= 8 (a host index over all of
        # them is out of reach here)
        order = np.random.default_rng(12345).permutation(n)
        sample = order[tiles[order, 0] >= 8][:64]
        X, Y = oracle.project(edges[first[:-1], 0:2])
        cell = np.minimum((Y * 256).astype(np.int64), 255) * 256 + np.minimum((X * 256).astype(np.int64), 255)
        need = set()
        for t in sample:
            z, x, y = (int(v) for v in tiles[t])
            cx, cy = x >> (z - 8), y >> (z - 8)
            need.update(yy * 256 + xx for yy in range(max(0, cy - 1), min(255, cy + 1) + 1)
                        for xx in range(max(0, cx - 1), min(255, cx + 1) + 1))
        keep = np.nonzero(np.isin(cell, np.fromiter(need, dtype=np.int64)))[0]
        sub_e = np.concatenate([edges[first[p]:first[p + 1]] for p in keep]) if len(keep) else np.zeros((0, 4))
        sub_f = np.concatenate([[0], np.cumsum(first[keep + 1] - first[keep])]).astype(np.int64)
        stage(f"oracle baseline: {len(keep)} polygons near the sampled requests")
        P = oracle.OraclePolygons(sub_e, sub_f)
        th = oracle.default_threads()
        done, c0 = 0, time.perf_counter()
        while done < len(sample) and time.perf_counter() - c0 < args.cpu_seconds:
            P.render(tiles[sample[done:done + th]], nthreads=th)
            done += len(sample[done:done + th])
        dt = time.perf_counter() - c0
        cpu = {"value": done / dt, "unit": "tiles/s", "cores": th, "kind": "oracle",
               "sample": f"{done} requests at zoom >= 8 drawn at random (seed 12345) from the {n}, {dt:.1f} s of "
                         f"CPU work on {th} threads; index over the {len(keep)} polygons whose first vertex lies "
                         "within one zoom-8 cell of them; index build untimed"}
    hv.hv_free(h)
    rec = {
        "metric": METRIC, "value": value, "unit": "tiles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["c4fill"]["name"], "n_edges": int(edges.shape[0]),
                   "n_polygons": int(len(first) - 1), "zooms": "2-20", "requests_per_launch": n, "launch": launch},
        "fill": {"tiles_per_s": value, "step_p50_ms": pct(step_ms, 50), "step_p99_ms": pct(step_ms, 99)},
        "per_tile_launch": per_tile, "build_ms": info["build_ms"], "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


class _Subset:
    """Serves a few requests of an executor once (warm-up)."""

    def __init__(self, ex, ids):
        self.ex, self.ids = ex, ids

    def request_bytes(self, rid):
        return self.ex.request_bytes(int(self.ids[rid]))

    def idle_lane(self):
        return self.ex.idle_lane()

    def launch(self, lane, ids):
        self.ex.launch(lane, self.ids[np.asarray(ids)])

    def poll(self):
        return [(np.searchsorted(self.ids, r[0]), *r[1:]) for r in self.ex.poll()]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--scale", type=float, default=1.0, help="object-count scale for c3 / c4")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-tile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-aa", action="store_true", help="skip the anti-aliased (0-4) output figure")
    ap.add_argument("--launch", default="", help="JSON hv_launch fields, e.g. '{\"region\": 64}'")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes per step (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "how the path would shard is described, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_bytes:
        a = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "steps": args.warmup + args.steps}))
        return

    from paper_2005_12489_amd import hv

    torch.cuda.set_device(0)
    if args.workload == "c5":
        return serve_bench(args, hv, torch)
    if args.workload == "c4fill":
        return fill_bench(args, hv, torch)
    wl = WORKLOADS[args.workload]
    stage(f"workload {args.workload}: generating")
    objs, tiles, rr, cfg = make_workload(args.workload, args.scale)
    n = len(tiles)
    stage(f"{objs.shape[0]} objects, {n} requests")

    d_objs = torch.from_numpy(objs).cuda()
    torch.cuda.synchronize()
    h = hv.hv_index_build(d_objs, wl["kind"])
    info = hv.hv_index_info(h)
    del d_objs
    torch.cuda.empty_cache()
    reqs = hv.requests(h, tiles, rr)
    out = torch.empty((n, hv.HV_MASK_BYTES), dtype=torch.uint8, device="cuda")
    stage(f"index built: {info['levels']} levels, {info['build_ms']:.1f} ms")

    launch = json.loads(args.launch) if args.launch else None
    tuned_ms = None
    if launch is None and not args.no_autotune:
        tune = np.arange(n) if n <= 4096 else np.arange(4096) * n // 4096
        launch, tuned_ms = hv.hv_autotune(reqs[tune], out[:len(tune)])
        stage(f"autotuned: {launch}")

    # batched: one graph launch per step
    batcher = hv.hv_batcher_create(n, max_indexes=1, max_levels=info["levels"], launch=launch)
    for _ in range(args.warmup):
        hv.hv_batcher_run(batcher, reqs, out)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        hv.hv_batcher_run(batcher, reqs, out)
        evs[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = [a.elapsed_time(b) for a, b in evs]
    lat_ms = hv.hv_batcher_latency(batcher, n) / 1e3
    hv.hv_batcher_free(batcher)
    wall = t1 - t0
    value = n * args.steps / wall
    stage(f"timed {args.steps} steps: {wall / args.steps * 1e3:.3f} ms/step")
    # the two kernels of a step, timed apart with HIP events on this stream
    frontier_ms, query_ms = hv.hv_time_kernels(reqs, out, launch, reps=args.steps)
    stage(f"kernels: frontier {frontier_ms:.4f} ms, query {query_ms:.4f} ms")

    # the same requests as one plain (not graph-captured) call
    for _ in range(2):
        hv.hv_render_batch(reqs, out, launch)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for _ in range(5):
        hv.hv_render_batch(reqs, out, launch)
    torch.cuda.synchronize()
    plain = n * 5 / (time.perf_counter() - p0)

    # Algorithm 1's anti-aliased output (one byte per pixel) for the same requests
    aa = None
    if not args.no_aa:
        out_aa = torch.empty((n, hv.HV_AA_BYTES), dtype=torch.uint8, device="cuda")
        hv.hv_render_batch_aa(reqs, out_aa, launch)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for _ in range(5):
            hv.hv_render_batch_aa(reqs, out_aa, launch)
        torch.cuda.synchronize()
        aa_s = (time.perf_counter() - a0) / 5
        aa = {"tiles_per_s": n / aa_s, "ms_per_call": aa_s * 1e3,
              "note": "values 0-4 per pixel: how many of its four sub-samples (centre -+ 1/4 px in x and y) lie "
                      "within r; requests on dense tiles (aa_split) render as their four child tiles at 2r, "
                      "the rest in one pass"}
        # the query kernels alone (child tiles, one pass), HIP events on the
        # stream they run on
        aa_frontier_ms, aa_query_ms = hv.hv_time_aa(reqs, out_aa, launch, reps=5)
        aa["roofline"] = roofline_record(
            wl["name"] + "/aa", launch, aa_frontier_ms, aa_query_ms, zooms=tiles[:, 0],
            kernel=f"{query_kernel_name(launch)} (child tiles) + {query_kernel_name(launch, aa=True)} (one pass)")
        del out_aa
        stage(f"anti-aliased: {n / aa_s:.0f} tiles/s")

    per_tile = None
    if not args.no_per_tile:
        # one launch per tile in the library's shape for a single request
        # (the batch's tuned shape is chosen for thousands of them), unless a
        # shape was given on the command line
        one = json.loads(args.launch) if args.launch else None
        m = min(n, 4096)
        pe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(m)]
        torch.cuda.synchronize()
        q0 = time.perf_counter()
        for k in range(m):
            pe[k][0].record()
            hv.hv_render_batch(reqs[k:k + 1], out[k], one)
            pe[k][1].record()
        torch.cuda.synchronize()
        q1 = time.perf_counter()
        lat = [a.elapsed_time(b) for a, b in pe]
        per_tile = {"tiles_per_s": m / (q1 - q0), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "launches": m}

    roofline = roofline_record(wl["name"], launch, frontier_ms, query_ms, zooms=tiles[:, 0])

    cpu = None
    if not args.no_cpu_baseline:
        stage("oracle baseline")
        cpu = cpu_baseline(objs, wl["kind"], tiles, rr, args.cpu_seconds,
                           zmin=6 if args.workload == "c3" else 0)

    hv.hv_free(h)
    rec = {
        "metric": METRIC, "value": value, "unit": "tiles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], **cfg, "launch": launch,
                   "index": {k: info[k] for k in ("levels", "nodes", "leaf_size", "fanout", "key_bits")}},
        "batched": {"tiles_per_s": value, "p50_ms": pct(lat_ms, 50), "p99_ms": pct(lat_ms, 99),
                    "step_p50_ms": pct(step_ms, 50), "step_p99_ms": pct(step_ms, 99),
                    "note": "one graph launch per step; a request's latency is its completion "
                            "after the batch started on the device"},
        "plain_call_tiles_per_s": plain,
        "anti_aliased": aa,
        "per_tile_launch": per_tile,
        "autotune_ms": tuned_ms,
        "build_ms": info["build_ms"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
