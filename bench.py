"""Tile-mask throughput on one MI355X.

One step renders every tile of the workload (one launch through
hv_render_tiles, the index resident in HBM).  Prints one JSON line.

Default workload: 10,000,000 linestring segments (random-walk polylines,
64-centre mixture), all 4,096 tiles of zoom 6, line width 1 px (r = 0.5).
Also reported: the same tiles rendered with one launch per tile (p50/p99
per-tile latency), the index build time, the query kernel against the HBM
roofline (algorithmic bytes per launch from the oracle's work counters), and
the CPU oracle timed on a bounded sample of the same tiles.
"""
from __future__ import annotations

import argparse
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

WORKLOADS = {
    "c2": dict(name="linestrings-10M-z6-all4096-w1", kind=1),
    "c1": dict(name="points-10k-z4-all256-r2", kind=0),
}


def make_workload(key: str):
    if key == "c2":
        objs = hvgen.gen_c2_segments()
        tiles, r = hvgen.c2_requests()
        cfg = {"n_segments": int(objs.shape[0]), "zoom": 6, "tiles": int(len(tiles)), "r_px": r,
               "line_width_px": 2 * r}
    else:
        objs = hvgen.gen_c1_points()
        tiles, r = hvgen.c1_requests()
        cfg = {"n_points": int(objs.shape[0]), "zoom": 4, "tiles": int(len(tiles)), "r_px": r}
    return objs, tiles, r, cfg


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def cpu_baseline(objs, kind, tiles, r, seconds: float):
    """The oracle (as it stands) on a bounded random sample of the same tiles."""
    import oracle
    ix = oracle.OracleIndex(objs, kind)
    threads = oracle.default_threads()
    order = np.random.default_rng(12345).permutation(len(tiles))
    done, t0 = 0, time.perf_counter()
    chunk = max(threads, 8)
    while done < len(tiles) and time.perf_counter() - t0 < seconds:
        sel = order[done:done + chunk]
        ix.render(tiles[sel], r, nthreads=threads, want_bit=False)
        done += len(sel)
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "tiles/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} tiles drawn at random (seed 12345) from the {len(tiles)} tiles, "
                      f"{dt:.1f} s of CPU work on {threads} threads; index build untimed"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-tile", action="store_true")
    ap.add_argument("--launch", default="", help="JSON hv_launch fields, e.g. '{\"block\": 8}'")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes per step (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_bytes:
        import torch
        a = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "steps": args.warmup + args.steps}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the multi-GPU design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_12489_amd import hv

    torch.cuda.set_device(0)
    wl = WORKLOADS[args.workload]
    objs, tiles, r, cfg = make_workload(args.workload)
    tiles4 = hv.tiles_array(tiles)
    n_tiles = len(tiles4)
    launch = json.loads(args.launch) if args.launch else None

    d_objs = torch.from_numpy(objs).cuda()
    torch.cuda.synchronize()
    h = hv.hv_index_build(d_objs, wl["kind"])
    info = hv.hv_index_info(h)
    del d_objs
    out = torch.empty((n_tiles, hv.HV_MASK_BYTES), dtype=torch.uint8, device="cuda")

    def step():
        if launch:
            hv.hv_render_tiles_ex(h, tiles4, r, out, launch)
        else:
            hv.hv_render_tiles(h, tiles4, r, out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        step()
        evs[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = [a.elapsed_time(b) for a, b in evs]
    wall = t1 - t0
    value = n_tiles * args.steps / wall
    kernel_ms = float(np.mean(step_ms))

    per_tile = None
    if not args.no_per_tile:
        pe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_tiles)]
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for k in range(n_tiles):
            pe[k][0].record()
            if launch:
                hv.hv_render_tiles_ex(h, tiles4[k:k + 1], r, out[k], launch)
            else:
                hv.hv_render_tiles(h, tiles4[k:k + 1], r, out[k])
            pe[k][1].record()
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        lat = [a.elapsed_time(b) for a, b in pe]
        per_tile = {"tiles_per_s": n_tiles / (p1 - p0), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                    "launches": n_tiles}

    roofline = None
    work = json.load(open(WORK_FILE)).get(wl["name"]) if os.path.exists(WORK_FILE) else None
    if work:
        bytes_launch = work["alg_bytes"]
        achieved = bytes_launch / (kernel_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "alg_bytes_per_launch": bytes_launch,
                    "fp64_tflops": work["alg_flops"] / (kernel_ms * 1e-3) / 1e12,
                    "fp64_frac": work["alg_flops"] / (kernel_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                    "kernel_ms": kernel_ms}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(objs, wl["kind"], tiles4[:, :3], r, args.cpu_seconds)

    hv.hv_free(h)
    rec = {
        "metric": METRIC, "value": value, "unit": "tiles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl["name"], **cfg, "launch": launch or "default",
                   "index": {k: info[k] for k in ("levels", "nodes", "leaf_size", "fanout", "key_bits")}},
        "batched": {"tiles_per_s": value, "p50_ms": pct(step_ms, 50), "p99_ms": pct(step_ms, 99),
                    "note": "one launch renders every tile; a tile's latency is the launch's"},
        "per_tile_launch": per_tile,
        "build_ms": info["build_ms"],
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
