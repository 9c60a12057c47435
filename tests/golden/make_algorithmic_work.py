"""Writes tests/golden/algorithmic_work.json from the CPU oracle's counters.

Algorithmic work of one launch that renders every tile of a workload,
independent of any tree layout (it counts what the display-driven method must
move or compute, not what a particular index happens to touch):
  bytes = sum over tiles of  8192 (the mask) + s_obj * N_unlit_cand(t)
  flops = sum over tiles of  f * (sum over unlit pixels of N_box(p) + N_lit(t))
N_unlit_cand(t): distinct objects whose bounding box meets the (c +- r) box of
some unlit pixel -- each must be read to certify that pixel, nothing else can
exclude it.  N_box(p): objects whose box meets pixel p's (c +- r) box.  A lit
pixel needs one witness test.  s_obj = 16 B (point) / 32 B (segment); f = 6
(point: 2 sub, 2 mul-add, 1 compare) / 18 (segment distance) FP64 operations.

The counters are pinned in tests/oracle_pins.py (closed forms and a numpy
brute force of N_box and N_unlit_cand).  Per-zoom sums are kept beside the
totals.

Calls only the oracle and the seeded generators.  Usage:
    python tests/golden/make_algorithmic_work.py [c1] [c2] [c4] [c3] [c4fill] [c1aa] [c2aa] [c4aa] [c3aa]
(c3: sampled and extrapolated per zoom, see c3_sampled; c4fill: the fill
counters, see c4fill; c<k>aa: anti-aliased output of c<k>, see aa_counts; c3aa sampled as c3).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

import hvgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "algorithmic_work.json")


def workload(key):
    """(name, objects, kind, tiles (n, 3), r (n,))."""
    if key == "c1":
        tiles, r = hvgen.c1_requests()
        return "points-10k-z4-all256-r2", hvgen.gen_c1_points(), oracle.POINTS, tiles, np.full(len(tiles), r)
    if key == "c2":
        tiles, r = hvgen.c2_requests()
        return ("linestrings-10M-z6-all4096-w1", hvgen.gen_c2_segments(), oracle.SEGMENTS, tiles,
                np.full(len(tiles), r))
    if key == "c4":
        edges = hvgen.gen_c4_edges()
        tiles, r = hvgen.c4_requests(edges, n=4096)
        return "polygon-edges-2e8-4096mixed-z2-20-w1-5", edges, oracle.POLYGON_EDGES, tiles, r
    raise KeyError(key)


def c3_sampled(data, aa=False):
    """The 1e9 points cannot be indexed whole on the host.  Their work is
    counted on the zoom-stratified sample of tests/golden/fullsize_c3.npz (27
    requests per zoom at zooms 3-18, each tile against an oracle index over
    the points near it, as make_fullsize_parity.py does) and extrapolated per
    zoom to every request of the 10,000 at those zooms: the mean per sampled
    tile of a zoom times the number of requests at that zoom.  aa: the
    anti-aliased output instead, each sampled request counted over its four
    child tiles at 2r (see aa_counts), whose reach lies inside the parent's
    near points."""
    import make_fullsize_parity as mfp
    from helpers import stratified_sample
    name = "points-1e9-clustered-10000tiles-z0-18-r1-3"
    n = 1_000_000_000
    tiles, r = hvgen.c3_requests(10_000)
    idx = stratified_sample(tiles, mfp.PER_ZOOM, mfp.SEED, zmin=mfp.ZMIN_C3)
    pts = hvgen.gen_c3_points(n)
    cells = np.empty(n, dtype=np.uint16)
    for s in range(0, n, 10_000_000):
        cells[s:s + 10_000_000] = mfp._cell_of(pts[s:s + 10_000_000])
    start = np.zeros(65537, dtype=np.int64)
    start[1:] = np.cumsum(np.bincount(cells, minlength=65536))
    order = np.argsort(cells, kind="stable")
    del cells
    pts = pts[order]
    del order
    cnt = np.zeros((len(idx), 5), dtype=np.int64)
    t0 = time.time()
    for k, t in enumerate(idx):
        z, x, y = (int(v) for v in tiles[t])
        if z >= 8:
            x0 = x1 = x >> (z - 8)
            y0 = y1 = y >> (z - 8)
        else:
            x0, x1 = x << (8 - z), ((x + 1) << (8 - z)) - 1
            y0, y1 = y << (8 - z), ((y + 1) << (8 - z)) - 1
        xa, xb = max(0, x0 - 1), min(255, x1 + 1)
        sub = np.concatenate([pts[start[cy * 256 + xa]:start[cy * 256 + xb + 1]]
                              for cy in range(max(0, y0 - 1), min(255, y1 + 1) + 1)])
        if len(sub):
            if aa:
                kids = np.array([[z + 1, 2 * x + a, 2 * y + b] for b in (0, 1) for a in (0, 1)], dtype=np.int64)
                cnt[k] = oracle.OracleIndex(sub, oracle.POINTS).render(
                    kids, np.full(4, 2.0 * r[t]), want_bit=False, want_counters=True)["counters"].sum(0)
            else:
                cnt[k] = oracle.OracleIndex(sub, oracle.POINTS).render(tiles[t:t + 1], r[t:t + 1], want_bit=False,
                                                                       want_counters=True)["counters"][0]
        if k % 20 == 0:
            print(f"{name}: sampled tile {k + 1}/{len(idx)} z{z}, {time.time() - t0:.0f}s", flush=True)
    zooms, tot_b, tot_f, tot_n = {}, 0.0, 0.0, 0
    mask = 65536 if aa else 8192
    for z in np.unique(tiles[idx, 0]):
        sel = tiles[idx, 0] == z
        n_z = int((tiles[:, 0] == z).sum())
        cz = cnt[sel].mean(0)
        b = mask + 16 * cz[oracle.C_UNLIT_CAND]
        f = 6 * (cz[oracle.C_NBOX_UNLIT] + cz[oracle.C_LIT])
        zooms[str(int(z))] = {"sampled_tiles": int(sel.sum()), "requests": n_z, "bytes_per_tile": float(b),
                              "flops_per_tile": float(f)}
        tot_b += n_z * b
        tot_f += n_z * f
        tot_n += n_z
    key = name + ("/aa" if aa else "") + "/zooms-3-18-extrapolated"
    data[key] = {
        "tiles": tot_n, "objects": n, "alg_bytes": int(round(tot_b)), "alg_flops": int(round(tot_f)),
        "bytes_per_tile": tot_b / tot_n, "per_zoom": zooms, "extrapolated": True, "mask_bytes": mask,
        "note": "counted by the oracle on 27 sampled requests per zoom at zooms 3-18 and extrapolated per zoom to "
                "the requests of the 10,000 at those zooms (zooms 0-2 are not covered); bytes = 8192 per mask + "
                "16 per point needed to certify an unlit pixel; flops = 6 per (unlit pixel, box-meeting point) "
                "pair + one witness test per lit pixel"}
    if aa:
        data[key]["alg_bytes_upper_bound"] = True
        data[key]["note"] = ("anti-aliased output, counted by the oracle over the four child tiles at 2r of 27 "
                             "sampled requests per zoom at zooms 3-18 and extrapolated per zoom to the requests of "
                             "the 10,000 at those zooms (zooms 0-2 are not covered); bytes = 65536 per tile + 16 per "
                             "point needed to certify an unlit sub-sample, summed over the children (an upper "
                             "bound); flops = 6 per (unlit sub-sample, box-meeting point) pair + one witness test "
                             "per lit sub-sample")
    print(key, {k: v for k, v in data[key].items() if k != "per_zoom"}, flush=True)


def c4fill(data):
    """Polygon filling of the 2e8-edge polygons over the same 4,096 requests
    (Algorithm 2).  Per tile, from the oracle's fill counters:
      bytes = 8192 (the mask) + 32 * needed edges (edges of a candidate
              polygon -- its box holds a pixel centre -- that a ray on one of
              its centre rows crosses in y: the crossings that decide some
              pixel's parity);
      flops = 5 per (edge, row) crossing (the crossing's x: two differences,
              a product, a quotient, a sum) + 1 per (pixel, candidate polygon)
              pair (its parity test)."""
    name = "polygon-fill-2e8edges-4096mixed-z2-20"
    t0 = time.time()
    edges = hvgen.gen_c4_edges()
    first = hvgen.c4_polygon_first(edges)
    tiles, _ = hvgen.c4_requests(edges, n=4096)
    n_edges, n_poly = int(edges.shape[0]), int(len(first) - 1)
    print(f"{name}: {n_edges} edges, {n_poly} polygons, generated in {time.time() - t0:.1f}s", flush=True)
    P = oracle.OraclePolygons(edges, first)
    del edges
    print(f"{name}: oracle polygons built, {time.time() - t0:.1f}s", flush=True)
    cnt = P.counters(tiles)
    del P
    zooms = {}
    for z in np.unique(tiles[:, 0]):
        sel = tiles[:, 0] == z
        cz = cnt[sel].sum(0)
        zooms[str(int(z))] = {"tiles": int(sel.sum()), "alg_bytes": int(8192 * sel.sum() + 32 * cz[1]),
                              "alg_flops": int(5 * cz[2] + cz[3]), "candidate_polygons": int(cz[0])}
    c = cnt.sum(0)
    n = len(tiles)
    rec = {"tiles": n, "objects": n_edges, "polygons": n_poly, "candidate_polygons": int(c[0]),
           "needed_edges": int(c[1]), "edge_row_crossings": int(c[2]), "pixel_polygon_pairs": int(c[3]),
           "alg_bytes": int(8192 * n + 32 * c[1]), "alg_flops": int(5 * c[2] + c[3]),
           "bytes_per_tile": (8192 * n + 32 * float(c[1])) / n, "per_zoom": zooms,
           "note": "bytes = 8192 per mask + 32 per edge whose crossing decides some pixel's parity; flops = 5 per "
                   "(edge, row) crossing + 1 per (pixel, candidate polygon) parity test"}
    data[name] = rec
    print(name, {k: v for k, v in rec.items() if k != "per_zoom"}, f"{time.time() - t0:.1f}s", flush=True)


def aa_counts(data, key):
    """Anti-aliased output of a workload's requests (Algorithm 1's 0-4 per
    pixel).  A pixel's four sub-samples (centre -+ 1/4 px) are the pixel
    centres of its four children one zoom deeper, and r px at zoom z is 2r px
    there, so the oracle's counters of the child tiles at 2r count the
    sub-samples' work:
      bytes = 65536 per tile (one byte per pixel) + s_obj * N_unlit_cand
              summed over the four children (an object needed by two children
              counts twice: an upper bound);
      flops = f per (unlit sub-sample, box-meeting object) pair + one witness
              test per lit sub-sample, summed over the children (exact);
    with s_obj and f as for the binary masks (16 B and 6 for points, 32 B and
    18 for segments and edges)."""
    t0 = time.time()
    name, objs, kind, tiles, r = workload(key)
    n = len(tiles)
    kids = np.empty((4 * n, 3), dtype=np.int64)
    for k, (a, b) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
        kids[k::4] = np.stack([tiles[:, 0] + 1, 2 * tiles[:, 1] + a, 2 * tiles[:, 2] + b], 1)
    rk = np.repeat(2.0 * np.asarray(r, dtype=np.float64), 4)
    ix = oracle.OracleIndex(objs, kind)
    n_obj = int(ix.n)
    del objs
    print(f"{name}/aa: oracle index built, {time.time() - t0:.1f}s", flush=True)
    s_obj = 16 if kind == oracle.POINTS else 32
    f = 6 if kind == oracle.POINTS else 18
    cnt = np.zeros((4 * n, 5), dtype=np.int64)
    for s in range(0, 4 * n, 256):
        cnt[s:s + 256] = ix.render(kids[s:s + 256], rk[s:s + 256], want_bit=False, want_counters=True)["counters"]
        print(f"{name}/aa: child tiles {min(s + 256, 4 * n)}/{4 * n}, {time.time() - t0:.1f}s", flush=True)
    per = cnt.reshape(n, 4, 5).sum(1)
    zooms = {}
    for z in np.unique(tiles[:, 0]):
        sel = tiles[:, 0] == z
        cz = per[sel].sum(0)
        zooms[str(int(z))] = {"tiles": int(sel.sum()),
                              "alg_bytes": int(65536 * sel.sum() + s_obj * cz[oracle.C_UNLIT_CAND]),
                              "alg_flops": int(f * (cz[oracle.C_NBOX_UNLIT] + cz[oracle.C_LIT]))}
    c = per.sum(0)
    data[name + "/aa"] = {
        "tiles": n, "objects": n_obj, "lit_subsamples": int(c[oracle.C_LIT]),
        "ambiguous_subsamples": int(c[oracle.C_AMB]),
        "alg_bytes": int(65536 * n + s_obj * c[oracle.C_UNLIT_CAND]),
        "alg_flops": int(f * (c[oracle.C_NBOX_UNLIT] + c[oracle.C_LIT])),
        "alg_bytes_upper_bound": True, "per_zoom": zooms,
        "note": f"sub-samples = pixel centres of the four children one zoom deeper at 2r: bytes = 65536 per tile + "
                f"{s_obj} per object needed to certify an unlit sub-sample, summed over the children (an upper "
                f"bound); flops = {f} per (unlit sub-sample, box-meeting object) pair + one witness test per lit "
                f"sub-sample"}
    print(name + "/aa", {k: v for k, v in data[name + "/aa"].items() if k != "per_zoom"},
          f"{time.time() - t0:.1f}s", flush=True)


def main(keys):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for key in ("c3", "c3aa"):
        if key in keys:
            keys = [k for k in keys if k != key]
            c3_sampled(data, aa=key == "c3aa")
            with open(OUT, "w") as fh:
                json.dump(data, fh, indent=1, sort_keys=True)
    for key in [k for k in keys if k.endswith("aa")]:
        keys = [k for k in keys if k != key]
        aa_counts(data, key[:-2])
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    if "c4fill" in keys:
        keys = [k for k in keys if k != "c4fill"]
        c4fill(data)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    for key in keys:
        t0 = time.time()
        name, objs, kind, tiles, r = workload(key)
        print(f"{name}: {objs.shape[0]} objects, {len(tiles)} tiles, generated in {time.time() - t0:.1f}s",
              flush=True)
        ix = oracle.OracleIndex(objs, kind)
        del objs
        print(f"{name}: oracle index built, {time.time() - t0:.1f}s", flush=True)
        cnt = np.zeros((len(tiles), 5), dtype=np.int64)
        step = 64
        for s in range(0, len(tiles), step):
            out = ix.render(tiles[s:s + step], r[s:s + step], want_bit=False, want_counters=True)
            cnt[s:s + step] = out["counters"]
            print(f"{name}: tiles {s + len(out['counters'])}/{len(tiles)}, {time.time() - t0:.1f}s", flush=True)
        c = cnt.sum(0)
        s_obj = 16 if kind == oracle.POINTS else 32
        f = 6 if kind == oracle.POINTS else 18
        n_tiles = len(tiles)
        zooms = {}
        for z in np.unique(tiles[:, 0]):
            sel = tiles[:, 0] == z
            cz = cnt[sel].sum(0)
            zooms[str(int(z))] = {
                "tiles": int(sel.sum()),
                "alg_bytes": int(8192 * sel.sum() + s_obj * cz[oracle.C_UNLIT_CAND]),
                "alg_flops": int(f * (cz[oracle.C_NBOX_UNLIT] + cz[oracle.C_LIT])),
                "ambiguous_pixels": int(cz[oracle.C_AMB]),
            }
        rv = np.unique(r)
        rec = {
            "tiles": n_tiles,
            "r_px": float(rv[0]) if len(rv) == 1 else "per request",
            "objects": int(ix.n),
            "lit_pixels": int(c[oracle.C_LIT]),
            "ambiguous_pixels": int(c[oracle.C_AMB]),
            "sum_unlit_cand": int(c[oracle.C_UNLIT_CAND]),
            "sum_nbox_unlit": int(c[oracle.C_NBOX_UNLIT]),
            "alg_bytes": int(8192 * n_tiles + s_obj * c[oracle.C_UNLIT_CAND]),
            "alg_flops": int(f * (c[oracle.C_NBOX_UNLIT] + c[oracle.C_LIT])),
            "bytes_per_tile": (8192 * n_tiles + s_obj * float(c[oracle.C_UNLIT_CAND])) / n_tiles,
            "per_zoom": zooms,
            "note": "bytes = 8192 per mask + s_obj per object needed to certify an unlit pixel; "
                    "flops = f per (unlit pixel, box-meeting object) pair + one witness test per lit pixel",
        }
        data[name] = rec
        print(name, {k: v for k, v in rec.items() if k != "per_zoom"}, f"{time.time() - t0:.1f}s", flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        del ix


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
