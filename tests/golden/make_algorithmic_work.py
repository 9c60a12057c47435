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
    python tests/golden/make_algorithmic_work.py [c1] [c2] [c4]
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


def main(keys):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
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
