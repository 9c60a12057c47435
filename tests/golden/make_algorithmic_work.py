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

Calls only the oracle and the seeded generators.  Usage:
    python tests/golden/make_algorithmic_work.py [c1] [c2]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import hvgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "algorithmic_work.json")


def workload(key):
    if key == "c1":
        return "points-10k-z4-all256-r2", hvgen.gen_c1_points(), oracle.POINTS, *hvgen.c1_requests()
    if key == "c2":
        return "linestrings-10M-z6-all4096-w1", hvgen.gen_c2_segments(), oracle.SEGMENTS, *hvgen.c2_requests()
    raise KeyError(key)


def main(keys):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for key in keys:
        name, objs, kind, tiles, r = workload(key)
        t0 = time.time()
        ix = oracle.OracleIndex(objs, kind)
        out = ix.render(tiles, r, want_bit=False, want_counters=True)
        c = out["counters"].sum(0)
        s_obj = 16 if kind == oracle.POINTS else 32
        f = 6 if kind == oracle.POINTS else 18
        n_tiles = len(tiles)
        rec = {
            "tiles": n_tiles,
            "r_px": r,
            "objects": int(objs.shape[0]),
            "lit_pixels": int(c[oracle.C_LIT]),
            "ambiguous_pixels": int(c[oracle.C_AMB]),
            "sum_unlit_cand": int(c[oracle.C_UNLIT_CAND]),
            "sum_nbox_unlit": int(c[oracle.C_NBOX_UNLIT]),
            "alg_bytes": int(8192 * n_tiles + s_obj * c[oracle.C_UNLIT_CAND]),
            "alg_flops": int(f * (c[oracle.C_NBOX_UNLIT] + c[oracle.C_LIT])),
            "bytes_per_tile": (8192 * n_tiles + s_obj * float(c[oracle.C_UNLIT_CAND])) / n_tiles,
            "note": "bytes = 8192 per mask + s_obj per object needed to certify an unlit pixel; "
                    "flops = f per (unlit pixel, box-meeting object) pair + one witness test per lit pixel",
        }
        data[name] = rec
        print(name, rec, f"{time.time() - t0:.1f}s", flush=True)
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
