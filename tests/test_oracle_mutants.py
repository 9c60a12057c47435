"""Plants plausible mistakes in a copy of the oracle (on the CPU) and checks
that at least one pin fails for each.  The oracle's own source is untouched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hv_oracle.c")
RUNNER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_mutant_runner.py")

# (name, text in the oracle, planted replacement)
MUTANTS = [
    ("corner-sample", "const double px = i + 0.5, py = j + 0.5;", "const double px = i, py = j;"),
    ("rows-south-first", "size_t p = (size_t)j * 256 + (size_t)i;",
     "size_t p = (size_t)(255 - j) * 256 + (size_t)i;"),
    ("transposed", "size_t p = (size_t)j * 256 + (size_t)i;", "size_t p = (size_t)i * 256 + (size_t)j;"),
    ("y-sign", "*Y = 0.5 - log(", "*Y = 0.5 + log("),
    ("no-lat-clamp", "if (lat > OR_MAX_LAT) lat = OR_MAX_LAT;", ""),
    ("deg-to-rad", "double phi = lat * (OR_PI / 180.0);", "double phi = lat * (OR_PI / 360.0);"),
    ("x-scale", "*X = (lon + 180.0) / 360.0;", "*X = (lon + 180.0) / 380.0;"),
    ("no-end-clamp", "if (t > 1.0) t = 1.0;", ""),
    ("strict-compare", "int b = D <= r;", "int b = D < r;"),
    ("node-box-max-x", "if (c->x1 > b.x1) b.x1 = c->x1;", ""),
    ("query-box-half-r", "const double h = r + OR_QUERY_PAD;", "const double h = 0.5 * r + OR_QUERY_PAD;"),
    ("no-tile-offset", "const double ox = 256.0 * (double)tx,", "const double ox = 0.0 * (double)tx,"),
    ("zoom-off-by-one", "const double S = 256.0 * ldexp(1.0, z);", "const double S = 256.0 * ldexp(1.0, z + 1);"),
    ("point-d-squared", "return sqrt(ex * ex + ey * ey);\n    }\n    double bx",
     "return ex * ex + ey * ey;\n    }\n    double bx"),
    ("proj-sign", "t = ((px - ax) * dx + (py - ay) * dy) / len2;", "t = ((px - ax) * dx - (py - ay) * dy) / len2;"),
    ("band-label", "(D > r + OR_BAND ? 0 : 2)", "(D > r ? 0 : 2)"),
    ("early-exit", "if (D < r - OR_BAND) { certain = 1; break; }", "if (D < r + 1.0) { certain = 1; break; }"),
    ("str-child-ids", "ix->child[*n_child + k] = e[s + k].id;", "ix->child[*n_child + k] = e[s].id;"),
    ("edges-as-points", "if (ix->kind == OR_POINTS) {\n        double ex", "if (ix->kind != OR_SEGMENTS) {\n        double ex"),
    ("segment-b-is-a", "ix->bx[q] = (w == 4) ? o[2] : o[0];", "ix->bx[q] = o[0];"),
    ("box-meets-axis", "b->y0 <= a->y1;", "b->y0 <= a->x1;"),
    ("aa-sub-offset", "sx[4] = { -0.25, 0.25, -0.25, 0.25 }", "sx[4] = { -0.5, 0.5, -0.5, 0.5 }"),
    ("aa-strict", "v += D <= r;", "v += D < r;"),
    ("aa-r1-sign", "const double R1 = r - q4,", "const double R1 = r + q4,"),
    ("aa-inner-box", "h = sqrt(2.0) / 2.0 * R1;", "h = sqrt(2.0) * R1;"),
    ("aa-not-nearest", "if (d < D || (d == D && k < best)) {", "if (best < 0 || k < best) {"),
    ("aa-transposed", "const size_t p = (size_t)(256 * j + i);", "const size_t p = (size_t)(256 * i + j);"),
    ("fill-closed-rule", "if ((ay > cy) != (by > cy)) {\n                            double ax",
     "if ((ay >= cy) != (by > cy)) {\n                            double ax"),
    ("fill-ray-side", "if (x > cx) par ^= 1;", "if (x > cx - 1.0) par ^= 1;"),
    ("fill-first-polygon-only", "for (int32_t c = 0; c < M->count[nd] && !inside_sure; ++c) {",
     "for (int32_t c = 0; c < M->count[nd] && c < 1; ++c) {"),
    ("fill-box-min-y", "y0 = fmin(y0, fmin(P->ay[q], P->by[q]));", "y0 = fmin(y0, fmax(P->ay[q], P->by[q]));"),
    # work counters (the roofline's algorithmic bytes and flops)
    ("cnt-widened-box", "if (box_meets(&b, &qr)) {", "if (box_meets(&b, &q)) {"),
    ("cnt-duplicates", "uniq += sc->tile_ids[q] != sc->tile_ids[q - 1];", "uniq += 1;"),
    ("cnt-lit-pixels-too", "if (!b && npix > 0) {", "if (npix > 0) {"),
    ("cnt-lit-certain-only", "lit += b;", "lit += (t == 1);"),
    ("cnt-box-half-height", "obox qr = { (cx - r) / S, (cy - r) / S, (cx + r) / S, (cy + r) / S };",
     "obox qr = { (cx - r) / S, (cy - r) / S, (cx + r) / S, cy / S };"),
    ("cnt-unlit-ambiguous-only", "if (!b && npix > 0) {", "if (t == 0 && npix > 0) {"),
    # fill work counters (the fill roofline's algorithmic bytes and flops)
    ("fillcnt-other-half-open", "const double rj0 = fmax(ceil(lo - 0.5), fj0), rj1 = fmin(ceil(hi - 0.5) - 1.0, fj1);",
     "const double rj0 = fmax(floor(lo - 0.5) + 1.0, fj0), rj1 = fmin(floor(hi - 0.5), fj1);"),
    ("fillcnt-no-tile-clip", "fj1 = fmin(floor(by1 - 0.5), 255.0);", "fj1 = floor(by1 - 0.5);"),
    ("fillcnt-px-rows-only", "px += (int64_t)(fi1 - fi0 + 1.0) * (int64_t)(fj1 - fj0 + 1.0);",
     "px += (int64_t)(fj1 - fj0 + 1.0);"),
    ("fillcnt-need-per-row", "++need;\n                pairs +=", "need += (int64_t)(rj1 - rj0 + 1.0);\n                pairs +="),
    ("fillcnt-box-corner", "const double fi0 = fmax(ceil(bx0 - 0.5), 0.0)", "const double fi0 = fmax(ceil(bx0), 0.0)"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique/found: {name}"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    lib = ob.build(str(mut), str(tmp_path / "libmut.so"))
    family = name.split("-")[0] + "_" if name.startswith(("aa-", "fill-", "cnt-", "fillcnt-")) else ""
    res = subprocess.run([sys.executable, RUNNER, lib, family], capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"planted mistake {name!r} was not caught:\n{res.stdout}{res.stderr}"
