"""Pins for the CPU oracle: each checks it against something other than itself.

Every pin takes ``lib_path`` (None = the built oracle) so that the mutation
test can run the same pins against copies of the oracle with planted
mistakes.  A pin raises AssertionError when the oracle disagrees.

Kinds of pins used (paper sections in brackets):
  closed forms   -- projection constants, lattice-disk counts, segment
                    special cases [Sec. 3.2.1, Algorithm 1]
  brute force    -- every object against every pixel, numpy [definition]
  library        -- scipy cKDTree nearest-neighbour distance [points]
  invariants     -- union, permutation, monotone in r, own pixel,
                    parent-empty => child-empty, tile translation
  anti-aliasing  -- sub-sample lattice counts, exact ties, a two-point case
                    where Algorithm 1's printed step undercounts, brute force
                    over sub-samples, one zoom deeper at twice the radius
"""
from __future__ import annotations

import math
import os

import numpy as np

import oracle
from brute import brute_distance, brute_fill, near_band_edge, objects_merc01, tri_state

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ix(objs, kind, merc01=True, lib_path=None):
    return oracle.OracleIndex(np.asarray(objs, dtype=np.float64), kind, merc01=merc01,
                              lib_path=lib_path)


def _px_to_merc(z, x, y, u, v):
    """Tile-local pixel coordinates -> normalised Mercator (exact for dyadic u, v)."""
    S = 256.0 * 2.0 ** z
    return ((256.0 * x + np.asarray(u, dtype=np.float64)) / S,
            (256.0 * y + np.asarray(v, dtype=np.float64)) / S)


def _seg(z, x, y, u0, v0, u1, v1):
    a = _px_to_merc(z, x, y, u0, v0)
    b = _px_to_merc(z, x, y, u1, v1)
    return np.array([[a[0], a[1], b[0], b[1]]])


def _counts(out, t=0):
    tri = out["tri"][t]
    return int(out["bit"][t].sum()), int((tri == 1).sum()), int((tri == 2).sum())


# ------------------------------------------------------------ projection
def pin_projection(lib_path=None):
    # X is exact for dyadic longitudes -180 + 360 k / 2^m.
    lons, want = [], []
    for m in range(0, 21, 4):
        for k in (0, 1, (1 << m) // 3, (1 << m) - 1):
            lons.append(-180.0 + 360.0 * k / 2.0 ** m)
            want.append(k / 2.0 ** m)
    X, _ = oracle.project(np.stack([lons, np.zeros(len(lons))], 1), lib_path)
    assert np.array_equal(X, np.array(want)), "X not exact at dyadic longitudes"
    lat_max = 85.0511287798066
    lat_q = math.degrees(math.atan(math.sinh(math.pi / 2)))   # Y = 1/4 (z=2 row edge)
    lats = np.array([0.0, lat_max, -lat_max, 89.0, -90.0, lat_q, -lat_q])
    _, Y = oracle.project(np.stack([np.zeros(lats.size), lats], 1), lib_path)
    assert abs(Y[0] - 0.5) <= 2e-16, Y[0]
    assert abs(Y[1]) <= 1e-12 and abs(Y[2] - 1.0) <= 1e-12, (Y[1], Y[2])
    assert Y[3] == Y[1] and Y[4] == Y[2], "latitude not clamped to the Mercator limit"
    assert abs(Y[5] - 0.25) <= 1e-14 and abs(Y[6] - 0.75) <= 1e-14, (Y[5], Y[6])
    grid = np.linspace(-85.0, 85.0, 17001)
    _, Yg = oracle.project(np.stack([np.zeros(grid.size), grid], 1), lib_path)
    assert np.all(np.diff(Yg) < 0), "Y must decrease strictly with latitude (y = 0 north)"
    alt = 0.5 - np.arctanh(np.sin(np.radians(grid))) / (2 * math.pi)
    assert np.max(np.abs(Yg - alt)) <= 2e-15, np.max(np.abs(Yg - alt))


# ------------------------------------------------------------ addressing
def pin_addressing(lib_path=None):
    # Tile (0,0,0): pixel (i, j) centre is ((i+1/2)/256, (j+1/2)/256); row j = north-first.
    i, j = 3, 200
    ix = _ix([[(i + 0.5) / 256, (j + 0.5) / 256]], oracle.POINTS, lib_path=lib_path)
    out = ix.render([[0, 0, 0]], 0.1)
    lit = np.argwhere(out["bit"][0])
    assert lit.tolist() == [[j, i]], lit.tolist()
    # A northern-hemisphere point east of Greenwich is in tile (1,1,0).
    ix = _ix([[10.0, 60.0], [-10.0, -60.0]], oracle.POINTS, merc01=False, lib_path=lib_path)
    t = np.array([[1, 0, 0], [1, 1, 0], [1, 0, 1], [1, 1, 1]])
    out = ix.render(t, 0.75)
    n = out["bit"].reshape(4, -1).sum(1)
    assert n[1] > 0 and n[2] > 0 and n[0] == 0 and n[3] == 0, n.tolist()
    # Own pixel at random zooms (r >= sqrt(2)/2 covers the whole pixel).
    rng = np.random.default_rng(11)
    for _ in range(6):
        z = int(rng.integers(0, 18))
        X, Y = rng.uniform(0.01, 0.99, 2)
        S = 256.0 * 2.0 ** z
        gx, gy = int(X * S), int(Y * S)
        tx, ty = gx // 256, gy // 256
        ix = _ix([[X, Y]], oracle.POINTS, lib_path=lib_path)
        out = ix.render([[z, tx, ty]], 0.75)
        assert out["bit"][0][gy - 256 * ty, gx - 256 * tx] == 1, (z, X, Y)


# ------------------------------------------------------------ lattice disks
def _lattice_rows():
    rows = []
    with open(os.path.join(GOLDEN, "lattice_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                pos, r, b, l, a = line.split()
                rows.append((pos, float(r), int(b), int(l), int(a)))
    return rows


def pin_lattice(lib_path=None):
    z, x, y = 10, 300, 400
    for pos, r, nb, nl, na in _lattice_rows():
        off = 0.5 if pos == "centre" else 0.0
        for (pu, pv) in ((100 + off, 50 + off), (off, 50 + off)):   # interior, west seam
            X, Y = _px_to_merc(z, x, y, pu, pv)
            ix = _ix([[X, Y]], oracle.POINTS, lib_path=lib_path)
            out = ix.render([[z, x, y], [z, x - 1, y]], r)
            got = tuple(a + b for a, b in zip(_counts(out, 0), _counts(out, 1)))
            assert got == (nb, nl, na), (pos, r, pu, got, (nb, nl, na))
    # Band edges: a point at distance r + delta east of pixel (100, 50)'s centre,
    # delta an exact dyadic offset; |delta| <= 1e-6 px is ambiguous, beyond is certain.
    r = 2.0
    for delta, tri_want, bit_want in ((2.0 ** -21, 2, 0), (-2.0 ** -21, 2, 1),
                                      (2.0 ** -19, 0, 0), (-2.0 ** -19, 1, 1)):
        X, Y = _px_to_merc(z, x, y, 100.5 + r + delta, 50.5)
        out = _ix([[X, Y]], oracle.POINTS, lib_path=lib_path).render([[z, x, y]], r)
        got = (int(out["tri"][0][50, 100]), int(out["bit"][0][50, 100]))
        assert got == (tri_want, bit_want), (delta, got)


# ------------------------------------------------------------ segments
def pin_segments(lib_path=None):
    z, x, y = 12, 1000, 2000
    a, b, j = 20, 60, 77
    L = b - a + 1
    horiz = _seg(z, x, y, a + 0.5, j + 0.5, b + 0.5, j + 0.5)
    vert = _seg(z, x, y, j + 0.5, a + 0.5, j + 0.5, b + 0.5)
    for s in (horiz, vert):
        ix = _ix(s, oracle.SEGMENTS, lib_path=lib_path)
        out = ix.render([[z, x, y]], 0.5)
        assert _counts(out) == (L, L, 0), _counts(out)
        out = ix.render([[z, x, y]], 1.0)
        assert _counts(out) == (3 * L + 2, L, 2 * L + 2), _counts(out)
    # A segment on the boundary between rows j-1 and j: both rows at exactly 0.5.
    ix = _ix(_seg(z, x, y, a + 0.5, j, b + 0.5, j), oracle.SEGMENTS, lib_path=lib_path)
    out = ix.render([[z, x, y]], 0.5)
    assert _counts(out) == (2 * L, 0, 2 * L), _counts(out)
    # Diagonal through 21 centres; side neighbours at sqrt(2)/2.
    ix = _ix(_seg(z, x, y, 10.5, 10.5, 30.5, 30.5), oracle.SEGMENTS, lib_path=lib_path)
    out = ix.render([[z, x, y]], 0.5)
    assert _counts(out) == (21, 21, 0), _counts(out)
    out = ix.render([[z, x, y]], math.sqrt(2) / 2)
    assert _counts(out)[1:] == (21, 40), _counts(out)
    # End caps: distance is to the closed segment, not to its line.
    ix = _ix(horiz, oracle.SEGMENTS, lib_path=lib_path)
    out = ix.render([[z, x, y]], 2.0)
    tri = out["tri"][0]
    assert tri[j, b + 3] == 0 and tri[j, b + 2] == 2 and tri[j + 1, b + 1] == 1
    assert tri[j, a - 3] == 0 and tri[j, a - 2] == 2 and tri[j - 1, a - 1] == 1
    # Zero-length segment == point; segment mask contains its endpoints' masks.
    rng = np.random.default_rng(5)
    for r in (0.5, 1.3, 2.5):
        u = rng.uniform(5, 250, (8, 2))
        pts = np.stack(_px_to_merc(z, x, y, u[:, 0], u[:, 1]), 1)
        o_pt = _ix(pts, oracle.POINTS, lib_path=lib_path).render([[z, x, y]], r)
        o_sg = _ix(np.concatenate([pts, pts], 1), oracle.SEGMENTS,
                   lib_path=lib_path).render([[z, x, y]], r)
        assert np.array_equal(o_pt["tri"], o_sg["tri"]), r
        s = np.concatenate([pts[:4], pts[4:]], 1)
        o_s = _ix(s, oracle.SEGMENTS, lib_path=lib_path).render([[z, x, y]], r)
        assert np.all(o_s["bit"] >= o_pt["bit"]), r


# ------------------------------------------------------------ kinds
def pin_kinds(lib_path=None):
    rng = np.random.default_rng(7)
    z, x, y = 9, 100, 150
    k = 40
    ang = np.sort(rng.uniform(0, 2 * math.pi, k))
    rad = rng.uniform(30, 90, k)
    u = 128 + rad * np.cos(ang)
    v = 128 + rad * np.sin(ang)
    P = np.stack(_px_to_merc(z, x, y, u, v), 1)
    ring = np.concatenate([P, np.roll(P, -1, axis=0)], 1)      # k edges, closing included
    for r in (0.5, 1.5):
        a = _ix(ring, oracle.SEGMENTS, lib_path=lib_path).render([[z, x, y]], r)
        b = _ix(ring, oracle.POLYGON_EDGES, lib_path=lib_path).render([[z, x, y]], r)
        assert np.array_equal(a["tri"], b["tri"]) and np.array_equal(a["bit"], b["bit"])
        pts = _ix(P, oracle.POINTS, lib_path=lib_path).render([[z, x, y]], r)
        assert np.all(b["bit"] >= pts["bit"]) and b["bit"].sum() > pts["bit"].sum()


# ------------------------------------------------------------ brute force
def _random_objects(rng, kind, z, x, y, n, spread=10.0):
    """Objects within the tile +- spread px (many straddle the seams)."""
    u0 = rng.uniform(-spread, 256 + spread, (n, 2))
    if kind == oracle.POINTS:
        X, Y = _px_to_merc(z, x, y, u0[:, 0], u0[:, 1])
        return np.stack([X, Y], 1)
    d = rng.normal(0, 6.0, (n, 2)) * rng.choice([0.1, 1.0, 5.0], (n, 1))
    u1 = u0 + d
    if n >= 4:
        u1[0] = u0[0]                                        # a zero-length segment
    A = np.stack(_px_to_merc(z, x, y, u0[:, 0], u0[:, 1]), 1)
    B = np.stack(_px_to_merc(z, x, y, u1[:, 0], u1[:, 1]), 1)
    return np.concatenate([A, B], 1)


def _check_against_brute(out, t, objs, kind, tile, r):
    D = brute_distance(objs, kind if kind == 0 else 1, *tile)
    want = tri_state(D, r)
    ok = (out["tri"][t] == want) | near_band_edge(D, r)
    assert ok.all(), (tile, r, int((~ok).sum()))
    bit = D <= r
    okb = (out["bit"][t].astype(bool) == bit) | near_band_edge(D, r)
    assert okb.all(), (tile, r, int((~okb).sum()))
    if "dist" in out:
        sel = (out["tri"][t] != 1) & (D <= r + 1e-5 - 1e-9)
        assert np.allclose(out["dist"][t][sel], D[sel], rtol=0, atol=1e-9)


def pin_brute(lib_path=None, n_obj=160, seed=13):
    rng = np.random.default_rng(seed)
    for kind in (oracle.POINTS, oracle.SEGMENTS, oracle.POLYGON_EDGES):
        for z in (3, 12):
            x = int(rng.integers(1, (1 << z) - 1))
            y = int(rng.integers(1, (1 << z) - 1))
            objs = _random_objects(rng, kind, z, x, y, n_obj)
            ix = _ix(objs, kind, lib_path=lib_path)
            tiles = [(z, x, y), (z, x + 1, y), (z, x, y - 1)]
            rs = rng.choice([0.5, 0.7, 1.0, 2.0, 2.5], 3)
            out = ix.render(np.array(tiles), rs, want_dist=True)
            for t, tile in enumerate(tiles):
                _check_against_brute(out, t, objs, kind, tile, float(rs[t]))
    # lon/lat input: the brute force projects with its own formula.
    lonlat = np.stack([rng.uniform(10.0, 10.6, 100), rng.uniform(45.0, 45.4, 100)], 1)
    ix = _ix(lonlat, oracle.POINTS, merc01=False, lib_path=lib_path)
    m = objects_merc01(lonlat, 0)
    z = 10
    S = 2.0 ** z
    tile = (z, int(m[0, 0] * S), int(m[0, 1] * S))
    out = ix.render(np.array([tile]), 1.5, want_dist=True)
    _check_against_brute(out, 0, m, 0, tile, 1.5)


# ------------------------------------------------------------ work counters
# Per tile the oracle counts C_LIT (pixels with D <= r), C_NBOX_UNLIT (the sum
# over unlit pixels p of N_box(p), the objects whose bounding box meets p's
# c +- r box) and C_UNLIT_CAND (distinct objects whose box meets the c +- r
# box of some unlit pixel).  They give the algorithmic bytes and flops of the
# roofline, so they are pinned like the masks: closed forms and a brute force.
def _cnt(out, t=0):
    c = out["counters"][t]
    return (int(c[oracle.C_LIT]), int(c[oracle.C_AMB]), int(c[oracle.C_NBOX_UNLIT]),
            int(c[oracle.C_UNLIT_CAND]))


def pin_cnt_closed_forms(lib_path=None):
    z, x, y = 10, 300, 400
    t = [[z, x, y]]

    def pts(offsets, r):
        P = [_px_to_merc(z, x, y, u, v) for u, v in offsets]
        return _cnt(_ix(P, oracle.POINTS, lib_path=lib_path).render(t, r, want_counters=True))

    # One point on a pixel centre, r = 2: integer offsets (a, b) with |a|, |b| <= 2
    # put the point in the pixel's box (25 pixels); a^2 + b^2 <= 4 lights 13 of
    # them (4 exactly at 2: ambiguous, lit by the inclusive bit); the other 12
    # are unlit with one object in their box.
    assert pts([(100.5, 50.5)], 2.0) == (13, 4, 12, 1), pts([(100.5, 50.5)], 2.0)
    # On a pixel corner: half-integer offsets, 4 x 4 pixels in the box, 12 lit.
    assert pts([(100.0, 50.0)], 2.0) == (12, 0, 4, 1), pts([(100.0, 50.0)], 2.0)
    # Two far-apart points: everything doubles, two distinct candidates.
    assert pts([(100.5, 50.5), (200.5, 150.5)], 2.0) == (26, 8, 24, 2)
    # Two coincident points: each is its own object, each must be read.
    assert pts([(100.5, 50.5), (100.5, 50.5)], 2.0) == (13, 4, 24, 2)
    # A point 2^-18 px east of a pixel centre, r = 2: offsets a in {-1..2},
    # |b| <= 2 keep it in the pixel's c +- r box (20 pixels; a = -2 misses by
    # 2^-18 px, although the query box c +- (r + 1e-5) still meets it).  Lit:
    # b = 0 with a in {-1..2}, |b| = 1 with a in {-1, 0, 1}: 10.  (0, +-2) lie
    # 2^-38 px beyond r: ambiguous and unlit.  Unlit in the box: 10.
    d = 2.0 ** -18
    assert pts([(100.5 + d, 50.5)], 2.0) == (10, 2, 10, 1), pts([(100.5 + d, 50.5)], 2.0)
    # Far from every pixel of the tile: nothing lit, nothing in any box.
    assert pts([(-40.5, 50.5)], 2.0) == (0, 0, 0, 0)
    # A horizontal segment through the centres of row j, columns a..b (L pixels).
    a, b, j = 20, 60, 77
    L = b - a + 1
    ix = _ix(_seg(z, x, y, a + 0.5, j + 0.5, b + 0.5, j + 0.5), oracle.SEGMENTS, lib_path=lib_path)
    # r = 1/2: its box meets the c +- 1/2 boxes of row j, columns a..b only
    # (the end neighbours' boxes stop at x = a, short of the end at a + 1/2),
    # and all of those are lit: no unlit pixel needs it.
    assert _cnt(ix.render(t, 0.5, want_counters=True)) == (L, 0, 0, 0)
    # r = 1: rows j-1..j+1, columns a-1..b+1; lit: 3L + 2 (2L + 2 exactly at
    # 1); the four corners at sqrt(2) are the unlit ones.
    assert _cnt(ix.render(t, 1.0, want_counters=True)) == (3 * L + 2, 2 * L + 2, 4, 1)


def _brute_counters(objs, kind, z, x, y, r):
    """(C_LIT, C_NBOX_UNLIT, C_UNLIT_CAND, near ties) by enumeration: every
    pixel's c +- r box against every object's box, in tile-local pixels."""
    S = 256.0 * 2.0 ** z
    o = np.asarray(objs, dtype=np.float64).reshape(-1, 2 if kind == 0 else 4)
    if kind == 0:
        o = np.concatenate([o, o], 1)
    u0, u1 = o[:, 0] * S - 256.0 * x, o[:, 2] * S - 256.0 * x
    v0, v1 = o[:, 1] * S - 256.0 * y, o[:, 3] * S - 256.0 * y
    bx0, bx1 = np.minimum(u0, u1), np.maximum(u0, u1)
    by0, by1 = np.minimum(v0, v1), np.maximum(v0, v1)
    c = np.arange(256, dtype=np.float64) + 0.5
    # per axis: does object k's interval meet pixel column / row i's [c - r, c + r]
    mx = (bx0[:, None] <= c[None, :] + r) & (bx1[:, None] >= c[None, :] - r)     # (n, 256) columns
    my = (by0[:, None] <= c[None, :] + r) & (by1[:, None] >= c[None, :] - r)     # (n, 256) rows
    gaps = np.concatenate([np.abs(bx0[:, None] - (c + r)), np.abs(bx1[:, None] - (c - r)),
                           np.abs(by0[:, None] - (c + r)), np.abs(by1[:, None] - (c - r))])
    near = int((gaps < 1e-9).sum())
    D = brute_distance(objs, kind if kind == 0 else 1, z, x, y)
    unlit = D > r
    nbox = np.einsum("kj,ki->ji", my.astype(np.int64), mx.astype(np.int64))   # (row, column)
    hit = np.einsum("kj,ki,ji->k", my.astype(np.int64), mx.astype(np.int64), unlit.astype(np.int64))
    return int((~unlit).sum()), int(nbox[unlit].sum()), int((hit > 0).sum()), near + int(near_band_edge(D, r).sum())


def pin_cnt_brute(lib_path=None, n_obj=120, seed=17):
    rng = np.random.default_rng(seed)
    for kind in (oracle.POINTS, oracle.SEGMENTS):
        for z in (4, 13):
            x = int(rng.integers(1, (1 << z) - 1))
            y = int(rng.integers(1, (1 << z) - 1))
            objs = _random_objects(rng, kind, z, x, y, n_obj)
            # clustered copies too, so that several objects meet one pixel's box
            objs = np.concatenate([objs, objs[:20] + rng.normal(0, 1.0 / (256 * 2.0 ** z), objs[:20].shape)])
            ix = _ix(objs, kind, lib_path=lib_path)
            tiles = [(z, x, y), (z, x - 1, y + 1)]
            rs = (0.7, 2.5)
            out = ix.render(np.array(tiles), np.array(rs), want_counters=True)
            for t, tile in enumerate(tiles):
                lit, nbox, cand, near = _brute_counters(objs, kind, *tile, rs[t])
                assert near == 0, ("choose another seed: a box edge or distance is within 1e-9 px", tile)
                got = _cnt(out, t)
                assert (got[0], got[2], got[3]) == (lit, nbox, cand), (kind, tile, rs[t], got, (lit, nbox, cand))
                assert cand <= len(objs) and (nbox == 0) == (cand == 0)


# ------------------------------------------------------------ cKDTree
def pin_ckdtree(lib_path=None, n_tiles=256):
    from scipy.spatial import cKDTree
    import hvgen
    pts = hvgen.gen_c1_points()
    tiles, r = hvgen.c1_requests()
    tiles = tiles[:n_tiles]
    ix = oracle.OracleIndex(pts, oracle.POINTS, lib_path=lib_path)
    out = ix.render(tiles, r)
    z = 4
    S = 256.0 * 2 ** z
    m = objects_merc01(pts, 0) * S
    kd = cKDTree(m)
    c = np.arange(256) + 0.5
    for t, (tz, tx, ty) in enumerate(tiles):
        q = np.stack([np.tile(c, 256) + 256.0 * tx, np.repeat(c, 256) + 256.0 * ty], 1)
        D, _ = kd.query(q, k=1, workers=-1)
        D = D.reshape(256, 256)
        want = tri_state(D, r)
        ok = (out["tri"][t] == want) | near_band_edge(D, r, tol=1e-8)
        assert ok.all(), (t, int((~ok).sum()))


# ------------------------------------------------------------ invariants
def pin_invariants(lib_path=None):
    rng = np.random.default_rng(17)
    z, x, y = 11, 700, 900
    tiles = np.array([[z, x, y], [z, x + 1, y]])
    for kind in (oracle.POINTS, oracle.SEGMENTS):
        A = _random_objects(rng, kind, z, x, y, 120)
        B = _random_objects(rng, kind, z, x, y, 120)
        for r in (0.5, 1.0, 2.5):
            oa = _ix(A, kind, lib_path=lib_path).render(tiles, r)
            ob = _ix(B, kind, lib_path=lib_path).render(tiles, r)
            AB = np.concatenate([A, B])
            oab = _ix(AB, kind, lib_path=lib_path).render(tiles, r)
            assert np.array_equal(oab["bit"], oa["bit"] | ob["bit"]), ("union", kind, r)
            perm = rng.permutation(AB.shape[0])
            op = _ix(AB[perm], kind, lib_path=lib_path).render(tiles, r)
            assert np.array_equal(op["bit"], oab["bit"]) and np.array_equal(op["tri"], oab["tri"])
        # monotone in r
        ix = _ix(A, kind, lib_path=lib_path)
        prev = None
        for r in (0.3, 0.5, 0.75, 1.0, 1.7, 2.5, 4.0):
            cur = ix.render(tiles, r)["bit"]
            if prev is not None:
                assert np.all(cur >= prev), ("monotone", kind, r)
            prev = cur
    # parent-empty => child-empty for r >= sqrt(2)/2, same r in px at both zooms
    for kind in (oracle.POINTS, oracle.SEGMENTS):
        pz, px_, py_ = 8, 90, 120
        objs = _random_objects(rng, kind, pz, px_, py_, 60, spread=4.0)
        ix = _ix(objs, kind, lib_path=lib_path)
        kids = np.array([[pz + 1, 2 * px_ + a, 2 * py_ + b] for b in (0, 1) for a in (0, 1)])
        for r in (1.0, 2.5):
            par = ix.render([[pz, px_, py_]], r)["bit"][0]
            ch = ix.render(kids, r)["bit"]
            for k, (a, b) in enumerate([(0, 0), (1, 0), (0, 1), (1, 1)]):
                for q in range(2):
                    for s in range(2):
                        sub = ch[k][q::2, s::2]            # child rows 2j'+q, cols 2i'+s
                        parent = par[128 * b:128 * b + 128, 128 * a:128 * a + 128]
                        assert np.all(sub <= parent), ("parent-empty", kind, r, a, b)
    # tile translation: shifting by one tile width in X (exact on a dyadic grid)
    z, x, y = 7, 40, 50
    grid = 2.0 ** -30
    for kind in (oracle.POINTS, oracle.SEGMENTS):
        objs = np.round(_random_objects(rng, kind, z, x, y, 80) / grid) * grid
        sh = objs.copy()
        sh[:, 0::2] += 2.0 ** -z
        o1 = _ix(objs, kind, lib_path=lib_path).render([[z, x, y]], 1.5)
        o2 = _ix(sh, kind, lib_path=lib_path).render([[z, x + 1, y]], 1.5)
        assert np.array_equal(o1["tri"], o2["tri"]), ("translation", kind)


# ------------------------------------------------------------ anti-aliased output
SUB = ((-0.25, 0.25), (0.25, 0.25), (-0.25, -0.25), (0.25, -0.25))   # Algorithm 1's sub-samples


def _odd_lattice_count(r: float) -> int:
    """Sub-samples of the whole plane within r of a point on a pixel centre:
    points ((2k+1)/4, (2l+1)/4), counted with integers."""
    lim = 16.0 * r * r
    m = int(4 * r) + 2
    return sum(1 for k in range(-m, m) for l in range(-m, m) if (2 * k + 1) ** 2 + (2 * l + 1) ** 2 <= lim)


def pin_aa_lattice(lib_path=None):
    """One point on a pixel centre: the values summed over the tile are the
    quarter-odd lattice count; the pixel itself is 4 once r >= sqrt(2)/4."""
    z, x, y = 6, 20, 30
    u, v = 128.5, 100.5
    X, Y = _px_to_merc(z, x, y, u, v)
    ix = _ix([[X, Y]], oracle.POINTS, lib_path=lib_path)
    for r in (0.3, 0.4, 0.8, 1.0, 1.1, 1.6, 2.0, 3.3):
        ex = ix.render_aa([[z, x, y]], r)
        pa = ix.render_aa([[z, x, y]], r, mode="paper")
        assert int(ex["val"].sum()) == _odd_lattice_count(r), ("aa lattice", r)
        assert int(ex["val"][0, 100, 128]) == (4 if r >= math.sqrt(2) / 4 else 0), ("aa own pixel", r)
        assert not ex["amb"].any() and np.array_equal(ex["sure"], ex["val"]), ("aa no ties", r)
        assert np.array_equal(pa["val"], ex["val"]), ("aa one object: paper = exact", r)


def pin_aa_ties_and_paper(lib_path=None):
    """Exact ties count (inclusive); the printed step undercounts where a
    sub-sample's nearest object is not the centre's."""
    z, x, y = 0, 0, 0
    # a point exactly 0.5 px east of the north-east sub-sample of pixel (100, 80)
    cu, cv = 100.5, 80.5
    X, Y = _px_to_merc(z, x, y, cu + 0.25 + 0.5, cv - 0.25)
    ex = _ix([[X, Y]], oracle.POINTS, lib_path=lib_path).render_aa([[z, x, y]], 0.5)
    assert ex["amb"][0, 80, 100] == 1 and ex["val"][0, 80, 100] == 1 and ex["sure"][0, 80, 100] == 0
    # two points: A 0.625 px east of the centre (the nearest), B 0.640625 px
    # west; r = 0.5 px puts the centre in the transition band (R1 < 0.625 < R2)
    A = _px_to_merc(z, x, y, cu + 0.625, cv)
    B = _px_to_merc(z, x, y, cu - 0.640625, cv)
    ix = _ix([[A[0], A[1]], [B[0], B[1]]], oracle.POINTS, lib_path=lib_path)
    ex = ix.render_aa([[z, x, y]], 0.5)
    pa = ix.render_aa([[z, x, y]], 0.5, mode="paper")
    assert ex["val"][0, 80, 100] == 4, "east pair from A, west pair from B"
    assert pa["val"][0, 80, 100] == 2, "only A (the centre's nearest) is measured"
    assert not ex["amb"][0, 80, 100] and not pa["amb"][0, 80, 100]


def pin_aa_brute(lib_path=None, n_obj=120, seed=21):
    """Every object against every sub-sample (numpy), and the identity with
    binary masks one zoom deeper at twice the radius (the sub-samples are
    exactly that zoom's pixel centres)."""
    rng = np.random.default_rng(seed)
    for kind in (oracle.POINTS, oracle.SEGMENTS):
        for (z, x, y), r in (((3, 2, 5), 0.5), ((7, 40, 77), 1.3), ((12, 2000, 1500), 2.5)):
            objs = _random_objects(rng, kind, z, x, y, n_obj)
            ix = _ix(objs, kind, lib_path=lib_path)
            ex = ix.render_aa([[z, x, y]], r)
            val = np.zeros((256, 256), dtype=np.int32)
            edge = np.zeros((256, 256), dtype=bool)
            for off in SUB:
                D = brute_distance(objs, kind, z, x, y, off=off)
                val += D <= r
                edge |= near_band_edge(D, r)
            ok = ~edge
            assert np.array_equal(ex["val"][0][ok], val[ok]), ("aa brute", kind, z, r)
            kids = [(z + 1, 2 * x + dx, 2 * y + dy) for dy in (0, 1) for dx in (0, 1)]
            b = ix.render(kids, 2 * r)["bit"].reshape(2, 2, 256, 256)
            full = np.block([[b[0, 0], b[0, 1]], [b[1, 0], b[1, 1]]]).astype(np.int32)
            s4 = full.reshape(256, 2, 256, 2).sum(axis=(1, 3))
            assert np.array_equal(s4, ex["val"][0]), ("aa = deeper zoom at 2r", kind, z, r)
            pa = ix.render_aa([[z, x, y]], r, mode="paper")
            assert np.all(pa["val"] <= ex["val"]), ("paper <= exact", kind, z, r)
            # Algorithm 1's early answers: D(P) <= R1 -> 4, D(P) > R2 -> 0
            D0 = brute_distance(objs, kind, z, x, y)
            q = math.sqrt(2) / 4
            inner, outer = D0 < r - q - 1e-9, D0 > r + q + 1e-9
            assert np.all(ex["val"][0][inner] == 4) and np.all(pa["val"][0][inner] == 4), ("R1", kind)
            assert np.all(ex["val"][0][outer] == 0) and np.all(pa["val"][0][outer] == 0), ("R2", kind)


# ------------------------------------------------------------ polygon filling
def _ring(z, x, y, pts):
    """Closed ring of tile-local px vertices -> edges (k, 4) normalised."""
    X, Y = _px_to_merc(z, x, y, np.array([p[0] for p in pts]), np.array([p[1] for p in pts]))
    return np.stack([X, Y, np.roll(X, -1), np.roll(Y, -1)], 1)


def _polys(z, x, y, rings_per_poly):
    edges, first = [], [0]
    for rings in rings_per_poly:
        for ring in rings:
            edges.append(_ring(z, x, y, ring))
        first.append(first[-1] + sum(len(r) for r in rings))
    return np.concatenate(edges), np.array(first)


def _fill(edges, first, tiles, lib_path=None):
    return oracle.OraclePolygons(edges, first, merc01=True, lib_path=lib_path).render(tiles)


def _box(u0, v0, u1, v1):
    return [(u0, v0), (u1, v0), (u1, v1), (u0, v1)]


def pin_fill_closed_forms(lib_path=None):
    """Squares, a hole, a separate polygon over the hole, a right triangle."""
    z, x, y = 9, 300, 200
    t = [[z, x, y]]
    # square [10.25, 20.75] x [30.25, 40.75]: centres 10.5..20.5 and 30.5..40.5
    e, f = _polys(z, x, y, [[_box(10.25, 30.25, 20.75, 40.75)]])
    o = _fill(e, f, t, lib_path)
    assert int((o["tri"] == 1).sum()) == 121 and not (o["tri"] == 2).any(), "square"
    assert o["bit"][0, 35, 15] == 1 and o["bit"][0, 41, 15] == 0 and o["bit"][0, 35, 9] == 0, "square addressing"
    # the same square with a hole [13.25, 16.75]^2 + 20 as a second ring
    hole = _box(13.25, 33.25, 16.75, 36.75)
    e, f = _polys(z, x, y, [[_box(10.25, 30.25, 20.75, 40.75), hole]])
    o = _fill(e, f, t, lib_path)
    assert int((o["tri"] == 1).sum()) == 121 - 16 and o["bit"][0, 35, 15] == 0, "hole (one polygon, two rings)"
    # the hole as a polygon of its own lies inside the square: still filled
    e, f = _polys(z, x, y, [[_box(10.25, 30.25, 20.75, 40.75)], [hole]])
    o = _fill(e, f, t, lib_path)
    assert int((o["tri"] == 1).sum()) == 121, "union over polygons"
    # right triangle (100,100) (100+L,100) (100,100+L): centres with
    # (i+.5-100) + (j+.5-100) < L inside, = L on the hypotenuse (ambiguous)
    L = 37
    e, f = _polys(z, x, y, [[[(100.0, 100.0), (100.0 + L, 100.0), (100.0, 100.0 + L)]]])
    o = _fill(e, f, t, lib_path)
    assert int((o["tri"] == 1).sum()) == L * (L - 1) // 2, "triangle interior"
    assert int((o["tri"] == 2).sum()) == L, "triangle hypotenuse centres"
    # orientation and a vertex exactly on a row of centres (half-open rule)
    e, f = _polys(z, x, y, [[[(50.5, 60.0), (70.5, 80.5), (50.5, 101.0), (30.5, 80.5)]]])
    o1 = _fill(e, f, t, lib_path)
    e2 = e[::-1][:, [2, 3, 0, 1]]
    o2 = _fill(e2, f, t, lib_path)
    assert np.array_equal(o1["tri"], o2["tri"]), "orientation"
    assert o1["bit"][0, 80, 50] == 1 and o1["tri"][0, 80, 50] == 1, "diamond centre"


def _star_polys(rng, z, x, y, n_poly, spread=40.0):
    rings = []
    for _ in range(n_poly):
        c = rng.uniform(-spread, 256 + spread, 2)
        k = int(rng.integers(4, 25))
        rho = rng.uniform(3.0, 60.0)
        ang = np.sort(rng.uniform(0, 2 * np.pi, k))
        rad = rho * rng.uniform(0.5, 1.0, k)
        rings.append([[(c[0] + rad[q] * np.cos(ang[q]), c[1] + rad[q] * np.sin(ang[q])) for q in range(k)]])
    return _polys(z, x, y, rings)


def pin_fill_brute(lib_path=None, seed=31):
    """Random star polygons against a numpy crossing count towards -x."""
    rng = np.random.default_rng(seed)
    for (z, x, y), n_poly in (((4, 3, 5), 12), ((11, 900, 700), 30), ((17, 60000, 50000), 8)):
        e, f = _star_polys(rng, z, x, y, n_poly)
        o = _fill(e, f, [[z, x, y]], lib_path)
        inside, dist = brute_fill(e, f, z, x, y)
        ok = dist > 1e-6 + 1e-9
        assert np.array_equal(o["tri"][0][ok].astype(bool), inside[ok]), ("fill brute", z)
        assert np.all(o["tri"][0][~ok] == 2) or np.all(inside[~ok] | (o["tri"][0][~ok] != 1)), ("fill band", z)


def pin_fill_invariants(lib_path=None, seed=37):
    """Reversed edges, cut edges (Algorithm 2's segment cutting must not
    matter), permuted edges and polygons, tile translation."""
    rng = np.random.default_rng(seed)
    z, x, y = 10, 500, 400
    e, f = _star_polys(rng, z, x, y, 20)
    t = [[z, x, y]]
    base = _fill(e, f, t, lib_path)["tri"]
    rev = e[:, [2, 3, 0, 1]]
    assert np.array_equal(_fill(rev, f, t, lib_path)["tri"], base), "reversed edges"
    mid = 0.5 * (e[:, :2] + e[:, 2:])
    cut = np.empty((2 * len(e), 4))
    cut[0::2] = np.concatenate([e[:, :2], mid], 1)
    cut[1::2] = np.concatenate([mid, e[:, 2:]], 1)
    assert np.array_equal(_fill(cut, 2 * f, t, lib_path)["tri"], base), "cut edges"
    perm_e = np.concatenate([e[f[p]:f[p + 1]][rng.permutation(f[p + 1] - f[p])] for p in range(len(f) - 1)])
    assert np.array_equal(_fill(perm_e, f, t, lib_path)["tri"], base), "edges permuted within a polygon"
    order = rng.permutation(len(f) - 1)
    pe = np.concatenate([e[f[p]:f[p + 1]] for p in order])
    pf = np.concatenate([[0], np.cumsum([f[p + 1] - f[p] for p in order])])
    assert np.array_equal(_fill(pe, pf, t, lib_path)["tri"], base), "polygons permuted"
    sh = e.copy()
    S = 256.0 * 2 ** z
    sh[:, 0] += 256.0 / S
    sh[:, 2] += 256.0 / S
    assert np.array_equal(_fill(sh, f, [[z, x + 1, y]], lib_path)["tri"], base), "translation"


# ------------------------------------------------------------ fill work counters
# The fill roofline's algorithmic work: candidate polygons (boxes holding a
# pixel centre), needed edges (crossed in y by a ray on one of their polygon's
# centre rows, half-open as in the fill), (edge, row) crossings and
# (pixel, candidate polygon) pairs.
def _fillcnt(edges, first, tiles, lib_path=None):
    return oracle.OraclePolygons(edges, first, merc01=True, lib_path=lib_path).counters(np.array(tiles))


def pin_fillcnt_closed_forms(lib_path=None):
    z, x, y = 9, 300, 200
    t = [[z, x, y]]
    # square [10.25, 20.75] x [30.25, 40.75]: centres 10.5..20.5 (11 columns)
    # and 30.5..40.5 (11 rows); its two vertical sides cross all 11 rows, the
    # horizontal ones none
    e, f = _polys(z, x, y, [[_box(10.25, 30.25, 20.75, 40.75)]])
    assert _fillcnt(e, f, t, lib_path).tolist() == [[1, 2, 22, 121]]
    # a hole as a second ring: two more vertical sides over rows 33.5..36.5
    e, f = _polys(z, x, y, [[_box(10.25, 30.25, 20.75, 40.75), _box(13.25, 33.25, 16.75, 36.75)]])
    assert _fillcnt(e, f, t, lib_path).tolist() == [[1, 4, 30, 121]]
    # two polygons: the counts add
    e, f = _polys(z, x, y, [[_box(10.25, 30.25, 20.75, 40.75)], [_box(100.0, 100.0, 110.0, 105.0)]])
    assert _fillcnt(e, f, t, lib_path).tolist() == [[2, 4, 22 + 10, 121 + 50]]
    # a box between two centre columns holds no centre: no candidate
    e, f = _polys(z, x, y, [[_box(10.6, 30.25, 11.4, 40.75)]])
    assert _fillcnt(e, f, t, lib_path).tolist() == [[0, 0, 0, 0]]
    # vertices on centre rows, half-open rule: an edge crosses the rows
    # j + 0.5 in [min y, max y).  Diamond (50.5, 60) (70.5, 80.5) (50.5, 101)
    # (30.5, 80.5): box rows and columns 60.5..100.5 and 30.5..70.5 (41 each);
    # the upper sides cross 60.5..79.5 (20 rows each), the lower ones
    # 80.5..100.5 (21 each)
    e, f = _polys(z, x, y, [[[(50.5, 60.0), (70.5, 80.5), (50.5, 101.0), (30.5, 80.5)]]])
    got = _fillcnt(e, f, t, lib_path).tolist()[0]
    assert got == [1, 4, 20 + 20 + 21 + 21, 41 * 41], got
    # a top vertex on a centre row, both sides going south to y = 80.2 and a
    # horizontal base: each side crosses 60.5..79.5 (20 rows), the base none;
    # box columns 30.5..69.5 (40) by rows 60.5..79.5 (20)
    e, f = _polys(z, x, y, [[[(50.5, 60.5), (70.2, 80.2), (30.2, 80.2)]]])
    got = _fillcnt(e, f, t, lib_path).tolist()[0]
    assert got == [1, 2, 40, 800], got
    # the tile next door along x sees nothing of the square
    e, f = _polys(z, x, y, [[_box(10.25, 30.25, 20.75, 40.75)]])
    assert _fillcnt(e, f, [[z, x + 1, y]], lib_path).tolist() == [[0, 0, 0, 0]]


def _brute_fillcnt(edges, first, z, x, y):
    """The four fill counters by enumeration over all 256 x 256 centres."""
    S = 256.0 * 2.0 ** z
    e = np.asarray(edges, dtype=np.float64).reshape(-1, 4)
    ax, ay = e[:, 0] * S - 256.0 * x, e[:, 1] * S - 256.0 * y
    bx, by = e[:, 2] * S - 256.0 * x, e[:, 3] * S - 256.0 * y
    c = np.arange(256, dtype=np.float64) + 0.5
    cand = need = pairs = px = 0
    for p in range(len(first) - 1):
        q = slice(first[p], first[p + 1])
        x0, x1 = min(ax[q].min(), bx[q].min()), max(ax[q].max(), bx[q].max())
        y0, y1 = min(ay[q].min(), by[q].min()), max(ay[q].max(), by[q].max())
        cols = (c >= x0) & (c <= x1)
        rows = (c >= y0) & (c <= y1)
        if not cols.any() or not rows.any():
            continue
        cand += 1
        px += int(cols.sum()) * int(rows.sum())
        for k in range(first[p], first[p + 1]):
            crossed = rows & ((ay[k] > c) != (by[k] > c))
            if crossed.any():
                need += 1
                pairs += int(crossed.sum())
    return cand, need, pairs, px


def pin_fillcnt_brute(lib_path=None, seed=43):
    rng = np.random.default_rng(seed)
    for z in (5, 12):
        x = int(rng.integers(1, (1 << z) - 1))
        y = int(rng.integers(1, (1 << z) - 1))
        e, f = _star_polys(rng, z, x, y, 30, spread=120.0)
        tiles = [(z, x, y), (z, x + 1, y), (z, x, y - 1)]
        got = _fillcnt(e, f, tiles, lib_path)
        for k, tile in enumerate(tiles):
            want = _brute_fillcnt(e, f, *tile)
            assert tuple(int(v) for v in got[k]) == want, (tile, got[k].tolist(), want)
        assert got[:, 0].sum() > 0 and got[:, 2].sum() > got[:, 1].sum()


PINS = {
    "projection": pin_projection,
    "addressing": pin_addressing,
    "lattice": pin_lattice,
    "segments": pin_segments,
    "kinds": pin_kinds,
    "brute": pin_brute,
    "invariants": pin_invariants,
    "aa_lattice": pin_aa_lattice,
    "aa_ties_and_paper": pin_aa_ties_and_paper,
    "aa_brute": pin_aa_brute,
    "fill_closed_forms": pin_fill_closed_forms,
    "fill_brute": pin_fill_brute,
    "fill_invariants": pin_fill_invariants,
    "cnt_closed_forms": pin_cnt_closed_forms,
    "cnt_brute": pin_cnt_brute,
    "fillcnt_closed_forms": pin_fillcnt_closed_forms,
    "fillcnt_brute": pin_fillcnt_brute,
}
