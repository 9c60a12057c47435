"""Seeded generators: reproducible, right shapes, sizes and ranges."""
import hashlib

import numpy as np

import hvgen


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_c1_reproducible():
    a = hvgen.gen_c1_points()
    b = hvgen.gen_c1_points()
    assert a.shape == (10_000, 2) and _h(a) == _h(b)
    assert a[:, 0].min() >= -180 and a[:, 0].max() < 180
    assert a[:, 1].min() >= -85 and a[:, 1].max() < 85
    t, r = hvgen.c1_requests()
    assert t.shape == (256, 3) and r == 2.0
    assert (t[:, 0] == 4).all() and t[1].tolist() == [4, 1, 0]      # row-major in y, then x


def test_c2_shape_and_recipe():
    s = hvgen.gen_c2_segments(n_segments=200_000)
    assert s.shape == (200_000, 4)
    assert np.abs(s[:, [0, 2]]).max() <= 180 and np.abs(s[:, [1, 3]]).max() <= 85
    step = np.hypot(s[:, 2] - s[:, 0], s[:, 3] - s[:, 1])
    assert 0.008 < np.median(step) < 0.012                 # log-normal median 0.01 deg
    # consecutive segments of a polyline share a vertex
    joined = np.mean((s[1:, 0] == s[:-1, 2]) & (s[1:, 1] == s[:-1, 3]))
    assert 0.9 < joined < 0.99
    assert _h(s) == _h(hvgen.gen_c2_segments(n_segments=200_000))
    t, r = hvgen.c2_requests()
    assert t.shape == (4096, 3) and r == 0.5


def test_c3_chunks_and_requests():
    a = hvgen.gen_c3_chunk(0, 50_000)
    b = hvgen.gen_c3_chunk(1, 50_000)
    assert a.shape == (50_000, 2) and _h(a) != _h(b)
    assert _h(a) == _h(hvgen.gen_c3_chunk(0, 50_000))
    t, r = hvgen.c3_requests(1000)
    n = 1 << t[:, 0].astype(np.int64)
    assert t[:, 0].min() >= 0 and t[:, 0].max() <= 18
    assert (t[:, 1] < n).all() and (t[:, 2] < n).all() and (t[:, 1:] >= 0).all()
    assert r.min() >= 1 and r.max() <= 3


def test_c4_polygons_closed():
    e = hvgen.gen_c4_edges(min_edges=20_000, batch_polygons=500)
    assert e.shape[0] >= 20_000
    # each polygon is a closed ring: the multiset of starts equals that of ends
    a = np.sort(e[:, 0] * 1e3 + e[:, 1])
    b = np.sort(e[:, 2] * 1e3 + e[:, 3])
    assert np.array_equal(a, b)
    t, r = hvgen.c4_requests(e, n=512)
    assert set(np.unique(r)) <= {0.5, 1.0, 1.5, 2.0, 2.5}
    assert t[:, 0].min() >= 2 and t[:, 0].max() <= 20


def test_c5_arrivals():
    s = hvgen.gen_c2_segments(n_segments=10_000)
    d = hvgen.c5_arrivals(1000.0, c2_objects=s, max_requests=2000)
    assert np.all(np.diff(d["t"]) >= 0) and len(d["t"]) == 2000
    assert set(np.unique(d["dataset"])) == {0, 1}
