"""CPU oracle for per-pixel tile masks -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the GPU path and the product never
calls it.  The arithmetic lives in ``hv_oracle.c`` (plain C, FP64, no FMA
contraction); this module only marshals numpy arrays through ctypes.

What it computes is the plain definition of the binary mask read from the
paper's Algorithm 1 (Sec. 3.2.1): pixel (i, j) of tile (z, x, y) is lit iff
the distance D from its centre to the nearest object is <= r px.  Each pixel
also gets a tri-state value (0 unlit, 1 lit, 2 ambiguous when |D - r| <=
1e-6 px) and per-tile work counters.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

POINTS, SEGMENTS, POLYGON_EDGES = 0, 1, 2
MERC01 = 0x100
BAND = 1e-6
UNLIT, LIT, AMBIGUOUS = 0, 1, 2
# per-tile counters
C_NODES, C_LIT, C_AMB, C_NBOX_UNLIT, C_UNLIT_CAND = range(5)

_lib = None


def _load(path: str | None = None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _bind(lib):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_build.restype = P
    lib.oracle_build.argtypes = [P, ctypes.c_int, I64]
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [P]
    lib.oracle_render.restype = ctypes.c_int
    lib.oracle_render.argtypes = [P, P, I64, P, P, P, P, P, ctypes.c_int]
    lib.oracle_project.restype = ctypes.c_int
    lib.oracle_project.argtypes = [P, I64, P, P]
    lib.oracle_node_count.restype = I64
    lib.oracle_node_count.argtypes = [P]
    lib.oracle_depth.restype = ctypes.c_int
    lib.oracle_depth.argtypes = [P]
    lib.oracle_root_box.restype = ctypes.c_int
    lib.oracle_root_box.argtypes = [P, P]
    lib.oracle_build_polygons.restype = P
    lib.oracle_build_polygons.argtypes = [P, I64, P, I64, ctypes.c_int]
    lib.oracle_free_polygons.restype = None
    lib.oracle_free_polygons.argtypes = [P]
    lib.oracle_render_fill.restype = ctypes.c_int
    lib.oracle_render_fill.argtypes = [P, P, I64, P, P, ctypes.c_int]
    lib.oracle_fill_counters.restype = ctypes.c_int
    lib.oracle_fill_counters.argtypes = [P, P, I64, P, ctypes.c_int]
    lib.oracle_render_aa.restype = ctypes.c_int
    lib.oracle_render_aa.argtypes = [P, P, I64, P, ctypes.c_int, P, P, P, ctypes.c_int]
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def project(lonlat: np.ndarray, lib_path: str | None = None):
    """(n,2) lon/lat degrees -> (X, Y) normalised Web-Mercator, y south."""
    lib = _load(lib_path)
    ll = np.ascontiguousarray(lonlat, dtype=np.float64).reshape(-1, 2)
    X = np.empty(ll.shape[0])
    Y = np.empty(ll.shape[0])
    lib.oracle_project(_ptr(ll), ll.shape[0], _ptr(X), _ptr(Y))
    return X, Y


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


class OracleIndex:
    """Serial STR R-tree over points / segments / polygon edges."""

    def __init__(self, objects: np.ndarray, kind: int, merc01: bool = False,
                 lib_path: str | None = None):
        self._lib = _load(lib_path)
        width = 2 if kind == POINTS else 4
        self._obj = np.ascontiguousarray(objects, dtype=np.float64).reshape(-1, width)
        self.kind = kind
        self.n = self._obj.shape[0]
        self._h = self._lib.oracle_build(_ptr(self._obj), kind | (MERC01 if merc01 else 0), self.n)
        if not self._h:
            raise MemoryError("oracle_build failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_free(h)
            self._h = None

    @property
    def node_count(self) -> int:
        return int(self._lib.oracle_node_count(self._h))

    @property
    def depth(self) -> int:
        return int(self._lib.oracle_depth(self._h))

    def root_box(self):
        out = np.empty(4)
        return out if self._lib.oracle_root_box(self._h, _ptr(out)) else None

    def render(self, tiles: np.ndarray, r, nthreads: int | None = None,
               want_bit: bool = True, want_dist: bool = False, want_counters: bool = False):
        """Returns dict with 'tri' (n,256,256) u8 and optionally 'bit', 'dist',
        'counters' (n,5) int64.  ``r`` is a scalar or one value per tile."""
        t = np.ascontiguousarray(tiles, dtype=np.int32).reshape(-1, 3)
        n = t.shape[0]
        rr = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=np.float64), (n,)))
        tri = np.empty((n, 256, 256), dtype=np.uint8)
        bit = np.empty((n, 256, 256), dtype=np.uint8) if want_bit else None
        dist = np.empty((n, 256, 256), dtype=np.float64) if want_dist else None
        cnt = np.zeros((n, 5), dtype=np.int64) if want_counters else None
        th = default_threads() if nthreads is None else nthreads
        rc = self._lib.oracle_render(self._h, _ptr(t), n, _ptr(rr), _ptr(tri), _ptr(bit),
                                     _ptr(dist), _ptr(cnt), th)
        if rc != 0:
            raise ValueError("oracle_render rejected its arguments")
        out = {"tri": tri}
        if want_bit:
            out["bit"] = bit
        if want_dist:
            out["dist"] = dist
        if want_counters:
            out["counters"] = cnt
        return out

    def render_aa(self, tiles: np.ndarray, r, mode: str = "exact", nthreads: int | None = None):
        """Algorithm 1's anti-aliased output (Sec. 3.2.1): per pixel 0-4, the
        number of its sub-samples (centre +- 1/4 px in x and y) within r.

        mode "exact": each sub-sample against its own nearest object; returns
        'val', 'amb' (sub-samples within 1e-6 px of r) and 'sure' (sub-samples
        certainly within r).  mode "paper": Algorithm 1's steps as printed,
        counting the sub-samples within r of the object nearest to the pixel
        centre; returns 'val' and 'amb' (1 where a threshold or the choice of
        that object is within 1e-6 px)."""
        t = np.ascontiguousarray(tiles, dtype=np.int32).reshape(-1, 3)
        n = t.shape[0]
        rr = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=np.float64), (n,)))
        val = np.empty((n, 256, 256), dtype=np.uint8)
        amb = np.empty((n, 256, 256), dtype=np.uint8)
        sure = np.empty((n, 256, 256), dtype=np.uint8) if mode == "exact" else None
        m = {"exact": 0, "paper": 1}[mode]
        th = default_threads() if nthreads is None else nthreads
        rc = self._lib.oracle_render_aa(self._h, _ptr(t), n, _ptr(rr), m, _ptr(val), _ptr(amb), _ptr(sure), th)
        if rc != 0:
            raise ValueError("oracle_render_aa rejected its arguments")
        out = {"val": val, "amb": amb}
        if sure is not None:
            out["sure"] = sure
        return out


class OraclePolygons:
    """Polygon filling (Sec. 3.2.2, Algorithm 2) on the CPU: edges (n, 4)
    lon0, lat0, lon1, lat1 (or normalised Mercator with merc01=True);
    polygon p owns edges first[p] .. first[p+1]-1, which form closed rings."""

    def __init__(self, edges, first, merc01: bool = False, lib_path: str | None = None):
        self._lib = _load(lib_path)
        e = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1, 4)
        f = np.ascontiguousarray(first, dtype=np.int64)
        self._keep = (e, f)
        self._h = self._lib.oracle_build_polygons(_ptr(e), e.shape[0], _ptr(f), f.shape[0] - 1, int(merc01))
        if not self._h:
            raise ValueError("oracle_build_polygons rejected its arguments")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_free_polygons(h)
            self._h = None

    def render(self, tiles, nthreads: int | None = None):
        """Returns dict 'tri' (0 outside, 1 inside, 2 within 1e-6 px of an
        edge) and 'bit' (inside some polygon), each (n, 256, 256) u8."""
        t = np.ascontiguousarray(tiles, dtype=np.int32).reshape(-1, 3)
        n = t.shape[0]
        tri = np.empty((n, 256, 256), dtype=np.uint8)
        bit = np.empty((n, 256, 256), dtype=np.uint8)
        th = default_threads() if nthreads is None else nthreads
        if self._lib.oracle_render_fill(self._h, _ptr(t), n, _ptr(tri), _ptr(bit), th) != 0:
            raise ValueError("oracle_render_fill rejected its arguments")
        return {"tri": tri, "bit": bit}

    def counters(self, tiles, nthreads: int | None = None):
        """Work of filling each tile, (n, 4) int64: candidate polygons (boxes
        holding a pixel centre), needed edges (edges of those polygons that
        a ray on one of the polygon's centre rows crosses in y), (edge, row)
        crossings, and (pixel, candidate polygon) pairs."""
        t = np.ascontiguousarray(tiles, dtype=np.int32).reshape(-1, 3)
        n = t.shape[0]
        cnt = np.zeros((n, 4), dtype=np.int64)
        th = default_threads() if nthreads is None else nthreads
        if self._lib.oracle_fill_counters(self._h, _ptr(t), n, _ptr(cnt), th) != 0:
            raise ValueError("oracle_fill_counters rejected its arguments")
        return cnt
