"""Python binding of the tile-mask C ABI (include/hv.h): marshalling only.

Every entry point of the library has a function of the same name here; each
converts its arguments (torch tensors, numpy arrays, Python numbers) to the
C types, sets the library's stream to torch's current stream, calls the
library and turns a negative status into ``HvError``.  All computation runs
in the HIP kernels of ``libhv.so``; if that library is missing, importing
this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch supplies device memory and streams, and ships its own HIP runtime.
# It must be loaded first so that libhv.so binds to that same runtime (both
# carry the soname libamdhip64.so.7); two runtimes in one process would not
# recognise each other's allocations or streams.
import torch  # noqa: F401,E402

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhv.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2005_12489_amd/build.py "
                      "(or __graft_entry__.build()) first")


def _hip_runtimes() -> set:
    with open("/proc/self/maps") as f:
        return {ln.split()[-1] for ln in f if "libamdhip64" in ln and "/" in ln}

HV_POINTS, HV_SEGMENTS, HV_POLYGON_EDGES, HV_POLYGONS = 0, 1, 2, 3
HV_INPUT_MERC01 = 0x100
HV_OK, HV_EINVAL, HV_ENOMEM, HV_EHIP = 0, -1, -2, -3
HV_READ_ORDER, HV_READ_OBJECTS, HV_READ_NODES = 0, 1, 2
HV_MASK_BYTES = 8192
HV_AA_BYTES = 65536
HV_MAX_ZOOM = 22
HV_NOALLOC_MAX_REQUESTS = 4096
HV_NOALLOC_MAX_INDEXES = 16

SYMBOLS = ("hv_index_build", "hv_render_tiles", "hv_render_tiles_ex", "hv_free", "hv_last_error",
           "hv_set_stream", "hv_index_info", "hv_index_read", "hv_render_batch", "hv_batcher_create",
           "hv_batcher_run", "hv_batcher_latency", "hv_batcher_free", "hv_autotune", "hv_tuned_launch",
           "hv_time_kernels", "hv_time_aa", "hv_time_fill", "hv_render_batch_aa", "hv_polygon_index_build", "hv_render_fill",
           "hv_render_batch_noalloc", "hv_estimate_bytes", "hv_estimate_batch_bytes")

# hv_request as a numpy record (32 bytes, the C layout)
REQUEST_DTYPE = np.dtype([("index", np.uint64), ("z", np.int32), ("x", np.int32), ("y", np.int32),
                          ("pad", np.int32), ("r_px", np.float64)])


class hv_tile(ctypes.Structure):
    _fields_ = [("z", ctypes.c_int32), ("x", ctypes.c_int32), ("y", ctypes.c_int32), ("pad", ctypes.c_int32)]


class hv_style(ctypes.Structure):
    _fields_ = [("r_px", ctypes.c_double)]


class hv_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("cand_cap", ctypes.c_int32),
                ("waves_per_wg", ctypes.c_int32), ("grid_wgs", ctypes.c_int32), ("region", ctypes.c_int32),
                ("objs_per_lane", ctypes.c_int32), ("cull_nodes", ctypes.c_int32),
                ("aa_split", ctypes.c_int32)]


class hv_info(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("levels", ctypes.c_int32), ("n", ctypes.c_int64),
                ("nodes", ctypes.c_int64), ("leaf_size", ctypes.c_int32), ("fanout", ctypes.c_int32),
                ("key_bits", ctypes.c_int32), ("pad", ctypes.c_int32), ("root", ctypes.c_double * 4),
                ("device_bytes", ctypes.c_int64), ("build_ms", ctypes.c_double)]


class HvError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{code}: {message}")
        self.code = code


_P = ctypes.c_void_p
lib = ctypes.CDLL(LIB_PATH)
if len(_hip_runtimes()) > 1:
    raise ImportError(f"two HIP runtimes are loaded ({sorted(_hip_runtimes())}); "
                      "libhv.so must share torch's")
lib.hv_index_build.restype = _P
lib.hv_index_build.argtypes = [_P, ctypes.c_int, ctypes.c_int64]
lib.hv_render_tiles.restype = ctypes.c_int
lib.hv_render_tiles.argtypes = [_P, _P, ctypes.c_int64, ctypes.POINTER(hv_style), _P]
lib.hv_render_tiles_ex.restype = ctypes.c_int
lib.hv_render_tiles_ex.argtypes = [_P, _P, ctypes.c_int64, ctypes.POINTER(hv_style), _P,
                                   ctypes.POINTER(hv_launch)]
lib.hv_free.restype = None
lib.hv_free.argtypes = [_P]
lib.hv_last_error.restype = ctypes.c_char_p
lib.hv_last_error.argtypes = []
lib.hv_set_stream.restype = ctypes.c_int
lib.hv_set_stream.argtypes = [_P]
lib.hv_index_info.restype = ctypes.c_int
lib.hv_index_info.argtypes = [_P, ctypes.POINTER(hv_info)]
lib.hv_index_read.restype = ctypes.c_int
lib.hv_index_read.argtypes = [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int64]


lib.hv_render_batch.restype = ctypes.c_int
lib.hv_render_batch.argtypes = [_P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch)]
lib.hv_estimate_bytes.restype = ctypes.c_int64
lib.hv_estimate_bytes.argtypes = [_P, ctypes.POINTER(hv_tile), ctypes.POINTER(hv_style)]
lib.hv_estimate_batch_bytes.restype = ctypes.c_int64
lib.hv_estimate_batch_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
lib.hv_render_batch_noalloc.restype = ctypes.c_int
lib.hv_render_batch_noalloc.argtypes = [_P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch)]
lib.hv_batcher_create.restype = _P
lib.hv_batcher_create.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(hv_launch)]
lib.hv_batcher_run.restype = ctypes.c_int
lib.hv_batcher_run.argtypes = [_P, _P, ctypes.c_int64, _P]
lib.hv_batcher_latency.restype = ctypes.c_int
lib.hv_batcher_latency.argtypes = [_P, _P, ctypes.c_int64]
lib.hv_batcher_free.restype = None
lib.hv_batcher_free.argtypes = [_P]
lib.hv_autotune.restype = ctypes.c_int
lib.hv_autotune.argtypes = [_P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch), ctypes.POINTER(ctypes.c_double)]
lib.hv_tuned_launch.restype = ctypes.c_int
lib.hv_tuned_launch.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(hv_launch)]
lib.hv_polygon_index_build.restype = _P
lib.hv_polygon_index_build.argtypes = [_P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int]
lib.hv_render_fill.restype = ctypes.c_int
lib.hv_render_fill.argtypes = [_P, _P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch)]
lib.hv_render_batch_aa.restype = ctypes.c_int
lib.hv_render_batch_aa.argtypes = [_P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch)]
lib.hv_time_fill.restype = ctypes.c_int
lib.hv_time_fill.argtypes = [_P, _P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch), ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_double)]
lib.hv_time_aa.restype = ctypes.c_int
lib.hv_time_aa.argtypes = [_P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch), ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_double)]
lib.hv_time_kernels.restype = ctypes.c_int
lib.hv_time_kernels.argtypes = [_P, ctypes.c_int64, _P, ctypes.POINTER(hv_launch), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_double)]


def _check(rc: int) -> int:
    if rc < 0:
        raise HvError(rc, hv_last_error())
    return rc


def _device_ptr(t):
    """A torch tensor's device address, or an int address as given."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _sync_stream():
    """Points the library at torch's current stream (if torch has a GPU)."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        return
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        lib.hv_set_stream(torch.cuda.current_stream().cuda_stream)


def tiles_array(tiles) -> np.ndarray:
    """(n,3) or (n,4) integers z, x, y[, pad] -> contiguous (n,4) int32."""
    t = np.asarray(tiles, dtype=np.int64).reshape(-1, np.shape(tiles)[-1] if np.ndim(tiles) > 1 else 3)
    out = np.zeros((t.shape[0], 4), dtype=np.int32)
    if t.size and (t[:, :3].min() < np.iinfo(np.int32).min or t[:, :3].max() > np.iinfo(np.int32).max):
        raise HvError(HV_EINVAL, "tile coordinates do not fit int32")
    out[:, :3] = t[:, :3]
    return out


# ------------------------------------------------------------ entry points
def hv_last_error() -> str:
    return lib.hv_last_error().decode()


def hv_set_stream(stream) -> None:
    """stream: a torch.cuda.Stream, a raw hipStream_t address, or None."""
    ptr = getattr(stream, "cuda_stream", stream)
    _check(lib.hv_set_stream(ptr))


def hv_index_build(objects, kind: int, n: int | None = None) -> int:
    """objects: float64 device tensor (n,2) or (n,4), or a device address
    (then n is required).  Returns the opaque index handle."""
    if n is None:
        n = int(objects.shape[0])
    if hasattr(objects, "dtype") and n > 0:
        if str(objects.dtype) != "torch.float64" or not objects.is_contiguous():
            raise HvError(HV_EINVAL, "objects must be a contiguous float64 tensor")
    _sync_stream()
    h = lib.hv_index_build(_device_ptr(objects), int(kind), int(n))
    if not h:
        raise HvError(HV_EINVAL, hv_last_error())
    return h


def hv_render_tiles(index: int, tiles, style, out_masks) -> None:
    """tiles: (n,3)/(n,4) ints; style: r in px (float) or hv_style;
    out_masks: uint8 device tensor of n*8192 bytes (or a device address)."""
    t = tiles_array(tiles)
    st = style if isinstance(style, hv_style) else hv_style(float(style))
    _sync_stream()
    _check(lib.hv_render_tiles(index, t.ctypes.data_as(_P), t.shape[0], ctypes.byref(st),
                               _device_ptr(out_masks)))


def hv_render_tiles_ex(index: int, tiles, style, out_masks, launch: hv_launch | dict | None) -> None:
    t = tiles_array(tiles)
    st = style if isinstance(style, hv_style) else hv_style(float(style))
    if isinstance(launch, dict):
        launch = hv_launch(**launch)
    _sync_stream()
    _check(lib.hv_render_tiles_ex(index, t.ctypes.data_as(_P), t.shape[0], ctypes.byref(st),
                                  _device_ptr(out_masks), ctypes.byref(launch) if launch else None))


def hv_free(index: int | None) -> None:
    lib.hv_free(index)


def hv_index_info(index: int) -> dict:
    info = hv_info()
    _check(lib.hv_index_info(index, ctypes.byref(info)))
    d = {k: getattr(info, k) for k, _ in hv_info._fields_ if k not in ("pad", "root")}
    d["root"] = list(info.root)
    return d


def hv_index_read(index: int, what: int, level: int = 0) -> np.ndarray:
    info = hv_index_info(index)
    w = 2 if info["kind"] == HV_POINTS else 4
    if what == HV_READ_ORDER:
        out = np.empty(info["n"], dtype=np.uint32)
    elif what == HV_READ_OBJECTS:
        out = np.empty((info["n"], w), dtype=np.float64)
    elif what == HV_READ_NODES:
        # the level's node count is implicit in the tree shape
        cnt = -(-info["n"] // info["leaf_size"])
        for _ in range(level):
            cnt = -(-cnt // info["fanout"])
        out = np.empty((cnt, 4), dtype=np.float64)
    else:
        raise HvError(HV_EINVAL, "unknown array")
    _check(lib.hv_index_read(index, what, level, out.ctypes.data_as(_P), out.nbytes))
    return out


def requests(indexes, tiles, r) -> np.ndarray:
    """Builds an hv_request array: indexes (handles, one per request or one
    for all), tiles (n,3) z,x,y, r (scalar or n)."""
    t = np.asarray(tiles, dtype=np.int64).reshape(-1, 3)
    n = t.shape[0]
    out = np.zeros(n, dtype=REQUEST_DTYPE)
    out["index"] = np.broadcast_to(np.asarray(indexes, dtype=np.uint64), (n,))
    out["z"], out["x"], out["y"] = t[:, 0], t[:, 1], t[:, 2]
    out["r_px"] = np.broadcast_to(np.asarray(r, dtype=np.float64), (n,))
    return out


def _reqs(reqs) -> np.ndarray:
    r = np.ascontiguousarray(reqs)
    if r.dtype != REQUEST_DTYPE:
        raise HvError(HV_EINVAL, "requests must be built with hv.requests()")
    return r


def _launch(launch):
    if launch is None:
        return None
    return launch if isinstance(launch, hv_launch) else hv_launch(**launch)


def hv_render_batch(reqs, out_masks, launch=None) -> None:
    r = _reqs(reqs)
    L = _launch(launch)
    _sync_stream()
    _check(lib.hv_render_batch(r.ctypes.data_as(_P), r.shape[0], _device_ptr(out_masks),
                               ctypes.byref(L) if L else None))


def hv_estimate_bytes(index: int, tile, r_px: float | None) -> int:
    """Device bytes one request of (index, tile (z, x, y), r) holds in a batch."""
    z, x, y = (int(v) for v in tile[:3])
    t = hv_tile(z, x, y, 0)
    st = hv_style(float(r_px)) if r_px is not None else None
    return _check(lib.hv_estimate_bytes(index, ctypes.byref(t), ctypes.byref(st) if st else None))


def hv_estimate_batch_bytes(n_requests: int, n_indexes: int) -> int:
    """Device bytes of a batch of n_requests requests over n_indexes indexes."""
    return _check(lib.hv_estimate_batch_bytes(int(n_requests), int(n_indexes)))


def hv_render_batch_noalloc(reqs, out_masks, launch=None) -> None:
    """hv_render_batch on the library's static device scratch (no allocation);
    at most HV_NOALLOC_MAX_REQUESTS requests over HV_NOALLOC_MAX_INDEXES indexes."""
    r = _reqs(reqs)
    L = _launch(launch)
    _sync_stream()
    _check(lib.hv_render_batch_noalloc(r.ctypes.data_as(_P), r.shape[0], _device_ptr(out_masks),
                                       ctypes.byref(L) if L else None))


def hv_polygon_index_build(edges, first, flags: int = 0) -> int:
    """Polygon index from device edges (torch tensor (n, 4) float64) grouped
    by polygon, first (host, npoly + 1 int64)."""
    f = np.ascontiguousarray(first, dtype=np.int64)
    n = int(f[-1]) if f.size else 0
    if hasattr(edges, "dtype") and n > 0:
        if str(edges.dtype) != "torch.float64" or not edges.is_contiguous() or tuple(edges.shape) != (n, 4):
            raise HvError(HV_EINVAL, "edges must be a contiguous float64 tensor of shape (first[-1], 4)")
    h = lib.hv_polygon_index_build(_device_ptr(edges), int(n), f.ctypes.data_as(_P) if f.size else None,
                                   int(f.size - 1) if f.size else 0, int(flags))
    if not h:
        raise HvError(HV_EINVAL, hv_last_error())
    return h


def hv_render_fill(index: int, tiles, out_masks, launch=None) -> None:
    t = tiles_array(tiles)
    L = _launch(launch)
    _sync_stream()
    _check(lib.hv_render_fill(index, t.ctypes.data_as(_P), t.shape[0], _device_ptr(out_masks),
                              ctypes.byref(L) if L else None))


def hv_time_aa(reqs, out_values, launch=None, reps: int = 10):
    """Mean (frontier kernel ms, query kernel ms) over reps renders of the
    batch with hv_render_batch_aa, from HIP events on the current stream;
    with child-tile requests each is the sum over the two sub-batches."""
    r = _reqs(reqs)
    L = _launch(launch)
    ms = (ctypes.c_double * 2)()
    _sync_stream()
    _check(lib.hv_time_aa(r.ctypes.data_as(_P), r.shape[0], _device_ptr(out_values),
                          ctypes.byref(L) if L else None, int(reps), ms))
    return ms[0], ms[1]


def hv_time_fill(index: int, tiles, out_masks, launch=None, reps: int = 10):
    """Mean (frontier kernel ms, fill kernel ms) over reps fills of the tiles,
    from HIP events on the current stream."""
    t = tiles_array(tiles)
    L = _launch(launch)
    ms = (ctypes.c_double * 2)()
    _sync_stream()
    _check(lib.hv_time_fill(index, t.ctypes.data_as(_P), t.shape[0], _device_ptr(out_masks),
                            ctypes.byref(L) if L else None, int(reps), ms))
    return ms[0], ms[1]


def hv_render_batch_aa(reqs, out_values, launch=None) -> None:
    """Anti-aliased values 0-4 (one byte per pixel, HV_AA_BYTES per request)
    into the device buffer out_values."""
    r = _reqs(reqs)
    L = _launch(launch)
    _sync_stream()
    _check(lib.hv_render_batch_aa(r.ctypes.data_as(_P), r.shape[0], _device_ptr(out_values),
                                  ctypes.byref(L) if L else None))


def hv_batcher_create(max_requests: int, max_indexes: int = 8, max_levels: int = 10, launch=None) -> int:
    L = _launch(launch)
    h = lib.hv_batcher_create(int(max_requests), int(max_indexes), int(max_levels), ctypes.byref(L) if L else None)
    if not h:
        raise HvError(HV_EINVAL, hv_last_error())
    return h


def hv_batcher_run(batcher: int, reqs, out_masks) -> None:
    r = _reqs(reqs)
    _sync_stream()
    _check(lib.hv_batcher_run(batcher, r.ctypes.data_as(_P), r.shape[0], _device_ptr(out_masks)))


def hv_batcher_latency(batcher: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _check(lib.hv_batcher_latency(batcher, out.ctypes.data_as(_P), int(n)))
    return out


def hv_batcher_free(batcher: int | None) -> None:
    lib.hv_batcher_free(batcher)


def _launch_dict(L: hv_launch) -> dict:
    return {k: getattr(L, k) for k, _ in hv_launch._fields_}


def hv_autotune(reqs, scratch_masks):
    """Returns (best launch as a dict, its time per launch in ms)."""
    r = _reqs(reqs)
    best = hv_launch()
    ms = ctypes.c_double(0.0)
    _sync_stream()
    _check(lib.hv_autotune(r.ctypes.data_as(_P), r.shape[0], _device_ptr(scratch_masks), ctypes.byref(best),
                           ctypes.byref(ms)))
    return _launch_dict(best), ms.value


def hv_tuned_launch(reqs):
    r = _reqs(reqs)
    L = hv_launch()
    rc = lib.hv_tuned_launch(r.ctypes.data_as(_P), r.shape[0], ctypes.byref(L))
    return _launch_dict(L) if rc == HV_OK else None


def hv_time_kernels(reqs, out_masks, launch=None, reps: int = 10):
    """Mean (frontier kernel ms, query kernel ms) over reps renders of the
    batch, from HIP events on the current stream."""
    r = _reqs(reqs)
    L = _launch(launch)
    ms = (ctypes.c_double * 2)()
    _sync_stream()
    _check(lib.hv_time_kernels(r.ctypes.data_as(_P), r.shape[0], _device_ptr(out_masks),
                               ctypes.byref(L) if L else None, int(reps), ms))
    return ms[0], ms[1]


# ------------------------------------------------------------ convenience
class Index:
    """Owns one index handle; frees it when collected."""

    def __init__(self, objects, kind: int):
        self.kind = kind
        self.handle = hv_index_build(objects, kind)

    def render(self, tiles, r, out=None, launch=None):
        """Returns (or fills) a uint8 device tensor (n, 8192) of masks."""
        import torch
        t = tiles_array(tiles)
        if out is None:
            out = torch.empty((t.shape[0], HV_MASK_BYTES), dtype=torch.uint8, device="cuda")
        if launch is None:
            hv_render_tiles(self.handle, t, r, out)
        else:
            hv_render_tiles_ex(self.handle, t, r, out, launch)
        return out

    def info(self) -> dict:
        return hv_index_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            hv_free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()
