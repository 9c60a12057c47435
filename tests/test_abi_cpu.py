"""The C-ABI library loads, exports every symbol include/hv.h declares, and
rejects bad arguments on the host before any device call (no GPU needed)."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hv.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hv_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def hv():
    from paper_2005_12489_amd import hv as m
    return m


def test_every_declared_symbol_is_exported(hv):
    names = _declared()
    assert "hv_index_build" in names and "hv_render_tiles" in names and "hv_free" in names
    out = subprocess.run(["nm", "-D", "--defined-only", hv.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (hv_[a-z_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # and no internal helper leaks out with C linkage
    c_names = set(re.findall(r"\bT ([A-Za-z][A-Za-z0-9_]*)$", out, re.M))
    assert c_names == set(names), sorted(c_names ^ set(names))
    assert set(hv.SYMBOLS) == set(names), sorted(set(names) ^ set(hv.SYMBOLS))


def test_build_rejects_bad_arguments(hv):
    for args, msg in [((None, 7, 3), "unknown kind"), ((None, 0x200, 3), "unknown kind"),
                      ((None, 0, 3), "NULL"), ((None, 0, -1), "n outside"),
                      ((None, 1, 3_000_000_000), "n outside")]:
        with pytest.raises(hv.HvError, match=msg) as e:
            hv.hv_index_build(*args)
        assert e.value.code == hv.HV_EINVAL
    host = np.zeros((4, 2))
    with pytest.raises(hv.HvError, match="device memory"):
        hv.hv_index_build(host.ctypes.data, hv.HV_POINTS, 4)


def test_empty_index_needs_no_device(hv):
    h = hv.hv_index_build(None, hv.HV_SEGMENTS, 0)
    info = hv.hv_index_info(h)
    assert info["n"] == 0 and info["levels"] == 0 and info["device_bytes"] == 0
    hv.hv_render_tiles(h, np.zeros((0, 3)), 1.0, 0)         # nothing to do
    hv.hv_free(h)
    hv.hv_free(None)


@pytest.mark.parametrize("tile,r,msg", [
    ((23, 0, 0), 1.0, "zoom"), ((-1, 0, 0), 1.0, "zoom"), ((3, 8, 0), 1.0, "x or y"),
    ((3, 0, -1), 1.0, "x or y"), ((22, 1 << 22, 0), 1.0, "x or y"), ((3, 1, 1), 0.0, "r_px"),
    ((3, 1, 1), -1.0, "r_px"), ((3, 1, 1), float("nan"), "r_px"), ((3, 1, 1), float("inf"), "r_px"),
    ((3, 1, 1), 64.5, "r_px")])
def test_render_rejects_bad_requests(hv, tile, r, msg):
    h = hv.hv_index_build(None, hv.HV_POINTS, 0)
    try:
        with pytest.raises(hv.HvError, match=msg):
            hv.hv_render_tiles(h, [tile], r, 1)              # a non-NULL dummy, never touched
    finally:
        hv.hv_free(h)


def test_render_rejects_host_output_and_bad_shapes(hv):
    h = hv.hv_index_build(None, hv.HV_POINTS, 0)
    buf = np.zeros(8192, np.uint8)
    try:
        with pytest.raises(hv.HvError, match="device memory"):
            hv.hv_render_tiles(h, [(3, 1, 1)], 1.0, buf.ctypes.data)
        for bad in (dict(block=12), dict(cand_cap=32), dict(cand_cap=5000), dict(waves_per_wg=3),
                    dict(waves_per_wg=8), dict(grid_wgs=-1), dict(grid_wgs=1 << 21), dict(region=16),
                    dict(region=64, waves_per_wg=4, cand_cap=128), dict(region=32, objs_per_lane=3),
                    dict(region=32, waves_per_wg=2, objs_per_lane=4, cand_cap=64), dict(cull_nodes=257),
                    dict(cull_nodes=-1)):
            with pytest.raises(hv.HvError, match="launch"):
                hv.hv_render_tiles_ex(h, [(3, 1, 1)], 1.0, buf.ctypes.data, bad)
        with pytest.raises(hv.HvError, match="NULL"):
            hv.hv_render_tiles(h, [(3, 1, 1)], 1.0, 0)
        assert (buf == 0).all()
    finally:
        hv.hv_free(h)


def test_batch_validation_before_any_device_call(hv):
    h = hv.hv_index_build(None, hv.HV_POINTS, 0)
    try:
        for reqs, msg in [(hv.requests(0, [(3, 1, 1)], 1.0), "index is NULL"),
                          (hv.requests(h, [(3, 1, 1), (23, 0, 0)], 1.0), "request 1: zoom"),
                          (hv.requests(h, [(3, 8, 1)], 1.0), "x or y"),
                          (hv.requests(h, [(3, 1, 1)], 0.0), "r_px")]:
            with pytest.raises(hv.HvError, match=msg):
                hv.hv_render_batch(reqs, 1)
        with pytest.raises(hv.HvError, match="NULL"):
            hv.hv_render_batch(hv.requests(h, [(3, 1, 1)], 1.0), 0)
        hv.hv_render_batch(hv.requests(h, np.zeros((0, 3)), 1.0), 0)       # empty batch
        for args, msg in [((0,), "max_requests"), ((10, 0), "max_indexes"), ((10, 1, 0), "max_levels"),
                          ((10, 1, 17), "max_levels")]:
            with pytest.raises(hv.HvError, match=msg):
                hv.hv_batcher_create(*args)
        with pytest.raises(hv.HvError, match="empty"):
            hv.hv_autotune(hv.requests(h, np.zeros((0, 3)), 1.0), 1)
        assert hv.hv_tuned_launch(hv.requests(h, [(3, 1, 1)], 1.0)) is None
        for reqs, msg in [(hv.requests(h, [(23, 0, 0)], 1.0), "zoom"),
                          (hv.requests(h, [(3, 8, 1)], 1.0), "x or y"),
                          (hv.requests(h, [(3, 1, 1)], 65.0), "r_px")]:
            with pytest.raises(hv.HvError, match=msg):
                hv.hv_render_batch_aa(reqs, 1)
        with pytest.raises(hv.HvError, match="NULL"):
            hv.hv_render_batch_aa(hv.requests(h, [(3, 1, 1)], 1.0), 0)
        for split in (-3, 63):
            with pytest.raises(hv.HvError, match="aa_split"):
                hv.hv_render_batch_aa(hv.requests(h, [(3, 1, 1)], 1.0), 1, {"aa_split": split})
        hv.hv_render_batch_aa(hv.requests(h, np.zeros((0, 3)), 1.0), 0)     # empty batch
        for reqs, reps, msg in [(hv.requests(h, np.zeros((0, 3)), 1.0), 1, "empty"),
                                (hv.requests(h, [(3, 1, 1)], 1.0), 0, "reps"),
                                (hv.requests(h, [(3, 1, 1)], 1.0), 100001, "reps"),
                                (hv.requests(h, [(3, 1, 1)], 0.0), 1, "r_px")]:
            with pytest.raises(hv.HvError, match=msg):
                hv.hv_time_kernels(reqs, 1, reps=reps)
            with pytest.raises(hv.HvError, match=msg):
                hv.hv_time_aa(reqs, 1, reps=reps)
        # fill timing: its own checks, then hv_render_fill's
        for index, tiles, reps, msg in [(0, [(3, 1, 1)], 0, "reps"), (0, [(3, 1, 1)], 100001, "reps"),
                                        (0, np.zeros((0, 3)), 1, "empty"), (0, [(3, 1, 1)], 1, "index is NULL"),
                                        (h, [(3, 1, 1)], 1, "polygon index")]:
            with pytest.raises(hv.HvError, match=msg):
                hv.hv_time_fill(index, tiles, 1, reps=reps)
    finally:
        hv.hv_free(h)


def test_polygon_index_validation_before_any_device_call(hv):
    bad = [([1, 4], "first\\[0\\]"), ([0, 2], "npoly outside"), ([0, 2, 7], "3 edges"),
           ([0, 3, 2, 9], "3 edges"), ([0, 3, 6], "device memory")]
    for first, msg in bad:
        with pytest.raises(hv.HvError, match=msg):
            hv.hv_polygon_index_build(1, first)
    with pytest.raises(hv.HvError, match="flags"):
        hv.hv_polygon_index_build(1, [0, 3], flags=2)
    with pytest.raises(hv.HvError, match="NULL"):
        hv.hv_polygon_index_build(None, [0, 3])
    host = np.zeros((3, 4))
    with pytest.raises(hv.HvError, match="device memory"):
        hv.hv_polygon_index_build(host.ctypes.data, [0, 3])
    e = hv.hv_polygon_index_build(None, [0])            # no polygons: an empty index, no device memory
    try:
        info = hv.hv_index_info(e)
        assert info["kind"] == hv.HV_POLYGONS and info["n"] == 0
        with pytest.raises(hv.HvError, match="hv_render_fill"):
            hv.hv_render_tiles(e, [(0, 0, 0)], 1.0, 1)
        with pytest.raises(hv.HvError, match="hv_render_fill"):
            hv.hv_render_batch(hv.requests(e, [(0, 0, 0)], 1.0), 1)
        with pytest.raises(hv.HvError, match="region"):
            hv.hv_render_fill(e, [(0, 0, 0)], 1, dict(region=0, block=16))
        with pytest.raises(hv.HvError, match="zoom"):
            hv.hv_render_fill(e, [(23, 0, 0)], 1)
        hv.hv_render_fill(e, np.zeros((0, 3)), 0)      # nothing to render
    finally:
        hv.hv_free(e)
    p = hv.hv_index_build(None, hv.HV_POINTS, 0)
    try:
        with pytest.raises(hv.HvError, match="polygon index"):
            hv.hv_render_fill(p, [(0, 0, 0)], 1)
    finally:
        hv.hv_free(p)


C_PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "hv.h"

int main(void) {
    /* an empty index needs no device; bad requests fail on the host */
    hv_index *ix = hv_index_build(NULL, HV_POINTS, 0);
    if (!ix) { printf("build failed: %s\n", hv_last_error()); return 1; }
    hv_info info;
    if (hv_index_info(ix, &info) != HV_OK || info.n != 0) return 2;
    hv_tile bad = {23, 0, 0, 0};
    hv_style st = {1.0};
    if (hv_render_tiles(ix, &bad, 1, &st, NULL) != HV_EINVAL) return 3;
    if (strlen(hv_last_error()) == 0) return 4;
    hv_launch L;
    memset(&L, 0, sizeof L);
    L.cull_nodes = 300;
    if (hv_render_tiles_ex(ix, &bad, 0, &st, NULL, &L) != HV_EINVAL) return 5;
    hv_free(ix);
    printf("c-abi ok\n");
    return 0;
}
"""


def test_header_compiles_as_c99_and_links(hv, tmp_path):
    """include/hv.h is plain C: a C99 program compiles against it with
    -Wall -Werror, links against the library, and runs its host-only paths."""
    src = tmp_path / "abi.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "abi"
    libdir = os.path.dirname(hv.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe), f"-L{libdir}", "-l:libhv.so", f"-Wl,-rpath,{libdir}"], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and "c-abi ok" in out.stdout, (out.returncode, out.stdout, out.stderr)
