"""Helpers for GPU tests: render through the C ABI and compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np

from helpers import unpack_masks


def log(msg: str) -> None:
    """Names the case before each GPU step, flushed, so a failing run says where it was."""
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def build(hv, torch, objs: np.ndarray, kind: int):
    t = torch.from_numpy(np.ascontiguousarray(objs, dtype=np.float64)).cuda()
    h = hv.hv_index_build(t, kind)
    del t
    return h


def render(hv, torch, h, tiles, r, launch=None, one_per_call=False):
    tiles = np.asarray(tiles).reshape(-1, 3)
    out = torch.empty((max(1, tiles.shape[0]), 8192), dtype=torch.uint8, device="cuda")
    out.fill_(0xA5)   # masks must be fully overwritten
    if one_per_call:
        for k in range(tiles.shape[0]):
            hv.hv_render_tiles_ex(h, tiles[k:k + 1], r, out[k], launch)
    elif launch is not None:
        hv.hv_render_tiles_ex(h, tiles, r, out, launch)
    else:
        hv.hv_render_tiles(h, tiles, r, out)
    torch.cuda.synchronize()
    return unpack_masks(out[:tiles.shape[0]].cpu().numpy())


def render_mixed(hv, torch, h, tiles, rs):
    """Requests with their own radii: one call per distinct r."""
    tiles = np.asarray(tiles).reshape(-1, 3)
    rs = np.asarray(rs, dtype=np.float64)
    bits = np.zeros((tiles.shape[0], 256, 256), dtype=np.uint8)
    for r in np.unique(rs):
        sel = np.nonzero(rs == r)[0]
        bits[sel] = render(hv, torch, h, tiles[sel], float(r))
    return bits
