"""Geometric preprocessing of the grid (Alg. 3, Sec. 3.5) on the GPU.

Binding of ``sbmt_pre_query`` / ``sbmt_preprocess`` (include/sbmt.h):
argument marshalling only, the three steps (vertex snapping within ``a``,
repulsion to distance ``c``, edge elimination within ``b``) run in the HIP
kernels of the library.

    grid = preprocess(bitmap_u8_on_gpu, grid_h)        # paper thresholds
    grid.verts, grid.on_polyline, grid.tris, grid.n_snapped, ...
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

from . import _lib
from . import _image, _stream_ptr, context


def paper_thresholds(grid_h: float):
    """(a, b, c) = (0.26, 0.125, 0.183) * h / sqrt(0.45) (Sec. 3.3.4)."""
    u = float(grid_h) / math.sqrt(0.45)
    return 0.26 * u, 0.125 * u, 0.183 * u


@dataclass
class PreGrid:
    verts: object        # float64 [V, 2]: lattice vertex k * grid_cols + i, then the inserted ones
    on_polyline: object  # uint8 [V]
    tris: object         # int32 [T, 3], positive signed area
    n_snapped: int
    n_repelled: int
    n_inserted: int


def pre_query(width: int, height: int, grid_h: float):
    """(workspace bytes, vertex bound, triangle bound); host only."""
    img = _lib.Image(None, int(width), int(height), int(width), float(grid_h), 0)
    ws, vb, tb = ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
    _lib.check(_lib.lib().sbmt_pre_query(ctypes.byref(img), ctypes.byref(ws), ctypes.byref(vb), ctypes.byref(tb)),
               "sbmt_pre_query")
    return int(ws.value), int(vb.value), int(tb.value)


def preprocess(bitmap, grid_h: float, a: float | None = None, b: float | None = None, c: float | None = None,
               stream=None, ctx=None) -> PreGrid:
    """Preprocessed grid of a uint8 CUDA tensor [H, W] (waits for the stream).

    Thresholds default to the paper's; pass all three to override (all zero
    gives the plain lattice)."""
    import torch
    if a is None and b is None and c is None:
        a, b, c = paper_thresholds(grid_h)
    if a is None or b is None or c is None:
        raise ValueError("give all three thresholds or none")
    ctx = ctx or context(bitmap.device.index)
    img = _image(bitmap, grid_h, 0)
    ws_bytes, vbound, tbound = pre_query(bitmap.shape[1], bitmap.shape[0], grid_h)
    dev = bitmap.device
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    verts = torch.empty((vbound, 2), dtype=torch.float64, device=dev)
    onp = torch.empty((vbound,), dtype=torch.uint8, device=dev)
    tris = torch.empty((max(tbound, 0), 3), dtype=torch.int32, device=dev)
    counts = (ctypes.c_int64 * 6)()
    st = _lib.lib().sbmt_preprocess(ctx.handle, ctypes.byref(img), float(a), float(b), float(c), ws.data_ptr(),
                                    ws_bytes, verts.data_ptr() if vbound else None,
                                    onp.data_ptr() if vbound else None, vbound,
                                    tris.data_ptr() if tbound else None, tbound, counts, _stream_ptr(stream))
    _lib.check(st, "sbmt_preprocess")
    nv, nt = int(counts[0]), int(counts[1])
    return PreGrid(verts[:nv], onp[:nv], tris[:nt], int(counts[2]), int(counts[3]), int(counts[4]))
