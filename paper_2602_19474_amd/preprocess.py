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


class Preprocessor:
    """Workspace and outputs sized once for one image shape (bounds of
    ``pre_query``), so that repeated calls allocate nothing."""

    def __init__(self, bitmap, grid_h: float, a: float | None = None, b: float | None = None,
                 c: float | None = None):
        import torch
        if a is None and b is None and c is None:
            a, b, c = paper_thresholds(grid_h)
        if a is None or b is None or c is None:
            raise ValueError("give all three thresholds or none")
        self.bitmap, self.grid_h, self.th = bitmap, float(grid_h), (float(a), float(b), float(c))
        self.ws_bytes, self.vbound, self.tbound = pre_query(bitmap.shape[1], bitmap.shape[0], grid_h)
        dev = bitmap.device
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.verts = torch.empty((self.vbound, 2), dtype=torch.float64, device=dev)
        self.on_polyline = torch.empty((self.vbound,), dtype=torch.uint8, device=dev)
        self.tris = torch.empty((max(self.tbound, 1), 3), dtype=torch.int32, device=dev)
        self.ctx = context(dev.index)
        self.img = _image(bitmap, grid_h, 0)
        self.counts = (ctypes.c_int64 * 6)()

    def run(self, stream=None):
        """One call of sbmt_preprocess (waits for the stream); returns
        (n_vertices, n_triangles, n_snapped, n_repelled, n_inserted)."""
        a, b, c = self.th
        st = _lib.lib().sbmt_preprocess(self.ctx.handle, ctypes.byref(self.img), a, b, c, self.ws.data_ptr(),
                                        self.ws_bytes, self.verts.data_ptr(), self.on_polyline.data_ptr(),
                                        self.vbound, self.tris.data_ptr(), self.tbound, self.counts,
                                        _stream_ptr(stream))
        _lib.check(st, "sbmt_preprocess")
        return tuple(int(x) for x in self.counts[:5])


@dataclass
class PreMesh:
    verts: object     # float64 [V, 2]: the grid vertices a triangle uses (ids 0 .. n_grid_vertices-1), then the new ones
    tris: object      # int32 [T, 3], positive signed area
    codes: object     # uint8 [T]: 0 grid triangle kept whole, 1 piece of a cut one
    n_grid_vertices: int
    n_snapped: int
    n_repelled: int
    n_inserted: int
    n_cut: int


def preprocess_mesh(bitmap, grid_h: float, a: float | None = None, b: float | None = None, c: float | None = None,
                    stream=None, ctx=None) -> PreMesh:
    """The mesh of Alg. 3 on a uint8 CUDA tensor [H, W]: the preprocessed grid
    retriangulated against the polyline (waits for the stream; a first call
    sizes the outputs, a second fills them)."""
    import torch
    if a is None and b is None and c is None:
        a, b, c = paper_thresholds(grid_h)
    if a is None or b is None or c is None:
        raise ValueError("give all three thresholds or none")
    ctx = ctx or context(bitmap.device.index)
    img = _image(bitmap, grid_h, 0)
    L = _lib.lib()
    ws_bytes, gbound = ctypes.c_size_t(), ctypes.c_int64()
    _lib.check(L.sbmt_pre_mesh_query(ctypes.byref(img), ctypes.byref(ws_bytes), ctypes.byref(gbound)),
               "sbmt_pre_mesh_query")
    dev = bitmap.device
    ws = torch.empty(int(ws_bytes.value), dtype=torch.uint8, device=dev)
    counts = (ctypes.c_int64 * 8)()
    nv, nt = 0, 0
    for attempt in range(2):
        verts = torch.empty((max(nv, 1), 2), dtype=torch.float64, device=dev)
        tris = torch.empty((max(nt, 1), 3), dtype=torch.int32, device=dev)
        codes = torch.empty((max(nt, 1),), dtype=torch.uint8, device=dev)
        st = L.sbmt_preprocess_mesh(ctx.handle, ctypes.byref(img), float(a), float(b), float(c), ws.data_ptr(),
                                    int(ws_bytes.value), verts.data_ptr(), verts.shape[0], tris.data_ptr(),
                                    codes.data_ptr(), nt, counts, _stream_ptr(stream))
        if st == 0:
            break
        if st != -7 or attempt == 1:
            _lib.check(st, "sbmt_preprocess_mesh")
        nv, nt = max(int(counts[0]), nv), int(counts[1])
    return PreMesh(verts[:int(counts[0])], tris[:int(counts[1])], codes[:int(counts[1])], int(counts[6]),
                   int(counts[2]), int(counts[3]), int(counts[4]), int(counts[7]))


class MeshPreprocessor:
    """sbmt_preprocess_mesh with workspace and outputs kept across calls (sized
    by a first call on this image)."""

    def __init__(self, bitmap, grid_h: float, a: float | None = None, b: float | None = None,
                 c: float | None = None):
        import torch
        if a is None and b is None and c is None:
            a, b, c = paper_thresholds(grid_h)
        self.th = (float(a), float(b), float(c))
        self.ctx = context(bitmap.device.index)
        self.img = _image(bitmap, grid_h, 0)
        L = _lib.lib()
        ws_bytes, gbound = ctypes.c_size_t(), ctypes.c_int64()
        _lib.check(L.sbmt_pre_mesh_query(ctypes.byref(self.img), ctypes.byref(ws_bytes), ctypes.byref(gbound)),
                   "sbmt_pre_mesh_query")
        self.ws_bytes = int(ws_bytes.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=bitmap.device)
        self.counts = (ctypes.c_int64 * 8)()
        m = preprocess_mesh(bitmap, grid_h, *self.th, ctx=self.ctx)
        dev = bitmap.device
        self.verts = torch.empty((max(m.verts.shape[0], 1), 2), dtype=torch.float64, device=dev)
        self.tris = torch.empty((max(m.tris.shape[0], 1), 3), dtype=torch.int32, device=dev)
        self.codes = torch.empty((max(m.tris.shape[0], 1),), dtype=torch.uint8, device=dev)
        del m

    def run(self, stream=None):
        """One call (waits for the stream); returns (n_vertices, n_triangles, n_grid_vertices, n_cut)."""
        a, b, c = self.th
        st = _lib.lib().sbmt_preprocess_mesh(self.ctx.handle, ctypes.byref(self.img), a, b, c, self.ws.data_ptr(),
                                             self.ws_bytes, self.verts.data_ptr(), self.verts.shape[0],
                                             self.tris.data_ptr(), self.codes.data_ptr(), self.tris.shape[0],
                                             self.counts, _stream_ptr(stream))
        _lib.check(st, "sbmt_preprocess_mesh")
        return int(self.counts[0]), int(self.counts[1]), int(self.counts[6]), int(self.counts[7])
