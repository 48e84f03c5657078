"""MI355X-native Structured Bitmap-to-Mesh Triangulation (SBMT, arXiv 2602.19474).

Python front end of ``libsbmt.so``.  PyTorch provides device memory and
streams; every step of the meshing path (boundary extraction, exact
classification, canonical class, template lookup, emission) runs in the HIP
kernels behind the C ABI of ``include/sbmt.h``.

    verts, tris, codes = mesh_from_bitmap(bitmap_u8_on_gpu, grid_h)

``verts`` float64 [V, 2] (x, y) with pixel (r, c) centred at (c, r); ``tris``
int32 [T, 3] with positive signed area; ``codes`` uint8 [T]: 0 = uncut base
triangle, 1..num_classes() = canonical class of the cut parent triangle, bit 7
= background side (only with ``both_sides=True``).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _lib
from ._lib import BOTH_SIDES, NOALLOC_SCRATCH_BYTES, SIZE_WORDS, SbmtError

__all__ = ["Context", "mesh_from_bitmap", "plan", "run", "mesh_async", "query", "num_classes", "class_code",
           "BOTH_SIDES", "SbmtError", "SUPPORTED_GRID_H"]

SUPPORTED_GRID_H = (1, 2, 3, 4, 5, 6)


def _torch():
    import torch
    return torch


@dataclass
class Layout:
    stride_s: int
    coarse_w: int
    coarse_h: int
    grid_rows: int
    grid_cols: int
    workspace_bytes: int


@dataclass
class Sizes:
    n_vertices: int
    n_triangles: int
    n_cut: int
    n_segments: int = 0


def _image(bitmap, grid_h: float, flags: int) -> _lib.Image:
    torch = _torch()
    if bitmap.dtype != torch.uint8 or bitmap.dim() != 2:
        raise ValueError("bitmap must be a 2-D uint8 tensor")
    if bitmap.numel() and bitmap.shape[1] > 1 and bitmap.stride(1) != 1:
        raise ValueError("bitmap rows must be contiguous")
    H, W = bitmap.shape
    # a size-1 row dimension may carry any stride (numpy's a[None, :] has 0)
    stride = int(bitmap.stride(0)) if (bitmap.numel() and H > 1) else int(W)
    return _lib.Image(bitmap.data_ptr() if bitmap.numel() else None, int(W), int(H), stride, float(grid_h),
                      int(flags))


def query(width: int, height: int, grid_h: float, flags: int = 0) -> Layout:
    """Grid geometry and workspace size of an image (host only, no GPU work)."""
    img = _lib.Image(None, int(width), int(height), int(width), float(grid_h), int(flags))
    out = _lib.Layout()
    _lib.check(_lib.lib().sbmt_query(ctypes.byref(img), ctypes.byref(out)), "sbmt_query")
    return Layout(out.stride_s, out.coarse_w, out.coarse_h, out.grid_rows, out.grid_cols, out.workspace_bytes)


class Context:
    """One library context per device (owns a small pinned host buffer)."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().sbmt_create(self.device, ctypes.byref(h)), "sbmt_create")
        self.handle = h

    def close(self):
        if self.handle:
            _lib.lib().sbmt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict = {}


def context(device: int | None = None) -> Context:
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        _contexts[dev] = Context(dev)
    return _contexts[dev]


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace(bitmap, grid_h: float, flags: int = 0):
    torch = _torch()
    lay = query(bitmap.shape[1], bitmap.shape[0], grid_h, flags)
    return torch.empty(lay.workspace_bytes, dtype=torch.uint8, device=bitmap.device)


def plan(bitmap, grid_h: float, ws, flags: int = 0, stream=None, ctx: Context | None = None) -> Sizes:
    """Classify and count (synchronises the stream to return the sizes)."""
    ctx = ctx or context(bitmap.device.index)
    img = _image(bitmap, grid_h, flags)
    out = _lib.Sizes()
    _lib.check(_lib.lib().sbmt_plan(ctx.handle, ctypes.byref(img), ws.data_ptr(), ws.numel(), ctypes.byref(out),
                                    _stream_ptr(stream)), "sbmt_plan")
    return Sizes(out.n_vertices, out.n_triangles, out.n_cut, out.n_segments)


def run(bitmap, grid_h: float, ws, verts, tris, codes, flags: int = 0, stream=None, ctx: Context | None = None):
    """Emit the mesh planned in ``ws`` into preallocated outputs (asynchronous)."""
    ctx = ctx or context(bitmap.device.index)
    img = _image(bitmap, grid_h, flags)
    _lib.check(_lib.lib().sbmt_run(ctx.handle, ctypes.byref(img), ws.data_ptr(), ws.numel(),
                                   verts.data_ptr() if verts.numel() else None,
                                   tris.data_ptr() if tris.numel() else None,
                                   codes.data_ptr() if codes.numel() else None, _stream_ptr(stream)), "sbmt_run")


def mesh_from_bitmap(bitmap, grid_h: float, both_sides: bool = False, stream=None, return_sizes: bool = False):
    """Mesh a uint8 CUDA tensor [H, W]: plan -> allocate -> run on the current stream.

    Returns (verts, tris, codes), and the planned ``Sizes`` as a fourth item
    when ``return_sizes``."""
    torch = _torch()
    flags = BOTH_SIDES if both_sides else 0
    ws = workspace(bitmap, grid_h, flags)
    sz = plan(bitmap, grid_h, ws, flags, stream)
    dev = bitmap.device
    verts = torch.empty((sz.n_vertices, 2), dtype=torch.float64, device=dev)
    tris = torch.empty((sz.n_triangles, 3), dtype=torch.int32, device=dev)
    codes = torch.empty((sz.n_triangles,), dtype=torch.uint8, device=dev)
    run(bitmap, grid_h, ws, verts, tris, codes, flags, stream)
    return (verts, tris, codes, sz) if return_sizes else (verts, tris, codes)


def mesh_async(bitmap, grid_h: float, ws, verts, tris, codes, sizes_dev, flags: int = 0, stream=None,
               ctx: Context | None = None):
    """Plan and emit without a host round trip into outputs of given capacity.

    ``sizes_dev`` is an int64 CUDA tensor of ``SIZE_WORDS`` (5) entries that receives
    (n_vertices, n_triangles, n_cut, status, n_segments); status -7 means the mesh did
    not fit.
    """
    ctx = ctx or context(bitmap.device.index)
    img = _image(bitmap, grid_h, flags)
    _lib.check(_lib.lib().sbmt_mesh_async(ctx.handle, ctypes.byref(img), ws.data_ptr(), ws.numel(),
                                          verts.data_ptr(), int(verts.shape[0]), tris.data_ptr(), codes.data_ptr(),
                                          int(tris.shape[0]), sizes_dev.data_ptr(), _stream_ptr(stream)),
               "sbmt_mesh_async")


def mesh_noalloc(bitmap, grid_h: float, verts, tris, codes, sizes_dev, flags: int = 0, stream=None,
                 ctx: Context | None = None):
    """``mesh_async`` on the library's own scratch array: no workspace argument and no
    device allocation (for callers that cannot allocate).  Images whose workspace
    exceeds ``NOALLOC_SCRATCH_BYTES`` raise (status -4); calls on one GPU must not
    overlap (they share the array)."""
    ctx = ctx or context(bitmap.device.index)
    img = _image(bitmap, grid_h, flags)
    _lib.check(_lib.lib().sbmt_mesh_noalloc(ctx.handle, ctypes.byref(img), verts.data_ptr(), int(verts.shape[0]),
                                            tris.data_ptr(), codes.data_ptr(), int(tris.shape[0]),
                                            sizes_dev.data_ptr(), _stream_ptr(stream)), "sbmt_mesh_noalloc")


def num_classes() -> int:
    return int(_lib.lib().sbmt_num_classes())


def class_code(class_id: int) -> int:
    return int(_lib.lib().sbmt_class_code(int(class_id)))
