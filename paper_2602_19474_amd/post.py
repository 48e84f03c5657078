"""Consumers of a mesh on the GPU: field sampling and quality statistics.

Thin front end of the entry points declared in ``include/sbmt_post.h``; the
work runs in the HIP kernels of ``libsbmt.so``.

    vals, tri_vals = sample_field(field_f32_on_gpu, verts, tris)
    stats = mesh_quality(verts, tris)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from . import _stream_ptr, context


def _torch():
    import torch
    return torch


def sample_field(field, verts, tris=None, stream=None):
    """Bilinear values of an FP32 CUDA field [H, W] at the vertices (FP64 [V]).

    With ``tris``, also the per-triangle means of the linear interpolant
    (FP64 [T]; NaN for a triangle with an index out of range).
    """
    torch = _torch()
    if field.dtype != torch.float32 or field.dim() != 2 or field.stride(1) != 1:
        raise ValueError("field must be a float32 [H, W] tensor with unit column stride")
    ctx = context(verts.device.index)
    nv = int(verts.shape[0])
    vv = torch.empty((nv,), dtype=torch.float64, device=verts.device)
    nt = int(tris.shape[0]) if tris is not None else 0
    tv = torch.empty((nt,), dtype=torch.float64, device=verts.device) if tris is not None else None
    f = _lib.Field(field.data_ptr() if field.numel() else None, int(field.shape[1]), int(field.shape[0]),
                   int(field.stride(0)))
    _lib.check(_lib.lib().sbmt_sample_field(
        ctx.handle, ctypes.byref(f), verts.data_ptr() if nv else None, nv,
        tris.data_ptr() if nt else None, nt, vv.data_ptr() if nv else None,
        tv.data_ptr() if (tv is not None and nt) else None, _stream_ptr(stream)), "sbmt_sample_field")
    return (vv, tv) if tris is not None else vv


def quality_workspace_bytes(n_triangles: int) -> int:
    b = ctypes.c_size_t()
    _lib.check(_lib.lib().sbmt_quality_workspace(int(n_triangles), ctypes.byref(b)), "sbmt_quality_workspace")
    return int(b.value)


def _as_dict(q: _lib.Quality) -> dict:
    d = {n: getattr(q, n) for n, _ in _lib.Quality._fields_ if n != "angle_hist"}
    d["angle_hist"] = np.array(q.angle_hist[:], np.int64)
    return d


def mesh_quality(verts, tris, ws=None, stream=None, allow_invalid: bool = False) -> dict:
    """Quality statistics of a mesh on the GPU (waits for the stream)."""
    torch = _torch()
    ctx = context(verts.device.index)
    nv, nt = int(verts.shape[0]), int(tris.shape[0])
    need = quality_workspace_bytes(nt)
    if ws is None or ws.numel() < need:
        ws = torch.empty((need,), dtype=torch.uint8, device=verts.device)
    q = _lib.Quality()
    st = _lib.lib().sbmt_mesh_quality(ctx.handle, verts.data_ptr() if nv else None, nv,
                                      tris.data_ptr() if nt else None, nt, ws.data_ptr(), ws.numel(),
                                      ctypes.byref(q), _stream_ptr(stream))
    if not (allow_invalid and st == -1 and q.n_invalid):
        _lib.check(st, "sbmt_mesh_quality")
    return _as_dict(q)


def mesh_quality_async(verts, tris, ws, out_dev, stream=None):
    """Enqueue the statistics into ``out_dev`` (a uint8 CUDA tensor of at least
    ``ctypes.sizeof(Quality)`` bytes); read it with :func:`quality_from_bytes`."""
    ctx = context(verts.device.index)
    nv, nt = int(verts.shape[0]), int(tris.shape[0])
    _lib.check(_lib.lib().sbmt_mesh_quality_async(ctx.handle, verts.data_ptr() if nv else None, nv,
                                                  tris.data_ptr() if nt else None, nt, ws.data_ptr(), ws.numel(),
                                                  out_dev.data_ptr(), _stream_ptr(stream)),
               "sbmt_mesh_quality_async")


def quality_from_bytes(buf) -> dict:
    raw = bytes(buf.cpu().numpy().tobytes()[:ctypes.sizeof(_lib.Quality)])
    return _as_dict(_lib.Quality.from_buffer_copy(raw))
