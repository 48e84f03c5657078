"""Batched meshing: many bitmaps of different sizes and grid_h in one set of launches.

Front end of the ``sbmt_batch_*`` entry points of ``include/sbmt.h``
(argument marshalling only).  Typical uses:

    b = Batch([(bitmap0, 1), (bitmap1, 4), ...])      # uint8 CUDA tensors
    sizes = b.plan()                                   # exact sizes (one sync)
    outs = b.allocate(sizes)                           # or caller-owned views
    b.emit()                                           # asynchronous

    b = Batch(items, outputs=outs)                     # outputs known up front
    b.tune()                                           # autotuner (strategy, tile rows, grid)
    g = b.capture()                                    # hipGraph of the whole path
    g.replay()

The whole path of a bound batch (``mesh``) issues no host synchronisation and
no memset, so it can be captured in a graph and replayed; each replay
re-meshes the same bitmaps into the same outputs.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from . import _lib
from ._lib import STRATEGY_FUSED, STRATEGY_MULTI, SbmtError

__all__ = ["Batch", "Tuning", "mesh_batch", "STRATEGY_MULTI", "STRATEGY_FUSED"]


def _torch():
    import torch
    return torch


@dataclass
class Tuning:
    strategy: int = STRATEGY_MULTI
    tile_rows: int = 8
    groups_per_cu: int = 0
    record_cap: int = 0

    def c(self) -> _lib.Tuning:
        return _lib.Tuning(self.strategy, self.tile_rows, self.groups_per_cu, 0, self.record_cap)

    @staticmethod
    def of(t: _lib.Tuning) -> "Tuning":
        return Tuning(t.strategy, t.tile_rows, t.groups_per_cu, t.record_cap)


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Batch:
    """One batch object: images, workspace and (optionally) output views."""

    def __init__(self, items, outputs=None, tuning: Tuning | None = None, flags: int = 0, ctx=None, stream=None,
                 workspace=None, bind: bool = True):
        """``workspace``: optional callable bytes -> uint8 CUDA tensor (e.g. an arena
        sub-allocation); ``bind=False`` leaves binding to the caller."""
        from . import _image, context
        torch = _torch()
        self.items = [(t, float(h)) for t, h in items]
        if not self.items:
            raise ValueError("empty batch")
        dev = self.items[0][0].device
        self.ctx = ctx or context(dev.index)
        self.flags = int(flags)
        n = len(self.items)
        self._imgs = (_lib.Image * n)(*[_image(t, h, flags) for t, h in self.items])
        ws_bytes = ctypes.c_size_t()
        b = ctypes.c_void_p()
        tun = (tuning or Tuning()).c()
        _lib.check(_lib.lib().sbmt_batch_create(self.ctx.handle, self._imgs, n, ctypes.byref(tun),
                                                ctypes.byref(ws_bytes), ctypes.byref(b)), "sbmt_batch_create")
        self.handle = b
        self.n = n
        self.ws_bytes = max(int(ws_bytes.value), 1)
        self.ws = (workspace(self.ws_bytes) if workspace is not None
                   else torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev))
        self.outputs = None
        self._sizes_dev = None
        if bind:
            self.bind(outputs, stream)

    def close(self):
        if getattr(self, "handle", None):
            _lib.lib().sbmt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- binding -------------------------------------------------------------
    def bind(self, outputs=None, stream=None):
        """Upload the image table, with output views [(verts, tris, codes)] or none."""
        outs = None
        if outputs is not None:
            if len(outputs) != self.n:
                raise ValueError("one output triple per image")
            outs = (_lib.Outputs * self.n)()
            for i, (v, t, c) in enumerate(outputs):
                if v.shape[0] and (v.dtype != _torch().float64 or v.dim() != 2 or v.shape[1] != 2):
                    raise ValueError("verts must be float64 [V, 2]")
                if t.shape[0] != c.shape[0]:
                    raise ValueError("tris and codes must have the same number of rows")
                outs[i] = _lib.Outputs(v.data_ptr() if v.numel() else None, t.data_ptr() if t.numel() else None,
                                       c.data_ptr() if c.numel() else None, int(v.shape[0]), int(t.shape[0]))
        _lib.check(_lib.lib().sbmt_batch_bind(self.handle, self.ws.data_ptr(), self.ws.numel(), outs,
                                              _stream_ptr(stream)), "sbmt_batch_bind")
        self.outputs = outputs

    def allocate(self, sizes, slack: float = 0.0):
        """Allocate exact (or padded) outputs for the planned sizes and bind them."""
        torch = _torch()
        dev = self.ws.device
        outs = []
        for s in sizes:
            nv = int(s.n_vertices * (1 + slack))
            nt = int(s.n_triangles * (1 + slack))
            outs.append((torch.empty((nv, 2), dtype=torch.float64, device=dev),
                         torch.empty((nt, 3), dtype=torch.int32, device=dev),
                         torch.empty((nt,), dtype=torch.uint8, device=dev)))
        self.bind(outs)
        return outs

    # -- the path --------------------------------------------------------------
    def plan(self, stream=None):
        out = (_lib.Sizes * self.n)()
        _lib.check(_lib.lib().sbmt_batch_plan(self.handle, out, _stream_ptr(stream)), "sbmt_batch_plan")
        return list(out)

    def plan_async(self, stream=None):
        """Plan without waiting; read the sizes with host_sizes() once the stream got here."""
        _lib.check(_lib.lib().sbmt_batch_plan_async(self.handle, _stream_ptr(stream)), "sbmt_batch_plan_async")

    def host_sizes(self):
        """(sizes, statuses) copied by the last plan_async (no wait: the caller synchronises)."""
        out = (_lib.Sizes * self.n)()
        st = (ctypes.c_int64 * self.n)()
        _lib.check(_lib.lib().sbmt_batch_host_sizes(self.handle, out, st), "sbmt_batch_host_sizes")
        return list(out), list(st)

    @property
    def sizes_dev(self):
        """Device int64 [n, 5] that emit/mesh fill with (n_vertices, n_triangles, n_cut, status, n_segments)."""
        if self._sizes_dev is None:
            torch = _torch()
            self._sizes_dev = torch.zeros((self.n, _lib.SIZE_WORDS), dtype=torch.int64, device=self.ws.device)
        return self._sizes_dev

    def emit(self, stream=None, sizes: bool = True):
        ptr = self.sizes_dev.data_ptr() if sizes else None
        _lib.check(_lib.lib().sbmt_batch_emit(self.handle, ptr, _stream_ptr(stream)), "sbmt_batch_emit")

    def mesh(self, stream=None):
        """The whole path without host synchronisation (capturable)."""
        _lib.check(_lib.lib().sbmt_batch_mesh(self.handle, self.sizes_dev.data_ptr(), _stream_ptr(stream)),
                   "sbmt_batch_mesh")

    def sizes(self):
        """(n_vertices, n_triangles, n_cut, status, n_segments) per image of the last call (synchronises)."""
        _torch().cuda.synchronize(self.ws.device)
        return [tuple(int(x) for x in row) for row in self.sizes_dev.cpu().tolist()]

    # -- tuning and graphs -----------------------------------------------------
    @property
    def tuning(self) -> Tuning:
        t = _lib.Tuning()
        _lib.check(_lib.lib().sbmt_batch_get_tuning(self.handle, ctypes.byref(t)), "sbmt_batch_get_tuning")
        return Tuning.of(t)

    @tuning.setter
    def tuning(self, t: Tuning):
        c = t.c()
        _lib.check(_lib.lib().sbmt_batch_set_tuning(self.handle, ctypes.byref(c)), "sbmt_batch_set_tuning")

    def tune(self, reps: int = 3, stream=None):
        """Autotune on this batch (outputs must be bound); returns (Tuning, ms per run)."""
        if self.outputs is None:
            raise SbmtError(-1, "tune needs bound outputs")
        best = _lib.Tuning()
        ms = ctypes.c_float()
        _lib.check(_lib.lib().sbmt_batch_tune(self.handle, int(reps), ctypes.byref(best), ctypes.byref(ms),
                                              _stream_ptr(stream)), "sbmt_batch_tune")
        return Tuning.of(best), float(ms.value)

    def capture(self):
        """A CUDA/HIP graph of ``mesh`` (outputs must be bound)."""
        torch = _torch()
        if self.outputs is None:
            raise SbmtError(-1, "capture needs bound outputs")
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.ws.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=s):
            self.mesh(stream=s)
        torch.cuda.current_stream().wait_stream(s)
        return g


def mesh_batch(items, flags: int = 0, tuning: Tuning | None = None):
    """Plan, allocate and emit a list of (bitmap, grid_h); returns [(verts, tris, codes)]."""
    b = Batch(items, tuning=tuning, flags=flags)
    sizes = b.plan()
    outs = b.allocate(sizes)
    b.emit()
    st = b.sizes()
    for i, s in enumerate(st):
        if s[3] != 0:
            raise SbmtError(int(s[3]), f"image {i}")
    return outs
