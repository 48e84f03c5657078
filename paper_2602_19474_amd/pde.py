"""Cotangent Laplacian and explicit heat steps on a mesh (GPU).

Thin front end of the Laplacian entry points of ``include/sbmt_post.h``; the
assembly and the steps run in the HIP kernels of ``libsbmt.so``.

    lap = Laplacian(verts, tris)             # assemble (waits)
    u = lap.heat_init(x0, y0, sigma, 100.0)  # Gaussian pulse, 0 on the boundary
    lap.heat_steps(u, alpha=500.0, dt=1.9 / (500.0 * lap.info["lambda_bound"]), steps=100)
"""
from __future__ import annotations

import ctypes

from . import _lib
from . import _stream_ptr, context


def _torch():
    import torch
    return torch


class Laplacian:
    """The assembled operator of one mesh; keeps its workspace on the device."""

    def __init__(self, verts, tris, stream=None):
        torch = _torch()
        self.ctx = context(verts.device.index)
        self.verts = verts
        self.nv, self.nt = int(verts.shape[0]), int(tris.shape[0])
        b = ctypes.c_size_t()
        _lib.check(_lib.lib().sbmt_laplacian_workspace(self.nv, self.nt, ctypes.byref(b)),
                   "sbmt_laplacian_workspace")
        self.ws = torch.empty((max(int(b.value), 1),), dtype=torch.uint8, device=verts.device)
        info = _lib.LaplacianInfo()
        _lib.check(_lib.lib().sbmt_laplacian_assemble(
            self.ctx.handle, verts.data_ptr() if self.nv else None, self.nv, tris.data_ptr() if self.nt else None,
            self.nt, self.ws.data_ptr(), self.ws.numel(), ctypes.byref(info), _stream_ptr(stream)),
            "sbmt_laplacian_assemble")
        self.info = {n: getattr(info, n) for n, _ in _lib.LaplacianInfo._fields_}

    def _args(self):
        return self.ws.data_ptr(), self.ws.numel(), self.nv, self.nt

    def csr(self) -> dict:
        """Views of the operator's arrays inside the workspace (row_off, col, val, mass, boundary)."""
        torch = _torch()
        c = _lib.Csr()
        _lib.check(_lib.lib().sbmt_laplacian_csr(*self._args(), ctypes.byref(c)), "sbmt_laplacian_csr")
        base = self.ws.data_ptr()
        nnz = int(self.info["nnz"])

        def view(ptr, n, dtype, size):
            off = ptr - base
            return self.ws[off:off + n * size].view(dtype)
        return {"row_off": view(c.row_off, self.nv + 1, torch.int64, 8), "col": view(c.col, nnz, torch.int32, 4),
                "val": view(c.val, nnz, torch.float64, 8), "mass": view(c.mass, self.nv, torch.float64, 8),
                "boundary": view(c.boundary, self.nv, torch.uint8, 1)}

    def apply(self, u, stream=None):
        """y = K u."""
        torch = _torch()
        y = torch.empty_like(u)
        _lib.check(_lib.lib().sbmt_laplacian_apply(self.ctx.handle, *self._args(), u.data_ptr(), y.data_ptr(),
                                                   _stream_ptr(stream)), "sbmt_laplacian_apply")
        return y

    def heat_init(self, x0: float, y0: float, sigma: float, amp: float = 100.0, stream=None):
        torch = _torch()
        u = torch.empty((self.nv,), dtype=torch.float64, device=self.verts.device)
        _lib.check(_lib.lib().sbmt_heat_init(self.ctx.handle, *self._args()[:2], self.verts.data_ptr(), self.nv,
                                             self.nt, float(x0), float(y0), float(sigma), float(amp), u.data_ptr(),
                                             _stream_ptr(stream)), "sbmt_heat_init")
        return u

    def heat_steps(self, u, alpha: float, dt: float, steps: int, tmp=None, stream=None):
        """``steps`` explicit Euler steps on ``u`` in place (``tmp``: scratch of the same size)."""
        torch = _torch()
        tmp = torch.empty_like(u) if tmp is None else tmp
        _lib.check(_lib.lib().sbmt_heat_steps(self.ctx.handle, *self._args(), float(alpha), float(dt), int(steps),
                                              u.data_ptr(), tmp.data_ptr(), _stream_ptr(stream)), "sbmt_heat_steps")
        return u
