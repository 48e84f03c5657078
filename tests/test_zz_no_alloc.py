"""The allocation-free entry point against sbmt_mesh_async, through the C ABI.

Two calls in a row on the library's scratch array, the second with a smaller
image (the array keeps the first call's contents): each mesh and sizes record
must equal what sbmt_mesh_async gives with a caller-owned workspace (bit for
bit: the same kernels on the same inputs).  An image whose workspace exceeds
the array is refused on the host, and a capacity that is too small reports
SBMT_E_CAPACITY like the workspace variant.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2602_19474_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _outputs(nv, nt, fill=True):
    import torch
    v = torch.full((nv, 2), -1.0, dtype=torch.float64, device="cuda")
    t = torch.full((nt, 3), -1, dtype=torch.int32, device="cuda")
    c = torch.full((nt,), 255, dtype=torch.uint8, device="cuda")
    return v, t, c


def _both(bm, h):
    import torch

    import paper_2602_19474_amd as sbmt
    x = torch.from_numpy(np.ascontiguousarray(bm)).cuda()
    lay = sbmt.query(bm.shape[1], bm.shape[0], h)
    assert lay.workspace_bytes <= sbmt.NOALLOC_SCRATCH_BYTES
    ws = sbmt.workspace(x, h)
    cap_v, cap_t = 4 * bm.size // (h * h) + 64, 8 * bm.size // (h * h) + 64
    a = _outputs(cap_v, cap_t)
    b = _outputs(cap_v, cap_t)
    sa = torch.zeros(sbmt.SIZE_WORDS, dtype=torch.int64, device="cuda")
    sb = torch.zeros(sbmt.SIZE_WORDS, dtype=torch.int64, device="cuda")
    sbmt.mesh_async(x, h, ws, *a, sa)
    sbmt.mesh_noalloc(x, h, *b, sb)
    torch.cuda.synchronize()
    ra, rb = sa.cpu().tolist(), sb.cpu().tolist()
    assert ra == rb and ra[3] == 0, (ra, rb)
    nv, nt = ra[0], ra[1]
    assert np.array_equal(a[1][:nt].cpu().numpy(), b[1][:nt].cpu().numpy()), "connectivity"
    assert np.array_equal(a[2][:nt].cpu().numpy(), b[2][:nt].cpu().numpy()), "codes"
    assert np.array_equal(a[0][:nv].cpu().numpy(), b[0][:nv].cpu().numpy()), "coordinates"
    return nv, nt


def test_noalloc_matches_mesh_async_twice_then_smaller():
    big = wl.smoothed_noise(1500, 1300, 8.0, 0.0, False, wl.rng(96, 0))
    small = wl.disk(item=5)
    print(f"[gpu-noalloc] first call {big.shape} h=1", flush=True)
    n1 = _both(big, 1)
    print(f"[gpu-noalloc] second call {small.shape} h=1 (smaller)", flush=True)
    n2 = _both(small, 1)
    assert n2[1] < n1[1]
    print("[gpu-noalloc] third call ellipses h=2", flush=True)
    _both(wl.ellipses(), 2)


def test_noalloc_refuses_what_does_not_fit():
    import torch

    import paper_2602_19474_amd as sbmt
    bm = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    assert sbmt.query(4096, 4096, 1).workspace_bytes > sbmt.NOALLOC_SCRATCH_BYTES
    v, t, c = _outputs(16, 16)
    s = torch.zeros(sbmt.SIZE_WORDS, dtype=torch.int64, device="cuda")
    print("[gpu-noalloc] workspace larger than the scratch array: refused on the host", flush=True)
    with pytest.raises(sbmt.SbmtError) as e:
        sbmt.mesh_noalloc(bm, 1, v, t, c, s)
    assert e.value.status == -4
    print("[gpu-noalloc] capacity too small", flush=True)
    d = torch.from_numpy(wl.disk(item=2)).cuda()
    sbmt.mesh_noalloc(d, 1, v, t, c, s)
    torch.cuda.synchronize()
    r = s.cpu().tolist()
    assert r[3] == -7 and r[1] > 16
    assert (t.cpu().numpy() == -1).all()
