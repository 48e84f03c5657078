"""GPU parity of the mesh of Alg. 3 (sbmt_preprocess_mesh) against the oracle's
preprocessed mesh (oracle_mesh_preprocessed): the same triangles as coordinate
triples with their codes (within 1e-9 px; both sides evaluate the same FP64
formulas), the same number of vertices in use, the same counts of snapped,
repelled, inserted and cut; at the paper's thresholds every triangle meets the
area bound of Sec. 3.3.4 (and, on the full-size image, the angle bound).
Every case prints its name before touching the GPU.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import mesh_checks as mc
import oracle
from paper_2602_19474_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _canon(V, T, C):
    P = V[np.asarray(T, np.int64)]  # [n, 3, 2]
    key = P[:, :, 1] * 1e6 + P[:, :, 0]
    r = np.argmin(key, 1)
    idx = (r[:, None] + np.arange(3)[None]) % 3
    Q = np.take_along_axis(P, idx[:, :, None], 1).reshape(-1, 6)
    A = np.concatenate([Q, np.asarray(C, np.float64)[:, None]], 1)
    return A[np.lexsort(A.T[::-1])]


def _bounds(h, a, b, c):
    e = float(h)
    th = min(math.atan(b / (e + a - math.sqrt(a * a - b * b))), math.atan(c / (e + a)))
    return math.degrees(th), 0.5 * b * c


def _compare(name, bm, h, th=None):
    import torch
    from paper_2602_19474_amd.preprocess import preprocess_mesh
    print(f"[gpu-pre-mesh] {name} {bm.shape} h={h} th={th}", flush=True)
    ref = oracle.mesh_preprocessed(bm, h) if th is None else oracle.mesh_preprocessed(bm, h, *th)
    m = preprocess_mesh(torch.from_numpy(np.ascontiguousarray(bm, np.uint8)).cuda(), h, *ref.thresholds)
    torch.cuda.synchronize()
    v, t, c = m.verts.cpu().numpy(), m.tris.cpu().numpy(), m.codes.cpu().numpy()
    assert (m.n_snapped, m.n_repelled, m.n_inserted, m.n_cut) == (ref.n_snapped, ref.n_repelled, ref.n_inserted,
                                                                  ref.n_cut)
    assert t.shape == ref.tris.shape, (t.shape, ref.tris.shape)
    assert np.unique(t).size == ref.verts.shape[0]
    # only vertices some triangle uses are output: grid vertices first, then the new ones
    assert v.shape[0] == ref.verts.shape[0], (v.shape, ref.verts.shape)
    if t.shape[0]:
        assert np.unique(t).size == v.shape[0] and t.min() == 0 and t.max() == v.shape[0] - 1
    A, B = _canon(v, t, c), _canon(ref.verts, ref.tris, ref.codes)
    assert np.array_equal(A[:, 6], B[:, 6]), "codes differ"
    assert np.abs(A[:, :6] - B[:, :6]).max(initial=0.0) <= 1e-9, "triangles differ"
    if t.shape[0]:
        ar = mc.signed_areas(v, t)
        assert ar.min() > 0
        if th is None:  # the bounds of Sec. 3.3.4 at the paper's thresholds
            thb, amin = _bounds(h, *ref.thresholds)
            assert ar.min() > amin
    return m


@pytest.mark.parametrize("item", range(3))
def test_disk64(item):
    _compare(f"disk64#{item}", wl.disk(item=item), 1)


@pytest.mark.parametrize("h", [0.5, 1, 2, 4])
def test_ellipses(h):
    _compare("ellipses", wl.ellipses(200, 180, g=wl.rng(97, int(4 * h))), h)


@pytest.mark.parametrize("h", [0.75, 1.5, 6])
def test_ellipses_other_grid_edges(h):
    _compare("ellipses", wl.ellipses(220, 200, g=wl.rng(93, int(8 * h))), h)


@pytest.mark.parametrize("h,sigma", [(1, 2.0), (1, 4.0), (2, 3.0)])
def test_smoothed_noise(h, sigma):
    _compare(f"noise sigma={sigma}", wl.smoothed_noise(240, 220, sigma, 0.0, False, wl.rng(98, int(4 * h + sigma))), h)


def test_degenerate_and_zero_thresholds():
    _compare("empty", np.zeros((40, 50), np.uint8), 1)
    _compare("full", np.ones((33, 45), np.uint8), 2)
    _compare("zero thresholds", wl.disk(item=1), 1, (0.0, 0.0, 0.0))


def test_other_admissible_thresholds():
    bm = wl.smoothed_noise(256, 256, 3.0, 0.0, False, wl.rng(95, 1))
    for th in ((0.4, 0.19, 0.28), (0.3, 0.1, 0.05), (0.45, 0.2, 0.3)):
        _compare("thresholds", bm, 1, th)


def test_ragged_and_small_images():
    _compare("ragged 97x61", wl.smoothed_noise(61, 97, 2.0, 0.0, False, wl.rng(99, 0)), 1)
    _compare("one pixel", np.ones((1, 1), np.uint8), 1)
    bm = np.zeros((64, 64), np.uint8)
    bm[::2, ::2] = 1
    _compare("checker", bm, 0.5)
    _compare("noise h=1/2", wl.smoothed_noise(160, 150, 1.5, 0.0, False, wl.rng(94, 2)), 0.5)


def test_full_size_noise8192_bounds_and_crops():
    """The 8192 x 8192 noise workload at h = 1: every triangle meets the angle
    and area bounds of Sec. 3.3.4, and the interior of crops (the method is
    local) equals the oracle's mesh of the crop."""
    import torch
    from paper_2602_19474_amd.preprocess import paper_thresholds, preprocess_mesh
    bm_np = wl.noise8192()
    H, W = bm_np.shape
    print("[gpu-pre-mesh] noise8192 h=1", flush=True)
    m = preprocess_mesh(torch.from_numpy(bm_np).cuda(), 1)
    torch.cuda.synchronize()
    V, T = m.verts, m.tris.long()
    assert int(T.min()) >= 0 and int(T.max()) < V.shape[0]
    assert m.n_snapped > 10 ** 5 and m.n_cut > 10 ** 5
    A, B, C = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    ar2 = (B[:, 0] - A[:, 0]) * (C[:, 1] - A[:, 1]) - (B[:, 1] - A[:, 1]) * (C[:, 0] - A[:, 0])
    a, b, c = paper_thresholds(1)
    thb, amin = _bounds(1, a, b, c)
    assert float(ar2.min()) > 2 * amin

    def ang(P, Q, R):
        u, w = Q - P, R - P
        return torch.rad2deg(torch.atan2((u[:, 0] * w[:, 1] - u[:, 1] * w[:, 0]).abs(), (u * w).sum(1)))
    amin_deg = float(torch.minimum(torch.minimum(ang(A, B, C), ang(B, C, A)), ang(C, A, B)).min())
    assert amin_deg > thb, (amin_deg, thb)
    del A, B, C, ar2
    Vh, Th, Ch = V.cpu().numpy(), m.tris.cpu().numpy(), m.codes.cpu().numpy()
    P = Vh[Th]
    for ox, wdt in ((4096, 320), (W - 320, 320)):
        crop = np.ascontiguousarray(bm_np[:320, ox:ox + wdt])
        print(f"[gpu-pre-mesh] crop x={ox} w={wdt}", flush=True)
        ref = oracle.mesh_preprocessed(crop, 1)
        lo = 16.0
        hi = np.inf if ox + wdt == W else wdt - 16.0
        Q = ref.verts[ref.tris]
        sel_r = ((Q[:, :, 0] > lo) & (Q[:, :, 0] < hi) & (Q[:, :, 1] < 300)).all(1)
        sel_g = ((P[:, :, 0] > lo + ox) & (P[:, :, 0] < hi + ox) & (P[:, :, 1] < 300)).all(1)
        shifted = ref.verts + np.array([float(ox), 0.0])
        Ra = _canon(shifted, ref.tris[sel_r], ref.codes[sel_r])
        Ga = _canon(Vh, Th[sel_g], Ch[sel_g])
        assert Ra.shape == Ga.shape and Ra.shape[0] > 1000, (Ra.shape, Ga.shape)
        assert np.array_equal(Ra[:, 6], Ga[:, 6])
        assert np.abs(Ra[:, :6] - Ga[:, :6]).max() <= 1e-9


def test_refusals_capacity_and_repeated_calls():
    """sbmt_preprocess_mesh through the C ABI: inadmissible thresholds and a short
    workspace are refused; too few rows give the capacity status with the counts
    filled in and nothing written past the capacity; exact capacities give the
    wrapper's mesh; calls on one workspace repeat exactly (every per-call state is
    cleared)."""
    import ctypes

    import torch
    from paper_2602_19474_amd import _lib, context, _image, _stream_ptr
    from paper_2602_19474_amd.preprocess import paper_thresholds, preprocess_mesh
    print("[gpu-pre-mesh] refusals, capacity, repeats", flush=True)
    bm = torch.from_numpy(wl.ellipses(150, 130, g=wl.rng(91, 4))).to("cuda")
    ref = preprocess_mesh(bm, 1)
    nv, nt = ref.verts.shape[0], ref.tris.shape[0]
    L = _lib.lib()
    img = _image(bm, 1, 0)
    ws_bytes, gbound = ctypes.c_size_t(), ctypes.c_int64()
    assert L.sbmt_pre_mesh_query(ctypes.byref(img), ctypes.byref(ws_bytes), ctypes.byref(gbound)) == 0
    ws = torch.empty(int(ws_bytes.value), dtype=torch.uint8, device="cuda")
    h = context(0).handle
    counts = (ctypes.c_int64 * 8)()
    a, b, c = paper_thresholds(1)
    # one spare row past each capacity, holding a sentinel
    verts = torch.full((nv + 1, 2), -7.0, dtype=torch.float64, device="cuda")
    tris = torch.full((nt + 1, 3), -7, dtype=torch.int32, device="cuda")
    codes = torch.full((nt + 1,), 7, dtype=torch.uint8, device="cuda")

    def call(th, wsb, vcap, tcap):
        return L.sbmt_preprocess_mesh(h, ctypes.byref(img), *th, ws.data_ptr(), wsb, verts.data_ptr(), vcap,
                                      tris.data_ptr(), codes.data_ptr(), tcap, counts, _stream_ptr(None))

    for th in ((0.4, 0.2, 0.1), (0.4, 0.1, 0.29), (0.5, 0.1, 0.1), (-0.1, 0.0, 0.0)):
        assert call(th, int(ws_bytes.value), nv, nt) == -1, th
    assert call((a, b, c), int(ws_bytes.value) - 1, nv, nt) == -4
    for vcap, tcap in ((0, 0), (nv - 1, nt), (nv, nt - 1)):
        verts.fill_(-7.0)
        tris.fill_(-7)
        codes.fill_(7)
        assert call((a, b, c), int(ws_bytes.value), vcap, tcap) == -7, (vcap, tcap)
        assert (counts[0], counts[1], counts[5]) == (nv, nt, -7)
        torch.cuda.synchronize()
        assert bool((verts[vcap:] == -7.0).all()) and bool((tris[tcap:] == -7).all()) and bool((codes[tcap:] == 7).all())
    for rep in range(3):
        verts[:nv] = 0.0
        tris[:nt] = 0
        assert call((a, b, c), int(ws_bytes.value), nv, nt) == 0, rep
        torch.cuda.synchronize()
        assert (counts[0], counts[1], counts[5], counts[6], counts[7]) == (nv, nt, 0, ref.n_grid_vertices, ref.n_cut)
        assert torch.equal(verts[:nv], ref.verts) and torch.equal(tris[:nt], ref.tris)
        assert torch.equal(codes[:nt], ref.codes)
        assert bool((verts[nv:] == -7.0).all()) and bool((tris[nt:] == -7).all())
