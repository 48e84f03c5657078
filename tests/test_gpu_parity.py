"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Connectivity and codes must be bit-exact; FP64 vertex coordinates must agree
within 1e-12 * grid_h (both sides evaluate the same IEEE formulas without
contraction, so the observed difference is 0).  Every case prints its name
before touching the GPU.
"""
from __future__ import annotations

import itertools
import sys

import numpy as np
import pytest

import mesh_checks as mc
import oracle
from paper_2602_19474_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _sbmt():
    import paper_2602_19474_amd as sbmt
    return sbmt


def _gpu_mesh(bm: np.ndarray, h: int, both: bool = False, sizes: bool = False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(bm, np.uint8)).to("cuda")
    v, tr, c, sz = _sbmt().mesh_from_bitmap(t, h, both_sides=both, return_sizes=True)
    torch.cuda.synchronize()
    out = (v.cpu().numpy(), tr.cpu().numpy(), c.cpu().numpy())
    return out + (sz,) if sizes else out


def _compare(name: str, bm: np.ndarray, h: int, both: bool = False, check_invariants: bool = True):
    print(f"[gpu-parity] {name} {bm.shape} h={h} both={both}", flush=True)
    v, t, c, sz = _gpu_mesh(bm, h, both, sizes=True)
    ref = oracle.mesh_from_bitmap(bm, h, oracle.BOTH_SIDES if both else 0)
    # boundary segments and cut base triangles counted by the kernels
    assert (sz.n_segments, sz.n_cut) == (ref.n_segments, ref.n_cut), (sz, ref.n_segments, ref.n_cut)
    assert t.shape == ref.tris.shape, (t.shape, ref.tris.shape)
    assert v.shape == ref.verts.shape, (v.shape, ref.verts.shape)
    assert np.array_equal(t, ref.tris), "triangle connectivity differs"
    assert np.array_equal(c, ref.codes), "case codes differ"
    dv = float(np.abs(v - ref.verts).max(initial=0.0))
    assert dv <= 1e-12 * h, dv
    if check_invariants:
        mc.check_mesh(v, t, c, bm, h, both_sides=both)
    return dv


@pytest.mark.parametrize("item", range(10))
def test_disk64(item):
    _compare(f"disk64#{item}", wl.disk(item=item), 1)


@pytest.mark.parametrize("h", [1, 2, 4])
@pytest.mark.parametrize("both", [False, True])
def test_ellipses1024(h, both):
    _compare("ellipses1024", wl.ellipses(), h, both)


@pytest.mark.parametrize("h", [1, 2, 3, 4, 5, 6])
def test_smoothed_noise_all_grid_edges(h):
    g = wl.rng(77, h)
    _compare("noise301x257", wl.smoothed_noise(301, 257, 8.0, 0.0, False, g), h)
    _compare("noise600x1100z", wl.smoothed_noise(1100, 600, 16.0, 0.3, True, g), h)


def test_brute_force_small_coarse_bitmaps():
    """All 3x3 coarse bitmaps and seeded 4x4..8x8 ones, several offsets, h in {1,2,4}."""
    for h in (1, 2, 4):
        s = mc.stride_for(h)
        cases = [np.array(b, np.uint8).reshape(3, 3) for b in itertools.product([0, 1], repeat=9)]
        rs = np.random.default_rng(1000 + h)
        cases += [rs.integers(0, 2, (n, n)).astype(np.uint8) for n in (4, 5, 6, 8) for _ in range(25)]
        print(f"[gpu-parity] brute force h={h}: {len(cases)} cases", flush=True)
        for ci, cb in enumerate(cases):
            big = np.kron(cb, np.ones((s, s), np.uint8))
            bm = np.zeros((big.shape[0] + ci % 3, big.shape[1] + (ci // 3) % 3), np.uint8)
            bm[ci % 3:, (ci // 3) % 3:] = big
            _compare(f"bf{ci}", bm, h, both=(ci % 5 == 0), check_invariants=False)


def test_edge_cases():
    _compare("empty 0x0", np.zeros((0, 0), np.uint8), 1)
    _compare("empty 7x0", np.zeros((7, 0), np.uint8), 2)
    _compare("all background", np.zeros((50, 70), np.uint8), 1)
    _compare("all foreground", np.ones((50, 70), np.uint8), 1)
    _compare("all foreground h=4", np.ones((61, 13), np.uint8), 4)
    _compare("single pixel", np.ones((1, 1), np.uint8), 1)
    _compare("one row", (np.arange(1000) % 7 < 4).astype(np.uint8)[None, :], 1)
    _compare("one column", (np.arange(999) % 5 < 3).astype(np.uint8)[:, None], 2)
    _compare("checkerboard", (np.indices((64, 64)).sum(0) % 2).astype(np.uint8), 1)
    _compare("nonzero values", (np.arange(40 * 40).reshape(40, 40) % 251).astype(np.uint8), 1)
    _compare("both sides empty", np.zeros((20, 20), np.uint8), 1, both=True)


def test_row_stride_and_errors():
    import torch
    sbmt = _sbmt()
    bm = wl.disk(item=4)
    big = np.zeros((64, 80), np.uint8)
    big[:, :64] = bm
    t = torch.from_numpy(big).to("cuda")[:, :64]  # row stride 80 > width 64
    assert t.stride(0) == 80
    print("[gpu-parity] strided view", flush=True)
    v, tr, c = sbmt.mesh_from_bitmap(t, 1)
    ref = oracle.mesh_from_bitmap(bm, 1)
    assert np.array_equal(tr.cpu().numpy(), ref.tris) and np.array_equal(c.cpu().numpy(), ref.codes)
    with pytest.raises(sbmt.SbmtError) as e:
        sbmt.mesh_from_bitmap(t.contiguous(), 7)
    assert e.value.status == -2
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(sbmt.SbmtError) as e:
        sbmt.plan(t.contiguous(), 1, ws)
    assert e.value.status == -4


def test_mesh_async_matches_and_respects_capacity():
    import torch
    sbmt = _sbmt()
    bm = wl.ellipses()
    t = torch.from_numpy(bm).to("cuda")
    ref_v, ref_t, ref_c = _gpu_mesh(bm, 2)
    ws = sbmt.workspace(t, 2)
    nv, nt = ref_v.shape[0], ref_t.shape[0]
    verts = torch.full((nv + 100, 2), -1.0, dtype=torch.float64, device="cuda")
    tris = torch.full((nt + 100, 3), -1, dtype=torch.int32, device="cuda")
    codes = torch.zeros((nt + 100,), dtype=torch.uint8, device="cuda")
    sizes = torch.zeros(5, dtype=torch.int64, device="cuda")
    print("[gpu-parity] mesh_async fits", flush=True)
    sbmt.mesh_async(t, 2, ws, verts, tris, codes, sizes)
    torch.cuda.synchronize()
    s = sizes.cpu().numpy()
    assert s[0] == nv and s[1] == nt and s[3] == 0
    assert np.array_equal(tris[:nt].cpu().numpy(), ref_t) and np.array_equal(verts[:nv].cpu().numpy(), ref_v)
    assert np.array_equal(codes[:nt].cpu().numpy(), ref_c)
    assert (tris[nt:].cpu().numpy() == -1).all()
    print("[gpu-parity] mesh_async too small", flush=True)
    small_t = torch.full((nt - 1, 3), -7, dtype=torch.int32, device="cuda")
    small_c = torch.zeros((nt - 1,), dtype=torch.uint8, device="cuda")
    sbmt.mesh_async(t, 2, ws, verts, small_t, small_c, sizes)
    torch.cuda.synchronize()
    s = sizes.cpu().numpy()
    assert s[3] == -7 and s[1] == nt
    assert (small_t.cpu().numpy() == -7).all()


def test_deterministic_and_stream():
    import torch
    bm = wl.smoothed_noise(900, 700, 8.0, 0.0, False, wl.rng(5, 5))
    a = _gpu_mesh(bm, 1)
    st = torch.cuda.Stream()
    print("[gpu-parity] side stream", flush=True)
    with torch.cuda.stream(st):
        t = torch.from_numpy(bm).to("cuda")
        v, tr, c = _sbmt().mesh_from_bitmap(t, 1)
    st.synchronize()
    assert np.array_equal(a[1], tr.cpu().numpy()) and np.array_equal(a[0], v.cpu().numpy())
    assert np.array_equal(a[2], c.cpu().numpy())


def test_batch256_sample():
    """A seeded sample of the batch workload images (sizes 128..2048, h in {1,2,4})."""
    for j in (0, 1, 2, 3):
        g = wl.rng(3, j)
        w, h = int(g.integers(128, 2049)), int(g.integers(128, 2049))
        gh = int(g.choice([1, 2, 4]))
        bm = wl.smoothed_noise(w, h, 8.0, 0.0, False, g)
        _compare(f"batch256#{j}", bm, gh)


@pytest.mark.slow
def test_noise8192_full_size():
    """The largest single-image workload, compared with the oracle in full."""
    import time
    t0 = time.time()
    bm = wl.noise8192()
    print(f"[gpu-parity] noise8192 generated in {time.time() - t0:.1f}s", flush=True)
    v, t, c = _gpu_mesh(bm, 1)
    print(f"[gpu-parity] noise8192 GPU mesh {v.shape[0]} verts {t.shape[0]} tris", flush=True)
    ref = oracle.mesh_from_bitmap(bm, 1)
    print(f"[gpu-parity] noise8192 oracle done at {time.time() - t0:.1f}s", flush=True)
    assert np.array_equal(t, ref.tris) and np.array_equal(c, ref.codes)
    assert float(np.abs(v - ref.verts).max(initial=0.0)) <= 1e-12
    del ref
    mc.check_mesh(v, t, c, bm, 1)
    print(f"[gpu-parity] noise8192 done at {time.time() - t0:.1f}s", flush=True)
    sys.stdout.flush()


@pytest.mark.slow
@pytest.mark.parametrize("h", [1, 4])
def test_tall_and_wide_strips(h):
    """Images 2^20 pixels long (the largest side the boundary accepts): coordinates
    there are largest, and so is the rounding of the double-precision sign filter
    that the exact fallback covers."""
    g = wl.rng(78, h)
    strip = wl.smoothed_noise(24, 1 << 20, 2.0, 0.0, False, g)
    _compare("tall strip", strip, h, check_invariants=False)
    _compare("wide strip", np.ascontiguousarray(strip.T), h, check_invariants=False)


@pytest.mark.parametrize("h", [0.5, 0.75, 1.25, 1.5, 2.5, 0.375])
def test_dyadic_grid_edges(h):
    """Grid edges p / 2^q, including the paper's h < 1 (Sec. 3.3)."""
    g = wl.rng(79, int(h * 8))
    _compare("disk64", wl.disk(item=1), h)
    _compare("ellipses", wl.ellipses(400, 330, g=g), h)
    _compare("noise", wl.smoothed_noise(257, 301, 4.0, 0.0, False, g), h, both=(h == 0.75))


def test_dyadic_brute_force_3x3():
    for h in (0.5, 0.75, 1.5):
        s = mc.stride_for(h)
        print(f"[gpu-parity] dyadic brute force h={h}", flush=True)
        for ci, b in enumerate(itertools.product([0, 1], repeat=9)):
            big = np.kron(np.array(b, np.uint8).reshape(3, 3), np.ones((s, s), np.uint8))
            bm = np.zeros((big.shape[0] + ci % 3, big.shape[1] + (ci // 3) % 3), np.uint8)
            bm[ci % 3:, (ci // 3) % 3:] = big
            _compare(f"bf{ci}", bm, h, check_invariants=False)


def test_fine_grid_edges():
    """h = 1/64 and 1/16: coordinates in units of 1/256 and 1/64 pixel, so the
    exact predicates and the floating-point band are 4096 and 256 times wider
    than at integer h for the same image."""
    g = wl.rng(80, 0)
    _compare("h=1/64", wl.smoothed_noise(60, 50, 3.0, 0.0, False, g), 1.0 / 64)
    _compare("h=1/16 strip", wl.smoothed_noise(2000, 3, 3.0, 0.0, False, g), 1.0 / 16, check_invariants=False)
