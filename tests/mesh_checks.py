"""Independent invariant checks for SBMT meshes (numpy/scipy only).

Nothing here comes from the oracle or from the HIP path: the expected values are
closed forms computed from the bitmap alone.

* closure: every directed edge occurs once; interior edges occur in both
  directions; boundary edges (one direction only) form closed loops along the
  extracted boundary (exact boundary embedding theorem, Sec. 3.3.4);
* boundary fidelity: boundary edges run along marching-squares directions
  (axis-aligned or 45 degrees) and their total length equals the polyline length;
* area: the triangle areas sum to the area enclosed by the boundary polylines,
  computed cell by cell from the coarse samples;
* Euler characteristic: V - E + F = (#8-connected foreground components) -
  (#4-connected background components - 1), from connected-component labelling;
* positive orientation of every triangle.
"""
from __future__ import annotations

import math

import numpy as np


def stride_for(h: int) -> int:
    s = 1
    while s * s <= 2 * h * h:
        s += 1
    return s


def coarse_samples(bitmap: np.ndarray, h: int) -> np.ndarray:
    """Block majority over s x s pixels (ties to foreground, missing pixels background)."""
    s = stride_for(h)
    H, W = bitmap.shape
    CH, CW = -(-H // s), -(-W // s)
    pad = np.zeros((CH * s, CW * s), np.int64)
    pad[:H, :W] = (bitmap != 0)
    cnt = pad.reshape(CH, s, CW, s).sum(axis=(1, 3))
    return (2 * cnt >= s * s).astype(np.uint8)


def _cells(coarse: np.ndarray):
    P = np.pad(coarse.astype(np.int64), 1)
    tl, tr, bl, br = P[:-1, :-1], P[:-1, 1:], P[1:, :-1], P[1:, 1:]
    return tl, tr, br, bl


def ms_area(coarse: np.ndarray, s: int) -> float:
    """Area inside the marching-squares polylines (foreground 8-connected at saddles)."""
    tl, tr, br, bl = _cells(coarse)
    n = tl + tr + br + bl
    saddle = (n == 2) & (tl == br)
    area8 = np.where(n == 0, 0, np.where(n == 1, 1, np.where(n == 2, np.where(saddle, 6, 4),
                                                             np.where(n == 3, 7, 8))))
    return float(area8.sum()) * s * s / 8.0


def ms_perimeter(coarse: np.ndarray, s: int):
    """(number of diagonal segments, number of straight segments)."""
    tl, tr, br, bl = _cells(coarse)
    n = tl + tr + br + bl
    saddle = (n == 2) & (tl == br)
    diag = ((n == 1) | (n == 3)).sum() + 2 * saddle.sum()
    straight = ((n == 2) & ~saddle).sum()
    return int(diag), int(straight)


def euler_expected(coarse: np.ndarray) -> int:
    from scipy.ndimage import label

    P = np.pad(coarse, 1)
    _, nfg = label(P, structure=np.ones((3, 3), int))
    _, nbg = label(1 - P, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    return int(nfg) - (int(nbg) - 1)


def signed_areas(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))


def check_mesh(verts: np.ndarray, tris: np.ndarray, codes: np.ndarray, bitmap: np.ndarray, h: int,
               both_sides: bool = False) -> dict:
    """Assert every invariant; return a few statistics."""
    s = stride_for(h)
    coarse = coarse_samples(bitmap, h)
    nv, nt = verts.shape[0], tris.shape[0]
    assert tris.dtype == np.int32 and codes.dtype == np.uint8 and verts.dtype == np.float64
    if nt:
        assert tris.min() >= 0 and tris.max() < nv, "triangle index out of range"
    # every vertex is used
    used = np.zeros(nv, bool)
    used[tris.ravel()] = True
    assert used.all() or nv == 0, f"{(~used).sum()} unused vertices"
    # orientation
    ar = signed_areas(verts, tris)
    assert (ar > 0).all(), f"{(ar <= 0).sum()} triangles without positive area"
    # closure
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]).astype(np.int64)
    key = e[:, 0] * nv + e[:, 1]
    order = np.argsort(key)
    sk = key[order]
    assert not (sk[1:] == sk[:-1]).any() if nt else True, "a directed edge occurs twice"
    rkey = e[:, 1] * nv + e[:, 0]
    has_rev = np.isin(rkey, key)
    bnd = e[~has_rev]
    n_und = (len(e) + len(bnd)) // 2
    stats = {"V": nv, "T": nt, "boundary_edges": len(bnd)}
    if not both_sides:
        # boundary loops: in-degree == out-degree == 1 on boundary vertices
        outdeg = np.bincount(bnd[:, 0], minlength=nv)
        indeg = np.bincount(bnd[:, 1], minlength=nv)
        assert (outdeg == indeg).all() and outdeg.max(initial=0) <= 1, "boundary is not a set of loops"
        d = verts[bnd[:, 1]] - verts[bnd[:, 0]]
        ax = (np.abs(d[:, 0]) <= 1e-9) | (np.abs(d[:, 1]) <= 1e-9)
        dg = np.abs(np.abs(d[:, 0]) - np.abs(d[:, 1])) <= 1e-9 * (1 + np.abs(d).max(initial=0))
        assert (ax | dg).all(), "boundary edge off the marching-squares directions"
        length = np.sqrt((d * d).sum(axis=1)).sum()
        ndiag, nstr = ms_perimeter(coarse, s)
        expect_len = ndiag * s / math.sqrt(2.0) + nstr * s
        assert abs(length - expect_len) <= 1e-9 * max(1.0, expect_len), (length, expect_len)
        # area
        area = ar.sum()
        expect_area = ms_area(coarse, s)
        assert abs(area - expect_area) <= 1e-9 * max(1.0, expect_area), (area, expect_area)
        # Euler characteristic
        chi = nv - n_und + nt
        assert chi == euler_expected(coarse), (chi, euler_expected(coarse))
        assert (codes < 0x80).all()
        stats.update(area=area, chi=chi, perimeter=length)
    return stats
