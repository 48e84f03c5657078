"""Independent invariant checks for SBMT meshes (numpy/scipy only).

Nothing here comes from the oracle or from the HIP path: the expected values are
closed forms computed from the bitmap alone.

* closure: every directed edge occurs once; interior edges occur in both
  directions; boundary edges (one direction only) form closed loops along the
  extracted boundary (exact boundary embedding theorem, Sec. 3.3.4);
* boundary fidelity: boundary edges are exactly the marching-squares segments
  of the coarse samples cut into pieces (each edge on one segment, in its
  direction; the pieces of a segment chain from its start to its end; every
  segment covered), and their total length equals the polyline length;
* area: the triangle areas sum to the area enclosed by the boundary polylines,
  computed cell by cell from the coarse samples;
* Euler characteristic: V - E + F = (#8-connected foreground components) -
  (#4-connected background components - 1), from connected-component labelling;
* positive orientation of every triangle.
"""
from __future__ import annotations

import math

import numpy as np


def stride_for(h) -> int:
    """Smallest s with s^2 > 2 h^2 (h a dyadic rational, compared exactly)."""
    from fractions import Fraction
    hf = Fraction(h)
    s = 1
    while s * s <= 2 * hf * hf:
        s += 1
    return s


def grid_x0(h) -> float:
    """x of lattice vertex (0, 0): -(2h+3)/4, moved left by 1/(4U) when h = p/U with
    U = 2^q > 1, so that 4U x is odd on every lattice vertex."""
    from fractions import Fraction
    hf = Fraction(h)
    U = hf.denominator
    x0 = -(2 * hf + 3) / 4 - (Fraction(1, 4 * U) if U > 1 else 0)
    return float(x0)


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


# Marching-squares segments of one dual cell, corners TL, TR, BR, BL (bit 0..3 of the
# case).  Cell edge j joins corner j and corner j+1 (0 top, 1 right, 2 bottom, 3 left).
# A segment starts on the edge of each foreground->background step (walking the
# corners in that order) and ends on the edge of the next background->foreground
# step, so background corners are cut off (foreground 8-connected at saddles).
def _ms_case_segments(case: int):
    v = [(case >> j) & 1 for j in range(4)]
    out = []
    for j in range(4):
        if v[j] == 1 and v[(j + 1) % 4] == 0:
            t = (j + 1) % 4
            while not (v[t] == 0 and v[(t + 1) % 4] == 1):
                t = (t + 1) % 4
            out.append((j, t))
    return out


_MS = [_ms_case_segments(c) for c in range(16)]
# midpoint of cell edge j relative to the TL sample, in units of s/2
_MID = np.array([[1, 0], [2, 1], [1, 2], [0, 1]], np.int64)


def ms_segments(coarse: np.ndarray, s: int):
    """Oriented marching-squares segments (foreground on the left) of the coarse
    samples with a background ring: (P, Q, cell) with P, Q in pixels, float64
    [n, 2] (exact half-integers), and the dual cell (R, C) of each, R, C >= -1."""
    tl, tr, br, bl = _cells(coarse)
    case = tl | (tr << 1) | (br << 2) | (bl << 3)
    Ps, Qs, cells = [], [], []
    for c in range(1, 15):
        R, C = np.nonzero(case == c)
        if R.size == 0:
            continue
        R = R - 1
        C = C - 1
        # TL sample of cell (R, C) sits at (s C + (s-1)/2, s R + (s-1)/2)
        x0 = s * C + (s - 1) / 2.0
        y0 = s * R + (s - 1) / 2.0
        for (a, b) in _MS[c]:
            Ps.append(np.stack([x0 + _MID[a, 0] * s / 2.0, y0 + _MID[a, 1] * s / 2.0], 1))
            Qs.append(np.stack([x0 + _MID[b, 0] * s / 2.0, y0 + _MID[b, 1] * s / 2.0], 1))
            cells.append(np.stack([R, C], 1))
    if not Ps:
        z = np.zeros((0, 2))
        return z, z, np.zeros((0, 2), np.int64)
    return np.concatenate(Ps), np.concatenate(Qs), np.concatenate(cells)


def check_boundary_exact(verts: np.ndarray, bnd: np.ndarray, coarse: np.ndarray, s: int) -> int:
    """Boundary embedding (Sec. 3.3.4): the mesh's boundary edges are exactly the
    marching-squares segments cut into pieces.  Every boundary edge lies on one
    segment with its direction; the pieces of each segment chain from its start
    point to its end point through shared vertices; every segment is covered.
    Returns the number of segments."""
    P, Q, cell = ms_segments(coarse, s)
    n = P.shape[0]
    assert (n == 0) == (bnd.shape[0] == 0), (n, bnd.shape)
    if n == 0:
        return 0
    CH, CW = coarse.shape
    # segments by cell: two slots per dual cell (R, C), R, C in -1 .. CH-1 / CW-1
    slot = np.full(((CH + 1) * (CW + 1), 2), -1, np.int64)
    ci = (cell[:, 0] + 1) * (CW + 1) + (cell[:, 1] + 1)
    first = np.ones(n, bool)
    order = np.argsort(ci, kind="stable")
    dup = np.zeros(n, bool)
    dup[order[1:]] = ci[order[1:]] == ci[order[:-1]]
    first[dup] = False
    slot[ci[first], 0] = np.nonzero(first)[0]
    slot[ci[dup], 1] = np.nonzero(dup)[0]
    a, b = verts[bnd[:, 0]], verts[bnd[:, 1]]
    m = 0.5 * (a + b)
    # the midpoint of a piece lies inside the open cell square of its segment
    C = np.floor((m[:, 0] - (s - 1) / 2.0) / s).astype(np.int64)
    R = np.floor((m[:, 1] - (s - 1) / 2.0) / s).astype(np.int64)
    assert ((R >= -1) & (R < CH) & (C >= -1) & (C < CW)).all(), "boundary edge outside the cells"
    cand = slot[(R + 1) * (CW + 1) + (C + 1)]
    seg = np.full(bnd.shape[0], -1, np.int64)
    tol = 1e-9 * (1.0 + np.abs(verts).max())
    for j in range(2):
        c = cand[:, j]
        ok = c >= 0
        cc = np.where(ok, c, 0)
        p, q = P[cc], Q[cc]
        d = q - p
        L2 = (d * d).sum(1)
        # both ends on the segment's line, between its ends, in its direction
        cr_a = d[:, 0] * (a[:, 1] - p[:, 1]) - d[:, 1] * (a[:, 0] - p[:, 0])
        cr_b = d[:, 0] * (b[:, 1] - p[:, 1]) - d[:, 1] * (b[:, 0] - p[:, 0])
        ta = ((a - p) * d).sum(1) / L2
        tb = ((b - p) * d).sum(1) / L2
        on = ok & (np.abs(cr_a) <= tol * s) & (np.abs(cr_b) <= tol * s) & (ta >= -1e-12) & (tb <= 1 + 1e-12) & (tb > ta)
        assert not (on & (seg >= 0)).any(), "boundary edge on two segments"
        seg = np.where(on, c, seg)
    assert (seg >= 0).all(), f"{(seg < 0).sum()} boundary edges off the marching-squares segments"
    # chain the pieces of every segment from P to Q
    d = Q[seg] - P[seg]
    ta = ((a - P[seg]) * d).sum(1) / (d * d).sum(1)
    o = np.lexsort((ta, seg))
    sg, ea, eb = seg[o], bnd[o, 0], bnd[o, 1]
    start = np.ones(len(sg), bool)
    start[1:] = sg[1:] != sg[:-1]
    end = np.ones(len(sg), bool)
    end[:-1] = sg[1:] != sg[:-1]
    assert len(np.unique(sg)) == n, f"{n - len(np.unique(sg))} segments without a boundary edge"
    assert np.array_equal(verts[ea[start]], P[sg[start]]), "a segment's first piece does not start at its start"
    assert np.array_equal(verts[eb[end]], Q[sg[end]]), "a segment's last piece does not end at its end"
    inner = ~end
    assert np.array_equal(eb[inner], ea[1:][inner[:-1]]), "pieces of a segment do not chain"
    return n


def lattice_inside(coarse: np.ndarray, s: int, h: int, NK: int, NI: int) -> np.ndarray:
    """Inside bit of every lattice vertex (k, i) by ray parity: the number of
    marching-squares segments crossed by the horizontal ray from the vertex to
    x = -inf (no degeneracy: row lines y = -1 + k h sqrt3/2 never meet the
    half-integer segment ends)."""
    P, Q, _ = ms_segments(coarse, s)
    inside = np.zeros((NK, NI), bool)
    if P.shape[0] == 0:
        return inside
    rh = float(h) * math.sqrt(3.0) / 2.0
    ylo = np.minimum(P[:, 1], Q[:, 1])
    yhi = np.maximum(P[:, 1], Q[:, 1])
    order = np.argsort(ylo)
    ylo_s = ylo[order]
    x0 = grid_x0(h)
    h = float(h)
    for k in range(NK):
        y = -1.0 + (h * k) * 0.86602540378443864676
        sel = order[:np.searchsorted(ylo_s, y)]
        sel = sel[yhi[sel] > y]
        if sel.size == 0:
            continue
        p, q = P[sel], Q[sel]
        xc = np.sort(p[:, 0] + (y - p[:, 1]) / (q[:, 1] - p[:, 1]) * (q[:, 0] - p[:, 0]))
        xs = x0 + h * np.arange(NI) + (h / 2.0) * (k & 1)
        inside[k] = (np.searchsorted(xc, xs) & 1) == 1
    return inside


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
        n_seg = check_boundary_exact(verts, bnd, coarse, s)
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
        stats.update(area=area, chi=chi, perimeter=length, n_segments=n_seg)
    return stats
