"""Independent check of the canonical output order (numpy only).

From the vertex coordinates and the grid formula alone, every vertex is given
its owner lattice vertex (k, i) and its kind, and every triangle its parent
base triangle; then the stated order is asserted:

* vertices ascend by (k, i, kind): the owner itself, then the crossings on its
  edges E0 = (k,i) -> (k,i+1), E1 = (k,i) -> (k+1,i+o-1), E2 = (k,i) -> (k+1,i+o)
  (o = k mod 2), each edge's crossings in order of distance from the owner,
  then the chain vertex inside its triangle Tb = [v(k,i), v(k+1,i+o), v(k+1,i+o-1)],
  then the one inside Ta = [v(k,i), v(k,i+1), v(k+1,i+o)];
* every triangle starts at its smallest index; triangles ascend by parent
  (row k, column i, Tb before Ta) and lexicographically within a parent.

Grid (Sec. 3.3, rows horizontal): vertex (k, i) is at
x = x0 + h i + (h/2)(k mod 2), y = -1 + k h sqrt3/2, evaluated as
y = -1.0 + (h k) * 0.86602540378443864676 in double precision, with
x0 = -(2h+3)/4, less 1/(4U) when h = p/U with U = 2^q > 1.  Boundary points
(marching-squares ends, the chain vertices) are half-integers; lattice x is an
odd multiple of 1/(4U); crossings lie strictly inside grid edges.
"""
from __future__ import annotations

import math

import numpy as np

HALF_SQRT3 = 0.86602540378443864676


def _row_y(h, k):
    return -1.0 + (float(h) * np.asarray(k, np.float64)) * HALF_SQRT3


def _units(h):
    """(h as float, U = 2^q, x of vertex (0, 0))."""
    from fractions import Fraction
    import mesh_checks
    hf = Fraction(h)
    return float(hf), hf.denominator, mesh_checks.grid_x0(hf)


def vertex_keys(verts: np.ndarray, h: int, NK: int, NI: int):
    """Per vertex: (kind, k, i, sub, param) with kind 0 lattice, 1 crossing, 2 chain vertex;
    sub = 0 self, 1 + d for a crossing on edge E_d, 4 chain vertex in Tb, 5 in Ta."""
    h, U, x0 = _units(h)
    x, y = verts[:, 0], verts[:, 1]
    n = x.shape[0]
    rh = h * math.sqrt(3.0) / 2.0
    tr = (y + 1.0) / rh
    kr = np.rint(tr).astype(np.int64)
    x4 = 4.0 * U * x
    odd4 = (x4 == np.rint(x4)) & (np.rint(x4).astype(np.int64) % 2 == 1)
    half = (2.0 * x == np.rint(2.0 * x)) & (2.0 * y == np.rint(2.0 * y))
    lat = odd4 & (y == _row_y(h, kr))
    kind = np.where(lat, 0, np.where(half, 2, 1))
    k = np.zeros(n, np.int64)
    i = np.zeros(n, np.int64)
    sub = np.zeros(n, np.int64)
    par = np.zeros(n, np.float64)
    # lattice vertices
    m = kind == 0
    k[m] = kr[m]
    i[m] = np.rint((x[m] - x0 - (h / 2.0) * (kr[m] & 1)) / h).astype(np.int64)
    assert np.allclose(x0 + h * i[m] + (h / 2.0) * (k[m] & 1), x[m], rtol=0, atol=1e-12), "lattice x"
    # crossings: a horizontal edge (on a row line) or a diagonal one inside a band
    m = kind == 1
    kb = np.floor(tr[m]).astype(np.int64)
    f = tr[m] - kb
    onrow = (np.abs(tr[m] - kr[m]) * rh) <= 1e-9 * (1.0 + np.abs(y[m]))
    kk = np.where(onrow, kr[m], kb)
    xo = x0 + (h / 2.0) * (kk & 1)
    u = (x[m] - xo) / h
    ih = np.floor(u)
    # down-left edge from (k, i): x = x(k,i) - f h/2; down-right: x = x(k,i) + f h/2
    udl, udr = u + f / 2.0, u - f / 2.0
    is_dl = np.abs(udl - np.rint(udl)) <= 1e-7
    is_dr = np.abs(udr - np.rint(udr)) <= 1e-7
    assert (onrow | (is_dl ^ is_dr)).all(), "crossing not on exactly one grid edge"
    ii = np.where(onrow, ih, np.where(is_dl, np.rint(udl), np.rint(udr))).astype(np.int64)
    d = np.where(onrow, 0, np.where(is_dl, 1, 2))
    k[m], i[m], sub[m] = kk, ii, 1 + d
    par[m] = np.where(onrow, u - ih, f)
    # strictly inside its edge
    assert ((par[m] > 0) & (par[m] < 1)).all(), "crossing at a lattice vertex"
    # chain vertices: the base triangle holding the point
    m = kind == 2
    kb = np.floor(tr[m]).astype(np.int64)
    f = tr[m] - kb
    u = (x[m] - x0 - (h / 2.0) * (kb & 1)) / h
    ib = np.floor(u + f / 2.0)
    dd = u + f / 2.0 - ib
    in_tb = dd < f
    k[m], i[m] = kb, ib.astype(np.int64)
    sub[m] = np.where(in_tb, 4, 5)
    assert ((k >= 0) & (k < NK) & (i >= 0) & (i < NI)).all(), "owner outside the grid"
    return kind, k, i, sub, par


def triangle_parents(verts: np.ndarray, tris: np.ndarray, h):
    """Parent base triangle (k, i, t) of every triangle, from its centroid."""
    h, U, x0 = _units(h)
    c = verts[tris].mean(axis=1)
    rh = h * math.sqrt(3.0) / 2.0
    tr = (c[:, 1] + 1.0) / rh
    kb = np.floor(tr).astype(np.int64)
    f = tr - kb
    u = (c[:, 0] - x0 - (h / 2.0) * (kb & 1)) / h
    ib = np.floor(u + f / 2.0)
    t = np.where(u + f / 2.0 - ib < f, 0, 1)
    return kb, ib.astype(np.int64), t


def check_numbering(verts: np.ndarray, tris: np.ndarray, h: int, NK: int, NI: int) -> dict:
    nv = verts.shape[0]
    kind, k, i, sub, par = vertex_keys(verts, h, NK, NI)
    key = np.stack([k, i, sub], 1)
    if nv > 1:
        a, b = key[:-1], key[1:]
        lt = (a[:, 0] < b[:, 0]) | ((a[:, 0] == b[:, 0]) & ((a[:, 1] < b[:, 1]) | ((a[:, 1] == b[:, 1]) & (
            (a[:, 2] < b[:, 2]) | ((a[:, 2] == b[:, 2]) & (par[:-1] < par[1:]))))))
        assert lt.all(), f"vertex order broken at {np.nonzero(~lt)[0][:5]}"
    # at most two crossings per edge, one chain vertex per triangle, one self
    _, cnt = np.unique(key, axis=0, return_counts=True) if nv else (None, np.zeros(0, int))
    assert cnt.max(initial=0) <= 2
    nt = tris.shape[0]
    if nt:
        assert ((tris[:, 0] < tris[:, 1]) & (tris[:, 0] < tris[:, 2])).all(), "triangle not rotated to its smallest id"
        pk, pi, pt = triangle_parents(verts, tris, h)
        pkey = (pk * (NI + 1) + pi) * 2 + pt
        step = np.diff(pkey)
        assert (step >= 0).all(), "parents do not ascend"
        same = step == 0
        t0, t1 = tris[:-1][same], tris[1:][same]
        lex = (t0[:, 0] < t1[:, 0]) | ((t0[:, 0] == t1[:, 0]) & ((t0[:, 1] < t1[:, 1]) | (
            (t0[:, 1] == t1[:, 1]) & (t0[:, 2] < t1[:, 2]))))
        assert lex.all(), "triangles of one parent not in lexicographic order"
        # every vertex of a triangle lies in the closed parent base triangle
        o = pk & 1
        hh, _, X0 = _units(h)
        ax = X0 + hh * pi + (hh / 2.0) * o
        ay = _row_y(h, pk)
        by = _row_y(h, pk + 1)
        for j in range(3):
            v = verts[tris[:, j]]
            ff = (v[:, 1] - ay) / (by - ay)
            assert ((ff >= -1e-9) & (ff <= 1 + 1e-9)).all()
            lo = np.where(pt == 0, ax - ff * hh / 2, ax + ff * hh / 2)
            hi = np.where(pt == 0, ax + ff * hh / 2, ax + hh - ff * hh / 2)
            assert ((v[:, 0] >= lo - 1e-9) & (v[:, 0] <= hi + 1e-9)).all(), "vertex outside its parent"
    return {"lattice": kind == 0, "k": k, "i": i, "kind": kind}
