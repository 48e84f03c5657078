"""Pins of the preprocessed grid the oracle returns (Alg. 3, Steps 1-3, before
the retriangulation against the polyline), checked by brute force over every
polyline vertex and segment, independently of the oracle's arithmetic:

* all thresholds zero: the grid is the plain lattice (closed form of the vertex
  positions) with its two base triangles per slot;
* Step 1 (snap, a): a lattice vertex sits on a polyline vertex exactly when its
  lattice position lies closer than a to one, and then on the nearest one;
* Step 2 (repel, c): a vertex left in place that lay closer than c to a segment
  now lies at distance c from it on the same side, having moved along the
  segment's normal; every other one is where the lattice put it and at least c
  from every segment;
* Step 3 (eliminate, b): the inserted vertices are exactly the polyline
  vertices no lattice vertex sits on that lie closer than b to a side of a
  base triangle of the moved lattice; afterwards every such free polyline
  vertex is at least b from every side of the grid;
* the grid is a triangulation of the same region: every triangle has positive
  area, the areas sum to those of the base triangles on the moved lattice, and
  each inserted vertex adds one triangle per base triangle on its side.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree

import mesh_checks as mc
import numbering_checks as nc
import oracle
from paper_2602_19474_amd import workloads as wl


def _lattice(h, NK, NI):
    hf = float(Fraction(h))
    k = np.repeat(np.arange(NK), NI)
    i = np.tile(np.arange(NI), NK)
    x = mc.grid_x0(h) + hf * i + 0.5 * hf * (k % 2)
    return np.stack([x, nc._row_y(h, k)], 1)


def _base_triangles(NK, NI):
    """Slot Tb = [(k,i), (k+1,i+o), (k+1,i+o-1)], Ta = [(k,i), (k,i+1), (k+1,i+o)]."""
    out = []
    for k in range(NK - 1):
        o = k & 1
        for i in range(NI):
            for t in range(2):
                cs = [(k, i), (k + 1, i + o), (k + 1, i + o - 1)] if t == 0 else [(k, i), (k, i + 1), (k + 1, i + o)]
                if all(0 <= ci < NI for _, ci in cs):
                    out.append([ck * NI + ci for ck, ci in cs])
    return np.array(out, np.int64).reshape(-1, 3)


def _seg_dist(X, P, Q):
    """Distances [len(X), len(P)] from points to segments P -> Q."""
    d = (Q - P)[None]
    w = X[:, None, :] - P[None]
    t = np.clip((w * d).sum(-1) / (d * d).sum(-1), 0.0, 1.0)
    r = w - t[..., None] * d
    return np.sqrt((r * r).sum(-1))


def _cross(X, P, Q):
    d = Q - P
    return d[:, 0] * (X[:, 1] - P[:, 1]) - d[:, 1] * (X[:, 0] - P[:, 0])


def _edges(tris):
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    return np.unique(np.sort(e, 1), axis=0)


def _grid(bm, h, th=None):
    plain = oracle.mesh_from_bitmap(bm, h)
    NK, NI, s = plain.grid
    g = oracle.preprocessed_grid(bm, h) if th is None else oracle.preprocessed_grid(bm, h, *th)
    P, Q, _ = mc.ms_segments(mc.coarse_samples(bm, h), s)
    return g, NK, NI, P, Q


CASES = [("disk", 1), ("disk", 2), ("ellipses", 0.5), ("ellipses", 1), ("ellipses", 2), ("noise", 1),
         ("noise", 4), ("square", 1)]


def _bitmap(name, h):
    if name == "disk":
        return wl.disk(item=2)
    if name == "ellipses":
        return wl.ellipses(150, 130, g=wl.rng(91, int(4 * h)))
    if name == "noise":
        return wl.smoothed_noise(140, 120, 3.0, 0.0, False, wl.rng(92, int(4 * h)))
    bm = np.zeros((60, 60), np.uint8)
    bm[13:47, 11:49] = 1
    return bm


def test_zero_thresholds_give_the_plain_lattice():
    for h in (0.5, 1, 2):
        bm = wl.disk(item=1)
        g, NK, NI, _, _ = _grid(bm, h, (0.0, 0.0, 0.0))
        assert np.array_equal(g.verts, _lattice(h, NK, NI))
        assert not g.on_polyline.any()
        assert (g.n_snapped, g.n_repelled, g.n_inserted) == (0, 0, 0)
        assert np.array_equal(g.tris, _base_triangles(NK, NI))


@pytest.mark.parametrize("name,h", CASES)
def test_steps_against_brute_force(name, h):
    bm = _bitmap(name, h)
    g, NK, NI, P, Q = _grid(bm, h)
    a, b, c = g.thresholds
    n = NK * NI
    lat = _lattice(h, NK, NI)
    V = g.verts
    assert V.shape[0] == n + g.n_inserted and g.on_polyline.shape[0] == V.shape[0]
    assert P.shape[0] > 0
    # Step 1: snapped exactly when a polyline vertex lies closer than a, onto the nearest
    # (brute force over the polyline vertices near each lattice vertex)
    near, jn = cKDTree(P).query(lat)
    snapped = g.on_polyline[:n].astype(bool)
    assert np.array_equal(snapped, near < a)
    assert snapped.sum() == g.n_snapped > 0
    assert np.array_equal(V[:n][snapped], P[jn[snapped]])
    # Step 2: the rest lie at least c from every segment; the moved ones at exactly c,
    # on their side, displaced along the segment's normal.  Candidates: vertices within
    # c + (longest segment)/2 of a segment midpoint; the others are farther than c.
    free = ~snapped
    Vf, Lf = V[:n][free], lat[free]
    reach = c + 0.5 * np.sqrt(((Q - P) ** 2).sum(1)).max() + 1e-9
    cand = np.isfinite(cKDTree(0.5 * (P + Q)).query(Lf, distance_upper_bound=reach)[0])
    d0 = _seg_dist(Lf[cand], P, Q)
    moved = np.zeros(Lf.shape[0], bool)
    moved[cand] = d0.min(1) < c
    assert moved.sum() == g.n_repelled > 0
    assert np.array_equal(Vf[~moved], Lf[~moved])
    j = d0[moved[cand]].argmin(1)
    d1 = _seg_dist(Vf[moved], P, Q)
    assert np.allclose(d1[np.arange(j.size), j], c, rtol=0, atol=1e-9)
    assert d1.min() > c * (1 - 1e-9)
    assert np.all(np.sign(_cross(Vf[moved], P[j], Q[j])) == np.sign(_cross(Lf[moved], P[j], Q[j])))
    disp = Vf[moved] - Lf[moved]
    dirs = Q[j] - P[j]
    assert np.allclose((disp * dirs).sum(1), 0.0, atol=1e-9)
    cand2 = np.isfinite(cKDTree(0.5 * (P + Q)).query(Vf, distance_upper_bound=reach)[0])
    assert _seg_dist(Vf[cand2], P, Q).min() > c * (1 - 1e-9)
    # Step 3: inserted = free polyline vertices closer than b to a side of a base
    # triangle of the moved lattice (candidate sides: midpoint within 2h of the polyline)
    base = _base_triangles(NK, NI)
    E = _edges(base)
    E = E[np.isfinite(cKDTree(P).query(0.5 * (V[E[:, 0]] + V[E[:, 1]]), distance_upper_bound=2.0 * float(h))[0])]
    onv = {tuple(p) for p in V[:n][snapped]}
    fp = np.array([p for p in P if tuple(p) not in onv]).reshape(-1, 2)
    de = _seg_dist(fp, V[E[:, 0]], V[E[:, 1]])
    want = {tuple(p) for p in fp[de.min(1) < b]}
    got = {tuple(p) for p in V[n:]}
    assert got == want and len(got) == g.n_inserted
    assert g.on_polyline[n:].all()
    # ... and afterwards no free polyline vertex off the grid's vertices is within b of a side
    E2 = _edges(g.tris)
    E2 = E2[np.isfinite(cKDTree(P).query(0.5 * (V[E2[:, 0]] + V[E2[:, 1]]), distance_upper_bound=2.0 * float(h))[0])]
    rest = np.array([p for p in fp if tuple(p) not in got]).reshape(-1, 2)
    if rest.shape[0]:
        assert _seg_dist(rest, V[E2[:, 0]], V[E2[:, 1]]).min() >= b
    # triangulation of the same region
    ar = mc.signed_areas(V, g.tris)
    assert ar.min() > 0
    assert abs(ar.sum() - mc.signed_areas(V, base).sum()) < 1e-9 * ar.sum()
    # each inserted vertex replaces every base triangle on its side by two
    be = np.sort(np.concatenate([base[:, [0, 1]], base[:, [1, 2]], base[:, [2, 0]]]), 1)
    per_edge = {}
    for e in map(tuple, be):
        per_edge[e] = per_edge.get(e, 0) + 1
    row = {tuple(p): r for r, p in enumerate(fp)}
    side_tris = sum(per_edge[tuple(E[int(np.argmin(de[row[tuple(V[m])]]))])] for m in range(n, V.shape[0]))
    assert g.tris.shape[0] == base.shape[0] + side_tris


def test_paper_thresholds_are_the_oracle_default():
    g = oracle.preprocessed_grid(wl.disk(item=0), 2)
    sc = 2 / 0.45 ** 0.5
    assert g.thresholds == (0.26 * sc, 0.125 * sc, 0.183 * sc)
