"""Pins of the preprocessing oracle (Alg. 3: snap a, repel c, edge elimination b).

* With every threshold at zero the path is the plain one: the meshes equal the
  pinned plain oracle's triangle for triangle (as geometric sets; the numbering
  of the preprocessed mesh is by coordinates).
* With the paper's thresholds (a, b, c) = (0.26, 0.125, 0.183) scaled by
  h / sqrt(0.45) (Sec. 4; they satisfy b < a/2, c < a/sqrt2, a < h/2):
  every invariant of mesh_checks holds (closure, exact boundary embedding,
  area, Euler characteristic, orientation), and every triangle meets the
  minimum-angle bound min{atan(b/(e + a - sqrt(a^2 - b^2))), atan(c/(e + a))}
  and the minimum-area bound b c / 2 (Sec. 3.3.4, App. D), with e = h.
* Away from the boundary the mesh is the base grid; the rules act (counts of
  snapped, repelled and inserted points); inadmissible thresholds are refused.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

import mesh_checks as mc
import oracle
from paper_2602_19474_amd import workloads as wl


def _tri_set(verts, tris):
    out = []
    for t in verts[tris]:
        pts = [tuple(np.round(p, 12)) for p in t]
        m = min(range(3), key=lambda j: pts[j])
        out.append(tuple(pts[m:] + pts[:m]))
    return sorted(out)


def _min_angles(verts, tris):
    A, B, C = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]

    def ang(P, Q, R):
        u, v = Q - P, R - P
        return np.degrees(np.arctan2(np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0]), (u * v).sum(1)))
    return np.minimum(np.minimum(ang(A, B, C), ang(B, C, A)), ang(C, A, B))


def _bounds(h, a, b, c):
    e = float(h)
    theta = min(math.atan(b / (e + a - math.sqrt(a * a - b * b))), math.atan(c / (e + a)))
    return math.degrees(theta), 0.5 * b * c


def _check(bm, h):
    pre = oracle.mesh_preprocessed(bm, h)
    mc.check_mesh(pre.verts, pre.tris, np.zeros_like(pre.codes), bm, h)
    th, amin = _bounds(h, *pre.thresholds)
    if pre.tris.shape[0]:
        ang = _min_angles(pre.verts, pre.tris)
        assert ang.min() > th, (ang.min(), th)
        assert (ang >= 5.0).all(), "sliver"
        ar = mc.signed_areas(pre.verts, pre.tris)
        assert ar.min() > amin, (ar.min(), amin)
    return pre


def test_paper_bounds_at_the_default_thresholds():
    a, b, c = oracle.PAPER_THRESHOLDS
    th, amin = _bounds(oracle.PAPER_EDGE, a, b, c)
    # the paper states about 10.1 degrees and 1.14e-2
    assert abs(th - 10.085) < 1e-3 and abs(amin - 0.0114375) < 1e-9
    assert b < a / 2 and c < a / math.sqrt(2) and a < oracle.PAPER_EDGE / 2


@pytest.mark.parametrize("case", ["disk", "ellipses", "noise"])
@pytest.mark.parametrize("h", [1, 2, 0.5])
def test_all_rules_off_is_the_plain_path(case, h):
    g = wl.rng(96, int(4 * h))
    bm = {"disk": wl.disk(item=1), "ellipses": wl.ellipses(260, 230, g=g),
          "noise": wl.smoothed_noise(190, 170, 4.0, 0.0, False, g)}[case]
    plain = oracle.mesh_from_bitmap(bm, h)
    pre = oracle.mesh_preprocessed(bm, h, 0.0, 0.0, 0.0)
    assert (pre.n_snapped, pre.n_repelled, pre.n_inserted) == (0, 0, 0)
    assert pre.n_cut == plain.n_cut
    assert _tri_set(pre.verts, pre.tris) == _tri_set(plain.verts, plain.tris)


@pytest.mark.parametrize("item", range(5))
def test_bounds_disks(item):
    pre = _check(wl.disk(item=item), 1)
    assert pre.n_snapped > 0 and pre.n_repelled > 0 and pre.n_inserted > 0


@pytest.mark.parametrize("h", [0.5, 1, 2, 4, 1.5, 0.75])
def test_bounds_ellipses(h):
    _check(wl.ellipses(320, 300, g=wl.rng(95, int(4 * h))), h)


@pytest.mark.parametrize("h,sigma", [(1, 2.0), (1, 4.0), (2, 3.0), (4, 8.0), (0.5, 1.5)])
def test_bounds_smoothed_noise(h, sigma):
    g = wl.rng(94, int(4 * h + sigma))
    _check(wl.smoothed_noise(260, 240, sigma, 0.0, False, g), h)


@pytest.mark.parametrize("h", [1, 2])
def test_bounds_every_3x3_coarse_bitmap(h):
    s = mc.stride_for(h)
    for ci, bits in enumerate(itertools.product([0, 1], repeat=9)):
        cb = np.array(bits, np.uint8).reshape(3, 3)
        big = np.kron(cb, np.ones((s, s), np.uint8))
        bm = np.zeros((big.shape[0] + ci % 2, big.shape[1] + (ci // 2) % 2), np.uint8)
        bm[ci % 2:, (ci // 2) % 2:] = big
        _check(bm, h)


def test_rules_off_show_the_slivers_the_rules_remove():
    """The ablation of Table 2 in small: without the rules the same input has
    angles far below the bound (E5), with them none (E1)."""
    bm = wl.smoothed_noise(400, 400, 2.0, 0.0, False, wl.rng(93, 0))
    plain = oracle.mesh_from_bitmap(bm, 1)
    pre = _check(bm, 1)
    th, _ = _bounds(1, *pre.thresholds)
    assert _min_angles(plain.verts, plain.tris).min() < 1.0 < th


def test_far_from_the_boundary_nothing_moves():
    bm = np.zeros((80, 80), np.uint8)
    bm[20:60, 20:60] = 1
    pre = oracle.mesh_preprocessed(bm, 1)
    plain = oracle.mesh_from_bitmap(bm, 1)
    far = lambda v: (np.abs(v[:, 0] - 39.5) < 15) & (np.abs(v[:, 1] - 39.5) < 15)
    a = _tri_set(pre.verts, pre.tris)
    b = _tri_set(plain.verts, plain.tris)
    fa = [t for t in a if all(abs(x - 39.5) < 15 and abs(y - 39.5) < 15 for x, y in (t[0], t[1], t[2]))]
    fb = [t for t in b if all(abs(x - 39.5) < 15 and abs(y - 39.5) < 15 for x, y in (t[0], t[1], t[2]))]
    assert fa == fb and len(fa) > 1000
    assert far(pre.verts).sum() == far(plain.verts).sum()


def test_closed_forms_and_refusals():
    assert oracle.mesh_preprocessed(np.zeros((30, 30), np.uint8), 1).tris.shape == (0, 3)
    pre = _check(np.ones((31, 29), np.uint8), 1)
    assert abs(mc.signed_areas(pre.verts, pre.tris).sum() - mc.ms_area(mc.coarse_samples(np.ones((31, 29), np.uint8), 1), 2)) < 1e-9
    bm = wl.disk(item=0)
    for (a, b, c) in ((0.3, 0.16, 0.1), (0.3, 0.1, 0.22), (0.6, 0.1, 0.1), (-0.1, 0, 0)):
        with pytest.raises(oracle.OracleError):
            oracle.mesh_preprocessed(bm, 1, a, b, c)
    d1 = oracle.mesh_preprocessed(bm, 1)
    d2 = oracle.mesh_preprocessed(bm, 1)
    assert np.array_equal(d1.tris, d2.tris) and np.array_equal(d1.verts, d2.verts)
