"""Pins of the CPU oracle of the mesh consumers (field sampling, mesh quality).

CPU only.  Each pin comes from outside the oracle: closed forms of hand-built
triangles (angles, aspect ratios, areas), fields the bilinear rule reproduces
exactly (linear and xy), numpy's mean and variance, and invariants of the
oracle's own meshes computed independently of the quality code (the area of
the boundary polygons by the shoelace formula, the uncut triangles being
equilateral).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2602_19474_amd import workloads as wl

ATAN_3_4_DEG = 36.869897645844021297  # atan(3/4) in degrees
TWO_OVER_SQRT3 = 1.1547005383792515290


def _tri(*pts):
    v = np.array(pts, np.float64)
    return v, np.array([[0, 1, 2]], np.int32)


def test_equilateral_and_345_closed_forms():
    v, t = _tri((0.0, 0.0), (1.0, 0.0), (0.5, math.sqrt(3.0) / 2))
    q = oracle.mesh_quality(v, t)
    assert q["n_triangles"] == 1 and q["n_equilateral"] == 1 and q["n_slivers"] == 0
    assert abs(q["ar_max"] - TWO_OVER_SQRT3) < 1e-15
    assert abs(q["min_angle_deg"] - 60.0) < 1e-12
    assert abs(q["min_area"] - math.sqrt(3.0) / 4) < 1e-16
    assert q["angle_hist"][29] == 1 and q["angle_hist"].sum() == 1
    assert q["var_area"] == 0.0
    v, t = _tri((0.0, 0.0), (4.0, 0.0), (4.0, 3.0))
    q = oracle.mesh_quality(v, t)
    assert q["ar_max"] == 25.0 / 12.0  # longest edge^2 / (2 area) = 25 / 12
    assert abs(q["min_angle_deg"] - ATAN_3_4_DEG) < 1e-12
    assert q["min_area"] == 6.0 and q["n_equilateral"] == 0
    assert q["angle_hist"][18] == 1  # 36.87 deg lies in [36, 38)


@pytest.mark.parametrize("deg,sliver,bin_", [(3.0, 1, 1), (4.5, 1, 2), (5.5, 0, 2), (7.0, 0, 3), (31.0, 0, 15),
                                             (59.0, 0, 29)])
def test_isosceles_apex_angle(deg, sliver, bin_):
    """Apex angle deg at the origin, legs of length 3: the smallest angle for deg < 60."""
    th = math.radians(deg)
    for (ox, oy, sc) in ((0.0, 0.0, 1.0), (100.25, -7.5, 0.37)):
        v, t = _tri((ox, oy), (ox + 3 * sc, oy), (ox + 3 * sc * math.cos(th), oy + 3 * sc * math.sin(th)))
        q = oracle.mesh_quality(v, t)
        assert q["n_slivers"] == sliver and q["angle_hist"][bin_] == 1, (deg, q)
        want = deg if deg < 60 else (180 - deg) / 2
        assert abs(q["min_angle_deg"] - want) < 1e-9
        # AR of an isosceles triangle with apex angle th < 60: legs are longest,
        # AR = L^2 / (L^2 sin th) = 1 / sin th
        assert abs(q["ar_max"] - 1.0 / math.sin(th)) < 1e-12 / math.sin(th)


def test_percentiles_nearest_rank():
    """Right triangles (0,0), (1,0), (0,t): AR = (1 + t^2) / t for t < 1."""
    ts = np.array([k / 16 for k in (1, 3, 4, 6, 7, 9, 10, 12, 13, 15)], np.float64)
    rs = np.random.default_rng(5)
    for n in (1, 2, 3, 7, 10):
        pick = rs.permutation(ts)[:n]
        verts, tris = [], []
        for j, t in enumerate(pick):
            verts += [(0.0 + 10 * j, 0.0), (1.0 + 10 * j, 0.0), (0.0 + 10 * j, t)]
            tris.append((3 * j, 3 * j + 1, 3 * j + 2))
        q = oracle.mesh_quality(np.array(verts), np.array(tris, np.int32))
        ar = sorted((1 + t * t) / t for t in pick)
        assert q["ar_median"] == ar[math.ceil(n / 2) - 1]
        assert q["ar_p95"] == ar[math.ceil(0.95 * n) - 1]
        assert q["ar_max"] == ar[-1]


def test_area_mean_and_variance_against_numpy():
    rs = np.random.default_rng(17)
    n = 5000
    p = rs.uniform(-50, 50, (n, 3, 2))
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0]))
    p[area < 0] = p[area < 0][:, [0, 2, 1]]  # positive orientation
    q = oracle.mesh_quality(p.reshape(-1, 2), np.arange(3 * n, dtype=np.int32).reshape(n, 3))
    a = np.abs(area)
    assert abs(q["mean_area"] - a.mean()) <= 1e-12 * a.mean()
    assert abs(q["var_area"] - a.var()) <= 1e-12 * a.var()
    assert q["min_area"] == pytest.approx(a.min(), rel=1e-13) and q["max_area"] == pytest.approx(a.max(), rel=1e-13)
    assert q["n_nonpositive"] == 0 and q["angle_hist"].sum() == n


def test_invalid_inverted_and_empty():
    v = np.array([(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)])
    q = oracle.mesh_quality(v, np.array([[0, 2, 1], [0, 1, 5], [0, 1, 2]], np.int32))
    assert q["n_triangles"] == 2 and q["n_invalid"] == 1 and q["n_nonpositive"] == 1
    assert q["min_area"] == -0.5 and q["max_area"] == 0.5
    q = oracle.mesh_quality(np.zeros((0, 2)), np.zeros((0, 3), np.int32))
    assert q["n_triangles"] == 0 and q["min_angle_tri"] == -1 and math.isnan(q["ar_median"])


def _shoelace_area(chains):
    tot = 0.0
    for c in chains:
        x, y = c[:, 0] / 4.0, c[:, 1] / 4.0
        tot += 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))
    return tot


@pytest.mark.parametrize("which,h", [("disk", 1), ("ellipses", 2), ("noise", 1), ("noise", 4)])
def test_mesh_invariants(which, h):
    if which == "disk":
        bm = wl.disk(item=2)
    elif which == "ellipses":
        bm = wl.ellipses(item=0)[:400, :500]
    else:
        bm = wl.smoothed_noise(300, 260, 8.0, 0.0, False, wl.rng(93, h))
    m = oracle.mesh_from_bitmap(bm, h)
    q = oracle.mesh_quality(m.verts, m.tris)
    n = m.tris.shape[0]
    assert q["n_triangles"] == n and q["n_nonpositive"] == 0 and q["angle_hist"].sum() == n
    # every uncut base triangle is equilateral; of the cut ones only corners
    # cut off by a horizontal segment can be (a smaller equilateral triangle)
    uncut = int((m.codes == 0).sum())
    assert uncut <= q["n_equilateral"] <= uncut + int((m.codes != 0).sum())
    # total area = area enclosed by the boundary polygons
    poly = abs(_shoelace_area(m.chains))
    assert abs(q["mean_area"] * n - poly) <= 1e-9 * poly
    assert abs(q["max_area"] - math.sqrt(3.0) / 4 * h * h) < 1e-12 * h * h
    if (m.codes == 0).mean() > 0.5:
        assert abs(q["ar_median"] - TWO_OVER_SQRT3) < 1e-12


def test_sampling_reproduces_linear_and_bilinear_fields():
    rs = np.random.default_rng(3)
    H, W = 37, 53
    r, c = np.mgrid[0:H, 0:W]
    lin = (2.0 + 3.0 * c - 5.0 * r).astype(np.float32)
    prod = (r * c).astype(np.float32)
    pts = np.stack([rs.uniform(0, W - 1, 400), rs.uniform(0, H - 1, 400)], 1)
    assert np.abs(oracle.sample_field(lin, pts) - (2.0 + 3.0 * pts[:, 0] - 5.0 * pts[:, 1])).max() < 1e-11
    assert np.abs(oracle.sample_field(prod, pts) - pts[:, 0] * pts[:, 1]).max() < 1e-11
    # pixel centres give the pixel values; outside points the clamped values
    cen = np.stack([c.ravel(), r.ravel()], 1).astype(np.float64)
    assert np.array_equal(oracle.sample_field(lin, cen), lin.ravel().astype(np.float64))
    out = np.array([(-3.0, 2.5), (W + 4.0, -1.0), (10.25, H + 0.5)])
    want = [2.0 + 0.0 - 12.5, 2.0 + 3.0 * (W - 1), 2.0 + 3.0 * 10.25 - 5.0 * (H - 1)]
    assert np.abs(oracle.sample_field(lin, out) - want).max() < 1e-12
    # a one-pixel field is constant
    assert np.all(oracle.sample_field(np.full((1, 1), 7.5, np.float32), pts) == 7.5)


def test_triangle_means_of_a_linear_field():
    bm = wl.disk(item=4)
    m = oracle.mesh_from_bitmap(bm, 1)
    H, W = bm.shape
    r, c = np.mgrid[0:H, 0:W]
    lin = (1.0 + 0.5 * c + 0.25 * r).astype(np.float32)
    vv, tv = oracle.sample_field(lin, m.verts, m.tris)
    cen = m.verts[m.tris].mean(axis=1)
    inside = (cen[:, 0] > 1) & (cen[:, 0] < W - 2) & (cen[:, 1] > 1) & (cen[:, 1] < H - 2)
    assert inside.mean() > 0.9
    assert np.abs(tv[inside] - (1.0 + 0.5 * cen[inside, 0] + 0.25 * cen[inside, 1])).max() < 1e-12
    bad = oracle.sample_field(lin, m.verts[:4], np.array([[0, 1, 9]], np.int32))[1]
    assert math.isnan(bad[0])


# ---------------------------------------------------------------------------
# Cotangent Laplacian and explicit heat steps.
# ---------------------------------------------------------------------------
def _hexagon():
    v = np.array([[0.0, 0.0]] + [[math.cos(k * math.pi / 3), math.sin(k * math.pi / 3)] for k in range(6)])
    t = np.array([[0, 1 + k, 1 + (k + 1) % 6] for k in range(6)], np.int32)
    return v, t


def test_laplacian_hexagon_closed_forms():
    """Six equilateral triangles around a vertex: w = cot 60 deg (twice 1/2) = 1/sqrt3, m = sqrt3/2."""
    v, t = _hexagon()
    L = oracle.laplacian(v, t)
    assert L["row_off"][1] == 6 and sorted(L["col"][:6].tolist()) == [1, 2, 3, 4, 5, 6]
    assert np.abs(L["val"][:6] - 1 / math.sqrt(3)).max() < 1e-15
    assert abs(L["mass"][0] - math.sqrt(3) / 2) < 1e-15
    assert not L["boundary"][0] and L["boundary"][1:].all() and L["n_boundary"] == 6
    # a rim vertex: two rim neighbours (one triangle each, 1/(2 sqrt3)) and the centre (two, 1/sqrt3)
    r1 = slice(L["row_off"][1], L["row_off"][2])
    got = dict(zip(L["col"][r1].tolist(), L["val"][r1].tolist()))
    assert set(got) == {0, 2, 6} and abs(got[0] - 1 / math.sqrt(3)) < 1e-15
    assert abs(got[2] - 0.5 / math.sqrt(3)) < 1e-15 and abs(got[6] - 0.5 / math.sqrt(3)) < 1e-15
    # one explicit step: u0' = u0 (1 - dt alpha sum(w) / m) = u0 (1 - 4 dt alpha), rim stays 0
    u = np.array([3.0, 0, 0, 0, 0, 0, 0])
    for dt, alpha in ((1e-3, 2.0), (0.01, 5.0)):
        got = oracle.heat_steps(v, t, u, alpha, dt, 1)
        assert abs(got[0] - 3.0 * (1 - 4 * dt * alpha)) < 1e-14 and (got[1:] == 0).all()
        got2 = oracle.heat_steps(v, t, u, alpha, dt, 2)
        assert abs(got2[0] - 3.0 * (1 - 4 * dt * alpha) ** 2) < 1e-13


def _edge_counts(t):
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e.sort(axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    return uniq, cnt


@pytest.mark.parametrize("which,h", [("disk", 1), ("ellipses", 2), ("noise", 3)])
def test_laplacian_of_meshes(which, h):
    if which == "disk":
        bm = wl.disk(item=6)
    elif which == "ellipses":
        bm = wl.ellipses(item=3)[:300, :360]
    else:
        bm = wl.smoothed_noise(240, 200, 8.0, 0.0, False, wl.rng(96, h))
    m = oracle.mesh_from_bitmap(bm, h)
    v, t = m.verts, m.tris
    L = oracle.laplacian(v, t)
    nv = v.shape[0]
    # boundary vertices: the ends of edges used by one triangle (numpy edge count)
    uniq, cnt = _edge_counts(t)
    bset = np.zeros(nv, bool)
    bset[uniq[cnt == 1].ravel()] = True
    assert np.array_equal(L["boundary"], bset)
    # rows list each neighbour once; the matrix is symmetric bit for bit
    rows = np.repeat(np.arange(nv), np.diff(L["row_off"]))
    assert L["nnz"] == 2 * uniq.shape[0]
    fwd = dict(zip(zip(rows.tolist(), L["col"].tolist()), L["val"].tolist()))
    assert all(fwd[(j, i)] == w for (i, j), w in fwd.items())
    # masses add up to the area inside the boundary polygons
    assert abs(L["mass"].sum() - abs(_shoelace_area(m.chains))) < 1e-9 * L["mass"].sum()
    # linear precision: K (a + b x + c y) = 0 at interior vertices
    lin = 0.7 - 1.3 * v[:, 0] + 2.1 * v[:, 1]
    k = oracle.laplacian_apply(v, t, lin)
    scale = np.abs(L["val"]).max() * np.abs(lin).max()
    assert np.abs(k[~L["boundary"]]).max() < 1e-9 * scale
    # x^2 + y^2 at a vertex whose six triangles are uncut equilateral ones: K u = -4 m
    par = oracle.laplacian_apply(v, t, v[:, 0] ** 2 + v[:, 1] ** 2)
    inc = np.zeros(nv, int)
    np.add.at(inc, t[m.codes == 0].ravel(), 1)
    full = inc == 6
    assert full.sum() > 10
    assert np.abs(par[full] + 4 * L["mass"][full]).max() < 1e-9 * np.abs(par[full]).max()


def test_heat_energy_decays_at_the_stable_step():
    m = oracle.mesh_from_bitmap(wl.disk(item=7), 1)
    v, t = m.verts, m.tris
    L = oracle.laplacian(v, t)
    alpha = 500.0
    dt = 1.9 / (alpha * L["lambda_bound"])
    u = oracle.heat_init(v, t, 31.5, 31.5, 6.0, 100.0)
    assert (u[L["boundary"]] == 0).all() and abs(u.max() - 100.0) < 2.0
    r2 = (v[:, 0] - 31.5) ** 2 + (v[:, 1] - 31.5) ** 2
    ok = ~L["boundary"]
    assert np.abs(u[ok] - 100.0 * np.exp(-r2[ok] / 72.0)).max() < 1e-12
    e_prev = float((L["mass"] * u * u).sum())
    for _ in range(20):
        u = oracle.heat_steps(v, t, u, alpha, dt, 5)
        e = float((L["mass"] * u * u).sum())
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e
    assert e_prev < float((L["mass"] * oracle.heat_init(v, t, 31.5, 31.5, 6.0) ** 2).sum())


def test_laplacian_skips_invalid_triangles():
    v, t = _hexagon()
    bad = np.concatenate([t, [[0, 0, 1], [0, 9, 2], [-1, 1, 2]]]).astype(np.int32)
    a, b = oracle.laplacian(v, t), oracle.laplacian(v, bad)
    assert b["n_invalid"] == 3 and a["n_invalid"] == 0
    assert np.array_equal(a["col"], b["col"]) and np.array_equal(a["val"], b["val"])
