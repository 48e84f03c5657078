"""SBMT CPU oracle -- test infrastructure only.

A plain, slow, independent CPU implementation of the meshing path of
Structured Bitmap-to-Mesh Triangulation (arXiv 2602.19474).  Only the tests,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  The product path (``paper_2602_19474_amd``) never
imports it and shares no code with it.

The arithmetic lives in ``sbmt_oracle.cpp`` (exact Z[sqrt3] predicates, a
segment-driven crossing registry, ray-parity labelling, procedural templates,
brute-force class enumeration).  This module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbmt_oracle.cpp")
_SRC_POST = os.path.join(_HERE, "post_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BOTH_SIDES = 1


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, no FMA contraction)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_POST))
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, _SRC_POST])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


class LocalResult(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("tok", ctypes.c_int32 * 4), ("code", ctypes.c_int32),
                ("canon_code", ctypes.c_int32), ("rot", ctypes.c_int32), ("class_id", ctypes.c_int32),
                ("paper_m", ctypes.c_int32), ("paper_n", ctypes.c_int32), ("n_tris", ctypes.c_int32),
                ("tris", (ctypes.c_int32 * 4) * 5), ("slot_seg", ctypes.c_int32 * 6),
                ("slot_xy", (ctypes.c_double * 2) * 6), ("chain_vertex", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        L.oracle_mesh_from_bitmap.restype = vp
        L.oracle_mesh_from_bitmap.argtypes = [vp, i32, i32, i64, ctypes.c_double, u32, ctypes.c_char_p, i32]
        for name in ("oracle_n_vertices", "oracle_n_triangles", "oracle_n_segments", "oracle_n_cut",
                     "oracle_n_contours"):
            getattr(L, name).restype = i64
            getattr(L, name).argtypes = [vp]
        L.oracle_grid_dims.restype = None
        L.oracle_grid_dims.argtypes = [vp, vp, vp, vp]
        L.oracle_copy.restype = None
        L.oracle_copy.argtypes = [vp, vp, vp, vp]
        L.oracle_copy_chains.restype = None
        L.oracle_copy_chains.argtypes = [vp, vp, vp]
        L.oracle_free.restype = None
        L.oracle_free.argtypes = [vp]
        L.oracle_class_table.restype = i32
        L.oracle_class_table.argtypes = [vp, i32]
        L.oracle_template_of_code.restype = i32
        L.oracle_template_of_code.argtypes = [i32, vp]
        L.oracle_mesh_preprocessed.restype = vp
        L.oracle_mesh_preprocessed.argtypes = [vp, i32, i32, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_char_p, i32]
        L.oracle_pre_grid.restype = vp
        L.oracle_pre_grid.argtypes = L.oracle_mesh_preprocessed.argtypes
        for name in ("oracle_pre_n_vertices", "oracle_pre_n_triangles"):
            getattr(L, name).restype = i64
            getattr(L, name).argtypes = [vp]
        L.oracle_pre_counts.restype = None
        L.oracle_pre_counts.argtypes = [vp, vp]
        L.oracle_pre_copy.restype = None
        L.oracle_pre_copy.argtypes = [vp, vp, vp, vp]
        L.oracle_pre_free.restype = None
        L.oracle_pre_free.argtypes = [vp]
        L.oracle_pre_grid_sizes.restype = None
        L.oracle_pre_grid_sizes.argtypes = [vp, vp]
        L.oracle_pre_grid_copy.restype = None
        L.oracle_pre_grid_copy.argtypes = [vp, vp, vp, vp]
        L.oracle_canonical.restype = i32
        L.oracle_canonical.argtypes = [i32, vp, vp]
        L.oracle_z3_sign.restype = i32
        L.oracle_z3_sign.argtypes = [i64, i64]
        L.oracle_local.restype = i32
        L.oracle_local.argtypes = [vp, vp, i32, ctypes.c_double, ctypes.POINTER(LocalResult),
                                   ctypes.c_char_p, i32]
        L.oracle_sample_field.restype = None
        L.oracle_sample_field.argtypes = [vp, i32, i32, i64, vp, i64, vp, i64, vp, vp]
        L.oracle_laplacian.restype = None
        L.oracle_laplacian.argtypes = [vp, i64, vp, i64, vp, vp, vp, vp, vp, ctypes.POINTER(LapInfo)]
        L.oracle_laplacian_apply.restype = None
        L.oracle_laplacian_apply.argtypes = [vp, i64, vp, i64, vp, vp]
        L.oracle_heat_init.restype = None
        L.oracle_heat_init.argtypes = [vp, i64, vp, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, vp]
        L.oracle_heat_steps.restype = None
        L.oracle_heat_steps.argtypes = [vp, i64, vp, i64, ctypes.c_double, ctypes.c_double, i32, vp]
        L.oracle_mesh_quality.restype = None
        L.oracle_mesh_quality.argtypes = [vp, i64, vp, i64, ctypes.POINTER(QualityOut)]
        _lib = L
    return _lib


class QualityOut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_triangles", "n_invalid", "n_nonpositive", "n_slivers",
                                              "n_equilateral", "min_angle_tri")] + \
               [(n, ctypes.c_double) for n in ("min_angle_deg", "min_area", "max_area", "mean_area", "var_area",
                                               "ar_median", "ar_p95", "ar_max")] + \
               [("angle_hist", ctypes.c_int64 * 30)]


class LapInfo(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("n_boundary", ctypes.c_int64), ("n_invalid", ctypes.c_int64),
                ("min_mass", ctypes.c_double), ("lambda_bound", ctypes.c_double)]


class OracleError(RuntimeError):
    pass


@dataclass
class OracleMesh:
    verts: np.ndarray        # float64 [V, 2]  (x, y) pixel units, pixel (r, c) centred at (c, r)
    tris: np.ndarray         # int32 [T, 3]    positive orientation in (x, y)
    codes: np.ndarray        # uint8 [T]       0 = uncut, 1..K = class id, bit 7 = background side
    n_segments: int
    n_cut: int
    n_contours: int
    chains: list             # list of int64 [n, 2] closed polylines in quarter-pixel units
    grid: tuple              # (NK, NI, s)


def mesh_from_bitmap(bitmap: np.ndarray, grid_h, flags: int = 0) -> OracleMesh:
    """Oracle mesh of a uint8 bitmap (nonzero = foreground) at grid edge ``grid_h``
    (a dyadic rational p / 2^q, q <= 8, in pixels)."""
    L = lib()
    bm = np.ascontiguousarray(bitmap, dtype=np.uint8)
    H, W = bm.shape
    err = ctypes.create_string_buffer(512)
    ptr = bm.ctypes.data if bm.size else None
    res = L.oracle_mesh_from_bitmap(ptr, W, H, W, float(grid_h), int(flags), err, 512)
    if not res:
        raise OracleError(err.value.decode())
    try:
        nv, nt = L.oracle_n_vertices(res), L.oracle_n_triangles(res)
        verts = np.zeros((nv, 2), np.float64)
        tris = np.zeros((nt, 3), np.int32)
        codes = np.zeros((nt,), np.uint8)
        L.oracle_copy(res, verts.ctypes.data, tris.ctypes.data, codes.ctypes.data)
        nc = L.oracle_n_contours(res)
        ns = L.oracle_n_segments(res)
        xy = np.zeros((ns, 2), np.int64)
        starts = np.zeros((nc + 1,), np.int64)
        L.oracle_copy_chains(res, xy.ctypes.data, starts.ctypes.data)
        chains = [xy[starts[j]:starts[j + 1]].copy() for j in range(nc)]
        nk, ni, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.oracle_grid_dims(res, ctypes.byref(nk), ctypes.byref(ni), ctypes.byref(s))
        return OracleMesh(verts, tris, codes, ns, L.oracle_n_cut(res), nc, chains,
                          (nk.value, ni.value, s.value))
    finally:
        L.oracle_free(res)


# Thresholds of the paper's experiments at base edge sqrt(0.45) (Sec. 4):
# snap a, edge elimination b, foot projection c.
PAPER_THRESHOLDS = (0.26, 0.125, 0.183)
PAPER_EDGE = 0.45 ** 0.5


@dataclass
class PreMesh:
    verts: np.ndarray   # float64 [V, 2], sorted by (y, x)
    tris: np.ndarray    # int32 [T, 3], rotated to the smallest index, sorted
    codes: np.ndarray   # uint8 [T]: 0 uncut base triangle, 1 piece of a cut one
    n_snapped: int
    n_repelled: int
    n_inserted: int
    n_cut: int
    thresholds: tuple


def mesh_preprocessed(bitmap: np.ndarray, grid_h, a=None, b=None, c=None) -> PreMesh:
    """Foreground mesh after the preprocessing of Alg. 3 (snap a, repel c, edge
    elimination b; pixels).  Defaults: the paper's thresholds scaled by
    grid_h / sqrt(0.45)."""
    L = lib()
    sc = float(grid_h) / PAPER_EDGE
    a = PAPER_THRESHOLDS[0] * sc if a is None else float(a)
    b = PAPER_THRESHOLDS[1] * sc if b is None else float(b)
    c = PAPER_THRESHOLDS[2] * sc if c is None else float(c)
    bm = np.ascontiguousarray(bitmap, dtype=np.uint8)
    H, W = bm.shape
    err = ctypes.create_string_buffer(512)
    res = L.oracle_mesh_preprocessed(bm.ctypes.data if bm.size else None, W, H, W, float(grid_h), a, b, c, err, 512)
    if not res:
        raise OracleError(err.value.decode())
    try:
        nv, nt = L.oracle_pre_n_vertices(res), L.oracle_pre_n_triangles(res)
        verts = np.zeros((nv, 2), np.float64)
        tris = np.zeros((nt, 3), np.int32)
        codes = np.zeros((nt,), np.uint8)
        L.oracle_pre_copy(res, verts.ctypes.data, tris.ctypes.data, codes.ctypes.data)
        cnt = np.zeros(4, np.int64)
        L.oracle_pre_counts(res, cnt.ctypes.data)
        return PreMesh(verts, tris, codes, *(int(x) for x in cnt), (a, b, c))
    finally:
        L.oracle_pre_free(res)


@dataclass
class PreGrid:
    verts: np.ndarray        # (V, 2) float64: lattice vertices k NI + i, then the inserted points
    on_polyline: np.ndarray  # (V,) uint8: the vertex sits on a polyline vertex (snapped or inserted)
    tris: np.ndarray         # (T, 3) int64: live triangles of the preprocessed grid
    n_snapped: int
    n_repelled: int
    n_inserted: int
    thresholds: tuple


def preprocessed_grid(bitmap: np.ndarray, grid_h, a=None, b=None, c=None) -> PreGrid:
    """The grid after Steps 1-3 of Alg. 3 (vertex snapping a, repulsion c, edge
    elimination b), before the retriangulation against the polyline."""
    L = lib()
    sc = float(grid_h) / PAPER_EDGE
    a = PAPER_THRESHOLDS[0] * sc if a is None else float(a)
    b = PAPER_THRESHOLDS[1] * sc if b is None else float(b)
    c = PAPER_THRESHOLDS[2] * sc if c is None else float(c)
    bm = np.ascontiguousarray(bitmap, dtype=np.uint8)
    H, W = bm.shape
    err = ctypes.create_string_buffer(512)
    res = L.oracle_pre_grid(bm.ctypes.data if bm.size else None, W, H, W, float(grid_h), a, b, c, err, 512)
    if not res:
        raise OracleError(err.value.decode())
    try:
        sz = np.zeros(2, np.int64)
        L.oracle_pre_grid_sizes(res, sz.ctypes.data)
        verts = np.zeros((int(sz[0]), 2), np.float64)
        onp = np.zeros((int(sz[0]),), np.uint8)
        tris = np.zeros((int(sz[1]), 3), np.int64)
        L.oracle_pre_grid_copy(res, verts.ctypes.data, onp.ctypes.data, tris.ctypes.data)
        cnt = np.zeros(4, np.int64)
        L.oracle_pre_counts(res, cnt.ctypes.data)
        return PreGrid(verts, onp, tris, int(cnt[0]), int(cnt[1]), int(cnt[2]), (a, b, c))
    finally:
        L.oracle_pre_free(res)


def class_table() -> np.ndarray:
    """Admissible canonical key codes, ascending; class id = 1 + index."""
    L = lib()
    buf = np.zeros(4096, np.int32)
    n = L.oracle_class_table(buf.ctypes.data, 4096)
    return buf[:n].copy()


def z3_sign(a: int, b: int) -> int:
    """Exact sign of a + b*sqrt(3) as the oracle decides it."""
    return int(lib().oracle_z3_sign(int(a), int(b)))


def canonical(code: int):
    """(class id, canonical code, rotation tag) of a raw key code, or None if inadmissible."""
    cc, rot = ctypes.c_int32(), ctypes.c_int32()
    cls = lib().oracle_canonical(int(code), ctypes.byref(cc), ctypes.byref(rot))
    if cls < 0:
        return None
    return int(cls), int(cc.value), int(rot.value)


def template_of_code(code: int):
    """Procedural template (both sides) of a key code: list of (a, b, c, side)."""
    L = lib()
    buf = np.zeros(5 * 4, np.int32)
    n = L.oracle_template_of_code(int(code), buf.ctypes.data)
    if n < 0:
        return None
    return [tuple(int(v) for v in buf[4 * j:4 * j + 4]) for j in range(n)]


def local(corners, chain, unit: float):
    """Classify and retriangulate one triangle against a polyline.

    ``corners``: 3 x (x, ya, yb) integers, y = ya + yb*sqrt(3), positive orientation.
    ``chain``: m x (x, y) integers.  All coordinates share the scale ``unit``
    (value = integer / unit).  Returns a ``LocalResult`` or raises; a degenerate
    contact (a vertex on an edge) raises ``ValueError``.
    """
    L = lib()
    c = np.ascontiguousarray(np.asarray(corners, dtype=np.int64).reshape(3, 3))
    p = np.ascontiguousarray(np.asarray(chain, dtype=np.int64).reshape(-1, 2))
    out = LocalResult()
    err = ctypes.create_string_buffer(512)
    rc = L.oracle_local(c.ctypes.data, p.ctypes.data, p.shape[0], float(unit), ctypes.byref(out), err, 512)
    if rc == -2:
        raise ValueError("degenerate contact")
    if rc != 0:
        raise OracleError(err.value.decode())
    return out


def sample_field(field: np.ndarray, verts: np.ndarray, tris: np.ndarray | None = None):
    """Bilinear field values at the vertices (and per-triangle means if ``tris``)."""
    L = lib()
    f = np.ascontiguousarray(field, dtype=np.float32)
    H, W = f.shape
    v = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 2)
    vv = np.zeros(v.shape[0], np.float64)
    if tris is None:
        L.oracle_sample_field(f.ctypes.data, W, H, W, v.ctypes.data, v.shape[0], None, 0, vv.ctypes.data, None)
        return vv
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    tv = np.zeros(t.shape[0], np.float64)
    L.oracle_sample_field(f.ctypes.data, W, H, W, v.ctypes.data, v.shape[0], t.ctypes.data if t.size else None,
                          t.shape[0], vv.ctypes.data, tv.ctypes.data)
    return vv, tv


def mesh_quality(verts: np.ndarray, tris: np.ndarray) -> dict:
    """Quality statistics of a mesh (see post_oracle.cpp for the definitions)."""
    L = lib()
    v = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 2)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    out = QualityOut()
    L.oracle_mesh_quality(v.ctypes.data if v.size else None, v.shape[0], t.ctypes.data if t.size else None,
                          t.shape[0], ctypes.byref(out))
    d = {n: getattr(out, n) for n, _ in QualityOut._fields_ if n != "angle_hist"}
    d["angle_hist"] = np.array(out.angle_hist[:], np.int64)
    return d


def _mesh_args(verts, tris):
    v = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 2)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    return v, t, (v.ctypes.data if v.size else None), (t.ctypes.data if t.size else None)


def laplacian(verts: np.ndarray, tris: np.ndarray) -> dict:
    """Cotangent stiffness rows (CSR), lumped masses and boundary flags."""
    L = lib()
    v, t, vp_, tp_ = _mesh_args(verts, tris)
    info = LapInfo()
    L.oracle_laplacian(vp_, v.shape[0], tp_, t.shape[0], None, None, None, None, None, ctypes.byref(info))
    nv = v.shape[0]
    row_off = np.zeros(nv + 1, np.int64)
    col = np.zeros(max(info.nnz, 1), np.int32)
    val = np.zeros(max(info.nnz, 1), np.float64)
    mass = np.zeros(max(nv, 1), np.float64)
    bnd = np.zeros(max(nv, 1), np.uint8)
    L.oracle_laplacian(vp_, nv, tp_, t.shape[0], row_off.ctypes.data, col.ctypes.data, val.ctypes.data,
                       mass.ctypes.data, bnd.ctypes.data, ctypes.byref(info))
    return {"row_off": row_off, "col": col[:info.nnz], "val": val[:info.nnz], "mass": mass[:nv],
            "boundary": bnd[:nv].astype(bool), "nnz": info.nnz, "n_boundary": info.n_boundary,
            "n_invalid": info.n_invalid, "min_mass": info.min_mass, "lambda_bound": info.lambda_bound}


def laplacian_apply(verts, tris, u) -> np.ndarray:
    L = lib()
    v, t, vp_, tp_ = _mesh_args(verts, tris)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    y = np.zeros_like(uu)
    L.oracle_laplacian_apply(vp_, v.shape[0], tp_, t.shape[0], uu.ctypes.data, y.ctypes.data)
    return y


def heat_init(verts, tris, x0: float, y0: float, sigma: float, amp: float = 100.0) -> np.ndarray:
    L = lib()
    v, t, vp_, tp_ = _mesh_args(verts, tris)
    u = np.zeros(v.shape[0], np.float64)
    L.oracle_heat_init(vp_, v.shape[0], tp_, t.shape[0], x0, y0, sigma, amp, u.ctypes.data)
    return u


def heat_steps(verts, tris, u, alpha: float, dt: float, steps: int) -> np.ndarray:
    L = lib()
    v, t, vp_, tp_ = _mesh_args(verts, tris)
    uu = np.array(u, dtype=np.float64, copy=True)
    L.oracle_heat_steps(vp_, v.shape[0], tp_, t.shape[0], alpha, dt, int(steps), uu.ctypes.data)
    return uu
