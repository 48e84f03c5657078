"""ctypes binding of libsbmt.so (the C ABI declared in include/sbmt.h and
include/sbmt_post.h).

Argument marshalling only: every step of the meshing path runs in the HIP
kernels of the library.  The library must have been built (see
``paper_2602_19474_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbmt.so")

SBMT_OK = 0
STATUS = {
    0: "ok", -1: "invalid argument", -2: "unsupported grid_h", -3: "index overflow", -4: "workspace",
    -5: "device error", -6: "protocol violation", -7: "capacity exceeded",
}
BOTH_SIDES = 1


class SbmtError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: sbmt status {status} ({STATUS.get(status, '?')})")


class Image(ctypes.Structure):
    _fields_ = [("bitmap", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("row_stride", ctypes.c_int64), ("grid_h", ctypes.c_double), ("flags", ctypes.c_uint32)]


NOALLOC_SCRATCH_BYTES = 64 << 20  # scratch of sbmt_mesh_noalloc
SIZE_WORDS = 5  # per-image device sizes record: n_vertices, n_triangles, n_cut, status, n_segments


class Sizes(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_triangles", ctypes.c_int64), ("n_cut", ctypes.c_int64),
                ("n_segments", ctypes.c_int64)]


class Layout(ctypes.Structure):
    _fields_ = [("stride_s", ctypes.c_int32), ("coarse_w", ctypes.c_int32), ("coarse_h", ctypes.c_int32),
                ("grid_rows", ctypes.c_int32), ("grid_cols", ctypes.c_int32), ("workspace_bytes", ctypes.c_size_t)]


class Outputs(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("tris", ctypes.c_void_p), ("codes", ctypes.c_void_p),
                ("vert_cap", ctypes.c_int64), ("tri_cap", ctypes.c_int64)]


STRATEGY_MULTI = 0
STRATEGY_FUSED = 1


class Tuning(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("record_cap", ctypes.c_int64)]

    def as_dict(self):
        return {"strategy": "fused" if self.strategy == STRATEGY_FUSED else "multi", "tile_rows": self.tile_rows,
                "groups_per_cu": self.groups_per_cu, "record_cap": self.record_cap}


EXPORTS = ("sbmt_create", "sbmt_destroy", "sbmt_query", "sbmt_plan", "sbmt_run", "sbmt_mesh_async",
           "sbmt_batch_create", "sbmt_batch_destroy", "sbmt_batch_bind", "sbmt_batch_plan", "sbmt_batch_emit",
           "sbmt_batch_plan_async", "sbmt_batch_host_sizes", "sbmt_mesh_noalloc",
           "sbmt_batch_mesh", "sbmt_batch_sizes", "sbmt_batch_get_tuning", "sbmt_batch_set_tuning",
           "sbmt_batch_tune", "sbmt_num_classes", "sbmt_class_code", "sbmt_status_string",
           "sbmt_sample_field", "sbmt_quality_workspace", "sbmt_mesh_quality_async", "sbmt_mesh_quality",
           "sbmt_laplacian_workspace", "sbmt_laplacian_assemble", "sbmt_laplacian_csr", "sbmt_laplacian_apply",
           "sbmt_heat_init", "sbmt_heat_steps", "sbmt_pre_query", "sbmt_preprocess",
           "sbmt_pre_mesh_query", "sbmt_preprocess_mesh")

ANGLE_BINS = 30


class LaplacianInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_boundary", ctypes.c_int64),
                ("n_invalid", ctypes.c_int64), ("min_mass", ctypes.c_double), ("lambda_bound", ctypes.c_double)]


class Csr(ctypes.Structure):
    _fields_ = [("row_off", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("mass", ctypes.c_void_p), ("boundary", ctypes.c_void_p)]


class Field(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("row_stride", ctypes.c_int64)]


class Quality(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_triangles", "n_invalid", "n_nonpositive", "n_slivers",
                                              "n_equilateral", "min_angle_tri")] + \
               [(n, ctypes.c_double) for n in ("min_angle_deg", "min_area", "max_area", "mean_area", "var_area",
                                               "ar_median", "ar_p95", "ar_max")] + \
               [("angle_hist", ctypes.c_int64 * ANGLE_BINS)]

_lib = None


def lib():
    """Load libsbmt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.sbmt_create.restype = i32
    L.sbmt_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    L.sbmt_destroy.restype = i32
    L.sbmt_destroy.argtypes = [vp]
    L.sbmt_query.restype = i32
    L.sbmt_query.argtypes = [ctypes.POINTER(Image), ctypes.POINTER(Layout)]
    L.sbmt_plan.restype = i32
    L.sbmt_plan.argtypes = [vp, ctypes.POINTER(Image), vp, sz, ctypes.POINTER(Sizes), vp]
    L.sbmt_run.restype = i32
    L.sbmt_run.argtypes = [vp, ctypes.POINTER(Image), vp, sz, vp, vp, vp, vp]
    L.sbmt_mesh_async.restype = i32
    L.sbmt_mesh_async.argtypes = [vp, ctypes.POINTER(Image), vp, sz, vp, i64, vp, vp, i64, vp, vp]
    L.sbmt_num_classes.restype = i32
    L.sbmt_num_classes.argtypes = []
    L.sbmt_class_code.restype = i32
    L.sbmt_class_code.argtypes = [i32]
    L.sbmt_status_string.restype = ctypes.c_char_p
    L.sbmt_status_string.argtypes = [i32]
    P = ctypes.POINTER
    L.sbmt_batch_create.restype = i32
    L.sbmt_batch_create.argtypes = [vp, P(Image), i32, P(Tuning), P(sz), P(vp)]
    L.sbmt_batch_destroy.restype = i32
    L.sbmt_batch_destroy.argtypes = [vp]
    L.sbmt_batch_bind.restype = i32
    L.sbmt_batch_bind.argtypes = [vp, vp, sz, P(Outputs), vp]
    L.sbmt_batch_plan.restype = i32
    L.sbmt_mesh_noalloc.restype = i32
    L.sbmt_mesh_noalloc.argtypes = [vp, ctypes.POINTER(Image), vp, i64, vp, vp, i64, vp, vp]
    L.sbmt_batch_plan.argtypes = [vp, P(Sizes), vp]
    L.sbmt_batch_plan_async.restype = i32
    L.sbmt_batch_plan_async.argtypes = [vp, vp]
    L.sbmt_batch_host_sizes.restype = i32
    L.sbmt_batch_host_sizes.argtypes = [vp, P(Sizes), P(i64)]
    L.sbmt_batch_emit.restype = i32
    L.sbmt_batch_emit.argtypes = [vp, vp, vp]
    L.sbmt_batch_mesh.restype = i32
    L.sbmt_batch_mesh.argtypes = [vp, vp, vp]
    L.sbmt_batch_sizes.restype = i32
    L.sbmt_batch_sizes.argtypes = [vp, P(Sizes), P(i64), vp]
    L.sbmt_batch_get_tuning.restype = i32
    L.sbmt_batch_get_tuning.argtypes = [vp, P(Tuning)]
    L.sbmt_batch_set_tuning.restype = i32
    L.sbmt_batch_set_tuning.argtypes = [vp, P(Tuning)]
    L.sbmt_batch_tune.restype = i32
    L.sbmt_batch_tune.argtypes = [vp, i32, P(Tuning), P(ctypes.c_float), vp]
    L.sbmt_sample_field.restype = i32
    L.sbmt_sample_field.argtypes = [vp, P(Field), vp, i64, vp, i64, vp, vp, vp]
    L.sbmt_quality_workspace.restype = i32
    L.sbmt_quality_workspace.argtypes = [i64, P(sz)]
    L.sbmt_mesh_quality_async.restype = i32
    L.sbmt_mesh_quality_async.argtypes = [vp, vp, i64, vp, i64, vp, sz, vp, vp]
    L.sbmt_mesh_quality.restype = i32
    L.sbmt_mesh_quality.argtypes = [vp, vp, i64, vp, i64, vp, sz, P(Quality), vp]
    f64 = ctypes.c_double
    L.sbmt_laplacian_workspace.restype = i32
    L.sbmt_laplacian_workspace.argtypes = [i64, i64, P(sz)]
    L.sbmt_laplacian_assemble.restype = i32
    L.sbmt_laplacian_assemble.argtypes = [vp, vp, i64, vp, i64, vp, sz, P(LaplacianInfo), vp]
    L.sbmt_laplacian_csr.restype = i32
    L.sbmt_laplacian_csr.argtypes = [vp, sz, i64, i64, P(Csr)]
    L.sbmt_laplacian_apply.restype = i32
    L.sbmt_laplacian_apply.argtypes = [vp, vp, sz, i64, i64, vp, vp, vp]
    L.sbmt_heat_init.restype = i32
    L.sbmt_heat_init.argtypes = [vp, vp, sz, vp, i64, i64, f64, f64, f64, f64, vp, vp]
    L.sbmt_heat_steps.restype = i32
    L.sbmt_heat_steps.argtypes = [vp, vp, sz, i64, i64, f64, f64, i32, vp, vp, vp]
    L.sbmt_pre_query.restype = i32
    L.sbmt_pre_query.argtypes = [P(Image), P(sz), P(i64), P(i64)]
    L.sbmt_preprocess.restype = i32
    L.sbmt_preprocess.argtypes = [vp, P(Image), f64, f64, f64, vp, sz, vp, vp, i64, vp, i64, P(i64), vp]
    L.sbmt_pre_mesh_query.restype = i32
    L.sbmt_pre_mesh_query.argtypes = [P(Image), P(sz), P(i64)]
    L.sbmt_preprocess_mesh.restype = i32
    L.sbmt_preprocess_mesh.argtypes = [vp, P(Image), f64, f64, f64, vp, sz, vp, i64, vp, vp, i64, P(i64), vp]
    _lib = L
    return L


def check(status: int, where: str):
    if status != SBMT_OK:
        raise SbmtError(status, where)
