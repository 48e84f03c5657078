"""The C ABI library loads and exports every entry point declared in include/*.h.

Runs on the CPU: only host-side entry points are called (no GPU work).
"""
import ctypes
import os
import re

import pytest

from paper_2602_19474_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", n) for n in ("sbmt.h", "sbmt_post.h")]


def _declared():
    names = set()
    for h in HEADERS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(sbmt_[a-z_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsbmt.so is not built")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "sbmt_plan" in names and "sbmt_run" in names and "sbmt_mesh_async" in names
    assert "sbmt_sample_field" in names and "sbmt_mesh_quality" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    assert set(names) <= set(_lib.EXPORTS)


def test_post_entry_points_on_host(L):
    """Workspace sizing and argument checks of the mesh consumers (no launch)."""
    b0, b1 = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.sbmt_quality_workspace(0, ctypes.byref(b0)) == 0
    assert L.sbmt_quality_workspace(1_000_000, ctypes.byref(b1)) == 0
    assert b1.value - b0.value >= 8 * 1_000_000 and b0.value > 0
    assert L.sbmt_quality_workspace(-1, ctypes.byref(b0)) == -1
    f = _lib.Field(None, 0, 0, 0)
    assert L.sbmt_sample_field(None, ctypes.byref(f), None, 0, None, 0, None, None, None) == -1
    q = _lib.Quality()
    assert L.sbmt_mesh_quality(None, None, 0, None, 0, None, 0, ctypes.byref(q), None) == -1
    w0, w1 = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.sbmt_laplacian_workspace(10, 0, ctypes.byref(w0)) == 0
    assert L.sbmt_laplacian_workspace(10, 1000, ctypes.byref(w1)) == 0
    assert w1.value - w0.value >= 1000 * (12 + 24 + 48)  # incident lists, columns, values
    assert L.sbmt_laplacian_workspace(-1, 0, ctypes.byref(w0)) == -1
    c = _lib.Csr()
    assert L.sbmt_laplacian_csr(None, 0, 10, 10, ctypes.byref(c)) == -4
    info = _lib.LaplacianInfo()
    assert L.sbmt_laplacian_assemble(None, None, 0, None, 0, None, 0, ctypes.byref(info), None) == -1


def test_host_only_entry_points(L):
    import oracle
    import paper_2602_19474_amd as sbmt
    assert sbmt.num_classes() == len(oracle.class_table())
    for c in range(1, sbmt.num_classes() + 1):
        assert sbmt.class_code(c) == int(oracle.class_table()[c - 1])
    assert sbmt.class_code(0) == -1
    assert L.sbmt_status_string(-2).decode().startswith("unsupported grid_h")


def test_query_geometry_matches_the_oracle(L):
    import numpy as np

    import oracle
    import paper_2602_19474_amd as sbmt
    for (H, W, h) in ((64, 64, 1), (100, 37, 2), (5, 300, 4), (1, 1, 3), (257, 301, 5), (33, 65, 6),
                      (64, 64, 0.5), (100, 37, 0.75), (5, 300, 1.25), (40, 41, 1.5), (33, 17, 0.375),
                      (20, 12, 1.0 / 64), (9, 7, 1.0 / 256)):
        lay = sbmt.query(W, H, h)
        m = oracle.mesh_from_bitmap(np.zeros((H, W), np.uint8), h)
        assert (lay.grid_rows, lay.grid_cols, lay.stride_s) == m.grid
        assert lay.workspace_bytes > 0


def test_invalid_arguments_rejected_on_host(L):
    import paper_2602_19474_amd as sbmt
    for bad_h in (0, 7, 8, -1, 0.3, 1.0 / 3.0, 1.0 / 512, 6.5):
        with pytest.raises(sbmt.SbmtError) as e:
            sbmt.query(64, 64, bad_h)
        assert e.value.status == -2
    # exact predicates in 64-bit integers bound the image side at fine grid edges
    sbmt.query(2000, 100, 1.0 / 256)
    with pytest.raises(sbmt.SbmtError) as e:
        sbmt.query(4000, 100, 1.0 / 256)
    assert e.value.status == -2
    with pytest.raises(sbmt.SbmtError) as e:
        sbmt.query(-1, 64, 1)
    assert e.value.status == -1
    with pytest.raises(sbmt.SbmtError):
        sbmt.query(64, 64, 1, flags=8)


def test_image_marshalling_of_degenerate_strides():
    """Row/column views with stride 0 on a size-1 dimension, strided rows, empty images."""
    import numpy as np
    import torch

    import paper_2602_19474_amd as sbmt
    row = torch.from_numpy((np.arange(10) % 3 < 2).astype(np.uint8)[None, :])
    col = torch.from_numpy((np.arange(9) % 3 < 2).astype(np.uint8)[:, None])
    assert row.stride(0) == 0 and col.stride(1) == 0
    a = sbmt._image(row, 1, 0)
    assert (a.width, a.height, a.row_stride) == (10, 1, 10)
    b = sbmt._image(col, 1, 0)
    assert (b.width, b.height, b.row_stride) == (1, 9, col.stride(0))
    big = torch.zeros((5, 12), dtype=torch.uint8)
    c = sbmt._image(big[:, :7], 2, 1)
    assert (c.width, c.height, c.row_stride, c.flags) == (7, 5, 12, 1)
    e = sbmt._image(torch.zeros((0, 0), dtype=torch.uint8), 1, 0)
    assert (e.width, e.height) == (0, 0) and not e.bitmap
    with pytest.raises(ValueError):
        sbmt._image(big.t(), 1, 0)
    with pytest.raises(ValueError):
        sbmt._image(big.float(), 1, 0)
