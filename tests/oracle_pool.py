"""Oracle meshes of many images in worker processes (test infrastructure).

GPU tests call this after the device is initialised, so the workers are
started with "spawn" (a fork would copy the parent's device state); they only
run the CPU oracle."""
from __future__ import annotations

import multiprocessing as mp
import os


def _one(args):
    import oracle
    bm, h, flags = args
    m = oracle.mesh_from_bitmap(bm, h, flags=flags)
    return m.verts, m.tris, m.codes, m.n_segments, m.n_cut


def oracle_meshes(items, flags: int = 0, workers: int | None = None):
    """[(verts, tris, codes, n_segments, n_cut)] for a list of (bitmap, grid_h)."""
    n = workers or min(8, os.cpu_count() or 1, max(1, len(items)))
    with mp.get_context("spawn").Pool(n) as pool:
        return pool.map(_one, [(bm, h, flags) for bm, h in items], chunksize=1)
