"""GPU parity of the batched paths (multi-kernel and fused persistent) against the oracle.

Every strategy, tile height and grid size must give the same bits as the
oracle (schedule independence), also when the slow-owner record list
overflows, when one image of the batch does not fit its outputs, and on
every replay of a captured graph.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2602_19474_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _items():
    g = wl.rng(91, 0)
    imgs = [
        (wl.disk(item=3), 1),
        (wl.ellipses(item=1)[:700, :900], 2),
        (wl.smoothed_noise(301, 257, 8.0, 0.0, False, g), 1),
        (wl.smoothed_noise(640, 200, 8.0, 0.0, False, g), 4),
        (wl.smoothed_noise(129, 517, 8.0, 0.0, False, g), 2),
        (np.zeros((0, 0), np.uint8), 1),
        (np.ones((40, 33), np.uint8), 3),
        ((np.arange(999) % 5 < 3).astype(np.uint8)[None, :], 1),
        (wl.smoothed_noise(2100, 64, 4.0, 0.0, False, g), 1),
        (wl.smoothed_noise(333, 444, 6.0, 0.2, True, g), 6),
    ]
    return imgs


@pytest.fixture(scope="module")
def expected():
    return [oracle.mesh_from_bitmap(bm, h) for bm, h in _items()]


def _gpu_items():
    import torch
    return [(torch.from_numpy(np.ascontiguousarray(bm)).cuda(), h) for bm, h in _items()]


def _check(outs, sizes, expected, label):
    for i, ((v, t, c), ref) in enumerate(zip(outs, expected)):
        nv, nt = ref.verts.shape[0], ref.tris.shape[0]
        if sizes is not None:
            assert sizes[i][0] == nv and sizes[i][1] == nt and sizes[i][3] == 0, (label, i, sizes[i], nv, nt)
        tv = t[:nt].cpu().numpy()
        assert np.array_equal(tv, ref.tris), f"{label}: image {i} connectivity differs"
        assert np.array_equal(c[:nt].cpu().numpy(), ref.codes), f"{label}: image {i} codes differ"
        h = _items()[i][1]
        dv = float(np.abs(v[:nv].cpu().numpy() - ref.verts).max(initial=0.0))
        assert dv <= 1e-12 * h, (label, i, dv)


def test_plan_allocate_emit_every_tile_height(expected):
    import torch

    from paper_2602_19474_amd.batch import Batch, Tuning
    items = _gpu_items()
    for rows in (4, 8, 16):
        print(f"[gpu-batch] multi tile_rows={rows}", flush=True)
        b = Batch(items, tuning=Tuning(tile_rows=rows))
        sizes = b.plan()
        for s, ref in zip(sizes, expected):
            assert (s.n_vertices, s.n_triangles) == (ref.verts.shape[0], ref.tris.shape[0])
        outs = b.allocate(sizes)
        b.emit()
        torch.cuda.synchronize()
        _check(outs, b.sizes(), expected, f"multi{rows}")


@pytest.mark.parametrize("strategy,rows,gpc", [(0, 8, 0), (1, 4, 2), (1, 8, 2), (1, 4, 6), (1, 8, 1)])
def test_mesh_without_host_round_trip(expected, strategy, rows, gpc):
    import torch

    from paper_2602_19474_amd.batch import Batch, Tuning
    items = _gpu_items()
    print(f"[gpu-batch] mesh strategy={strategy} rows={rows} gpc={gpc}", flush=True)
    b = Batch(items, tuning=Tuning(strategy=strategy, tile_rows=rows, groups_per_cu=gpc))
    outs = b.allocate(b.plan(), slack=0.01)
    for rep in range(2):
        for v, t, c in outs:
            v.fill_(-1.0)
            t.fill_(-1)
        b.mesh()
        torch.cuda.synchronize()
        _check(outs, b.sizes(), expected, f"s{strategy}r{rows}g{gpc}#{rep}")


@pytest.mark.parametrize("strategy,rows", [(0, 8), (0, 4), (1, 4), (1, 8)])
def test_record_list_overflow(expected, strategy, rows):
    """A tiny record list: most slow owners are classified where they are needed.

    The persistent kernel runs only when every owner of a band tile has a
    record, so a persistent tuning with this list runs the multi-kernel path."""
    import torch

    from paper_2602_19474_amd.batch import Batch, Tuning
    items = _gpu_items()
    print(f"[gpu-batch] record_cap=37 strategy={strategy} rows={rows}", flush=True)
    b = Batch(items, tuning=Tuning(strategy=strategy, tile_rows=rows, groups_per_cu=2, record_cap=37))
    assert b.tuning.strategy == 0
    outs = b.allocate(b.plan())
    b.mesh()
    torch.cuda.synchronize()
    _check(outs, b.sizes(), expected, f"overflow s{strategy}r{rows}")


def test_persistent_tuning_needs_room_for_records():
    """Switching a batch laid out for the multi-kernel path (records for half of the
    owners) to the persistent kernel is refused; a batch created for the persistent
    kernel accepts every persistent tuning and the autotuner tries them."""
    import torch

    from paper_2602_19474_amd import SbmtError
    from paper_2602_19474_amd.batch import Batch, Tuning
    items = _gpu_items()[:4]
    b = Batch(items)
    with pytest.raises(SbmtError):
        b.tuning = Tuning(strategy=1, tile_rows=8, groups_per_cu=2)
    f = Batch(items, tuning=Tuning(strategy=1, tile_rows=8, groups_per_cu=2))
    assert f.tuning.strategy == 1
    f.tuning = Tuning(strategy=1, tile_rows=4, groups_per_cu=3)
    assert f.tuning.strategy == 1
    del b, f
    torch.cuda.synchronize()


@pytest.mark.parametrize("strategy", [0, 1])
def test_one_image_over_capacity(expected, strategy):
    import torch

    from paper_2602_19474_amd.batch import Batch, Tuning
    items = _gpu_items()
    print(f"[gpu-batch] capacity strategy={strategy}", flush=True)
    b = Batch(items, tuning=Tuning(strategy=strategy, tile_rows=8, groups_per_cu=2))
    sizes = b.plan()
    outs = b.allocate(sizes)
    small = 2  # the smoothed-noise image at h=1 gets one triangle too few
    v, t, c = outs[small]
    nt = t.shape[0]
    outs[small] = (v, torch.full((nt - 1, 3), -7, dtype=torch.int32, device="cuda"),
                   torch.zeros((nt - 1,), dtype=torch.uint8, device="cuda"))
    b.bind(outs)
    b.mesh()
    torch.cuda.synchronize()
    st = b.sizes()
    assert st[small][3] == -7 and st[small][1] == nt
    if strategy == 0:
        assert (outs[small][1].cpu().numpy() == -7).all()
    keep = [i for i in range(len(outs)) if i != small]
    _check([outs[i] for i in keep], [st[i] for i in keep], [expected[i] for i in keep], "capacity")


def test_graph_replays_match_eager(expected):
    import torch

    from paper_2602_19474_amd.batch import Batch, Tuning
    items = _gpu_items()
    for strategy, rows in ((0, 8), (1, 4)):
        print(f"[gpu-batch] graph strategy={strategy}", flush=True)
        b = Batch(items, tuning=Tuning(strategy=strategy, tile_rows=rows, groups_per_cu=2))
        outs = b.allocate(b.plan())
        g = b.capture()
        for rep in range(3):
            for v, t, c in outs:  # eager work between replays
                v.zero_()
                t.zero_()
                c.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            _check(outs, b.sizes(), expected, f"graph s{strategy} replay {rep}")


def test_autotuner_keeps_results(expected):
    import torch

    from paper_2602_19474_amd.batch import Batch
    items = _gpu_items()
    print("[gpu-batch] autotune", flush=True)
    b = Batch(items)
    outs = b.allocate(b.plan())
    best, ms = b.tune(reps=1)
    assert ms > 0 and best.tile_rows in (4, 8, 16)
    for v, t, c in outs:
        t.zero_()
    b.mesh()
    torch.cuda.synchronize()
    _check(outs, b.sizes(), expected, f"tuned {best}")


def test_both_sides_batch_and_batch_of_one():
    import torch

    from paper_2602_19474_amd import BOTH_SIDES
    from paper_2602_19474_amd.batch import Batch, Tuning, mesh_batch
    items = _items()[:5]
    gpu = [(torch.from_numpy(np.ascontiguousarray(bm)).cuda(), h) for bm, h in items]
    print("[gpu-batch] both sides", flush=True)
    outs = mesh_batch(gpu, flags=BOTH_SIDES)
    torch.cuda.synchronize()
    for (bm, h), (v, t, c) in zip(items, outs):
        ref = oracle.mesh_from_bitmap(bm, h, oracle.BOTH_SIDES)
        assert np.array_equal(t.cpu().numpy(), ref.tris) and np.array_equal(c.cpu().numpy(), ref.codes)
        assert float(np.abs(v.cpu().numpy() - ref.verts).max(initial=0.0)) <= 1e-12 * h
    print("[gpu-batch] batch of one, fused", flush=True)
    bm, h = items[2]
    b = Batch([gpu[2]], tuning=Tuning(strategy=1, tile_rows=4, groups_per_cu=2))
    (v, t, c), = b.allocate(b.plan())
    b.mesh()
    torch.cuda.synchronize()
    ref = oracle.mesh_from_bitmap(bm, h)
    assert b.sizes()[0][3] == 0
    assert np.array_equal(t.cpu().numpy(), ref.tris) and np.array_equal(c.cpu().numpy(), ref.codes)


@pytest.mark.parametrize("rows", [8, 4])
def test_both_sides_with_record_overflow(rows):
    """Both sides and a tiny record list: slow owners without a record are
    classified by the slow pass and emitted by the missing-record kernel,
    background sub-triangles included."""
    import torch

    from paper_2602_19474_amd import BOTH_SIDES
    from paper_2602_19474_amd.batch import Batch, Tuning
    items = _items()[:5]
    gpu = [(torch.from_numpy(np.ascontiguousarray(bm)).cuda(), h) for bm, h in items]
    print(f"[gpu-batch] both sides, record_cap=37, rows={rows}", flush=True)
    b = Batch(gpu, tuning=Tuning(strategy=0, tile_rows=rows, record_cap=37), flags=BOTH_SIDES)
    outs = b.allocate(b.plan())
    b.mesh()
    torch.cuda.synchronize()
    for i, ((bm, h), (v, t, c)) in enumerate(zip(items, outs)):
        ref = oracle.mesh_from_bitmap(bm, h, oracle.BOTH_SIDES)
        assert b.sizes()[i][3] == 0
        assert np.array_equal(t.cpu().numpy(), ref.tris) and np.array_equal(c.cpu().numpy(), ref.codes), i
        assert float(np.abs(v.cpu().numpy() - ref.verts).max(initial=0.0)) <= 1e-12 * h


@pytest.mark.parametrize("strategy", [0, 1])
def test_dyadic_grid_edges_in_one_batch(strategy):
    """Grid edges p/2^q next to integer ones in one batch (and one graph)."""
    import torch

    from paper_2602_19474_amd.batch import Batch, Tuning
    g = wl.rng(92, strategy)
    items = [(wl.smoothed_noise(181, 163, 4.0, 0.0, False, g), 0.5),
             (wl.smoothed_noise(240, 97, 5.0, 0.0, False, g), 1.25),
             (wl.disk(item=2), 1),
             (wl.smoothed_noise(150, 210, 3.0, 0.0, False, g), 0.375),
             (wl.smoothed_noise(90, 400, 6.0, 0.0, False, g), 2.5)]
    refs = [oracle.mesh_from_bitmap(bm, h) for bm, h in items]
    gpu = [(torch.from_numpy(np.ascontiguousarray(bm)).cuda(), h) for bm, h in items]
    print(f"[gpu-batch] dyadic grid edges, strategy {strategy}", flush=True)
    b = Batch(gpu, tuning=Tuning(strategy=strategy, tile_rows=8, groups_per_cu=2))
    outs = b.allocate(b.plan())
    gr = b.capture()
    for rep in range(2):
        for v, t, c in outs:
            t.fill_(-1)
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        st = b.sizes()
        for i, ((bm, h), (v, t, c), ref) in enumerate(zip(items, outs, refs)):
            assert st[i][3] == 0 and st[i][:2] == (ref.verts.shape[0], ref.tris.shape[0]), (rep, i, st[i])
            assert np.array_equal(t.cpu().numpy(), ref.tris) and np.array_equal(c.cpu().numpy(), ref.codes), (rep, i)
            assert float(np.abs(v.cpu().numpy() - ref.verts).max(initial=0.0)) <= 1e-12 * h


def test_batch_argument_errors():
    import torch

    from paper_2602_19474_amd import SbmtError
    from paper_2602_19474_amd.batch import Batch, Tuning
    t = torch.zeros((10, 10), dtype=torch.uint8, device="cuda")
    with pytest.raises(SbmtError) as e:
        Batch([(t, 1), (t, 7)])
    assert e.value.status == -2
    with pytest.raises(SbmtError) as e:
        Batch([(t, 1)], tuning=Tuning(strategy=1, tile_rows=16))
    assert e.value.status == -1
    b = Batch([(t, 1)])
    with pytest.raises(SbmtError):
        b.emit()  # nothing planned yet


@pytest.mark.slow
def test_batch256_images_through_captured_graph():
    """The first 32 images of the batch workload (sides 128..2048, h in {1, 2, 4}),
    autotuned, meshed by a captured graph and replayed; every replay is compared
    element by element with the oracle."""
    import torch

    import oracle_pool
    from paper_2602_19474_amd.batch import Batch
    items = wl.batch256(n=32)
    print(f"[gpu-batch] batch256[:32] oracle ({sum(b.size for b, _ in items) / 1e6:.1f} Mpix)", flush=True)
    refs = oracle_pool.oracle_meshes(items)
    b = Batch([(torch.from_numpy(bm).cuda(), h) for bm, h in items])
    outs = b.allocate(b.plan())
    tn, ms = b.tune(reps=1)
    print(f"[gpu-batch] tuned {tn} {ms:.3f} ms; capture", flush=True)
    g = b.capture()
    for rep in range(3):
        for v, t, c in outs:
            v.fill_(-1.0)
            t.fill_(-1)
            c.fill_(255)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        sizes = b.sizes()
        for i, ((v, t, c), ref) in enumerate(zip(outs, refs)):
            rv, rt, rc, nseg, ncut = ref
            assert sizes[i][:5] == (rv.shape[0], rt.shape[0], ncut, 0, nseg), (rep, i, sizes[i])
            assert np.array_equal(t.cpu().numpy(), rt), f"replay {rep}: image {i} connectivity"
            assert np.array_equal(c.cpu().numpy(), rc), f"replay {rep}: image {i} codes"
            dv = float(np.abs(v.cpu().numpy() - rv).max(initial=0.0))
            assert dv <= 1e-12 * items[i][1], (rep, i, dv)
        print(f"[gpu-batch] replay {rep} matches the oracle", flush=True)
