"""The request server on the GPU: each result is the same alone and in the mix.

Requests of mixed sizes, contents and grid edges go through the server with
several streams (batches overlap on the device, and a tight budget splits
batches); every mesh must equal, bit for bit, the one the plain single-image
path gives for that request alone, and a sample is checked against the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2602_19474_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _requests(n=24, seed=11):
    g = wl.rng(95, seed)
    out = []
    for j in range(n):
        side = int(round(np.exp(g.uniform(np.log(96), np.log(700)))))
        gh = int(g.choice([1, 2, 4]))
        if g.uniform() < 0.5:
            bm = wl.ellipses(side, side, g=g)
        else:
            bm = wl.smoothed_noise(side, side, 8.0, 0.0, False, g)
        out.append((bm, gh))
    return out


def _alone(reqs):
    import torch

    import paper_2602_19474_amd as sbmt
    res = []
    for bm, gh in reqs:
        v, t, c = sbmt.mesh_from_bitmap(torch.from_numpy(bm).cuda(), gh)
        res.append((v.cpu().numpy(), t.cpu().numpy(), c.cpu().numpy()))
    return res


def _served(reqs, budget, streams, max_batch):
    import torch

    from paper_2602_19474_amd.serve import GpuBackend, Server, run_trace
    got = {}

    def done(r):
        if r.status == 0:
            v, t, c = r.outputs
            got[r.rid] = (v.cpu().numpy(), t.cpu().numpy(), c.cpu().numpy())

    srv = Server(GpuBackend(0), budget_bytes=budget, streams=streams, max_batch=max_batch, on_done=done)
    items = [(torch.from_numpy(bm).cuda(), gh) for bm, gh in reqs]
    arrivals = np.linspace(0.0, 0.002, len(items))
    out = run_trace(srv, items, arrivals)
    torch.cuda.synchronize()
    return srv, out, got


@pytest.mark.parametrize("budget,streams,max_batch", [(2 << 30, 3, 6), (48 << 20, 2, 8)])
def test_alone_equals_mixed(budget, streams, max_batch):
    reqs = _requests()
    print(f"[gpu-serve] budget={budget >> 20} MiB streams={streams} max_batch={max_batch}", flush=True)
    alone = _alone(reqs)
    srv, out, got = _served(reqs, budget, streams, max_batch)
    assert srv.failed == 0 and srv.completed == len(reqs)
    assert srv.arena.peak <= budget
    for r in out:
        a = alone[r.rid]
        v, t, c = got[r.rid]
        assert np.array_equal(t, a[1]) and np.array_equal(c, a[2]), f"request {r.rid}"
        assert np.array_equal(v, a[0]), f"request {r.rid} coordinates"
        assert r.t_done >= r.arrival
    print(f"[gpu-serve] batches={srv.batches} peak={srv.arena.peak >> 20} MiB", flush=True)


def test_served_sample_matches_oracle():
    reqs = _requests(8, seed=12)
    srv, out, got = _served(reqs, 1 << 30, 2, 4)
    for r in out[:8:2]:
        bm, gh = reqs[r.rid]
        ref = oracle.mesh_from_bitmap(bm, gh)
        v, t, c = got[r.rid]
        assert np.array_equal(t, ref.tris) and np.array_equal(c, ref.codes)
        assert float(np.abs(v - ref.verts).max(initial=0.0)) <= 1e-12 * gh


@pytest.mark.slow
def test_served_requests_from_the_serving_distribution():
    """Requests drawn from the serving workload itself (square sides 256..4096
    log-uniform, ellipses or smoothed noise, h in {1, 2, 4}): served in the mix,
    each equals the oracle's mesh."""
    import oracle_pool
    items = [wl.serve_request(j) for j in range(6)]
    print("[gpu-serve] sides " + " ".join(f"{bm.shape[0]}/h{gh}" for bm, gh in items), flush=True)
    refs = oracle_pool.oracle_meshes(items)
    srv, out, got = _served(items, 8 << 30, 3, 4)
    assert srv.failed == 0 and srv.completed == len(items)
    for r in out:
        rv, rt, rc, _, _ = refs[r.rid]
        v, t, c = got[r.rid]
        assert np.array_equal(t, rt) and np.array_equal(c, rc), f"request {r.rid}"
        assert float(np.abs(v - rv).max(initial=0.0)) <= 1e-12 * items[r.rid][1]
