"""Scheduling logic of the request server on a simulated device (no GPU).

The arena allocator, FIFO admission, the batch limits, the memory budget,
overlap across streams and per-request error isolation are checked against a
mock backend whose phases take a fixed time per pixel.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2602_19474_amd.serve import STATUS_NO_MEMORY, Arena, MockBackend, Server


def test_arena_first_fit_and_coalescing():
    a = Arena(4096, align=256)
    x = a.alloc(100)
    y = a.alloc(300)
    z = a.alloc(256)
    assert (x, y, z) == (0, 256, 768) and a.used == 1024
    a.free(y)
    assert a.alloc(512) == 256  # first fit reuses the hole
    a.free(256)
    a.free(x)
    a.free(z)
    assert a.used == 0 and a.largest_free() == 4096 and a._free == [(0, 4096)]
    assert a.alloc(4097) is None
    assert a.peak == 1024


def test_arena_random_sequence_never_overlaps():
    rs = np.random.default_rng(7)
    a = Arena(1 << 20, align=256)
    live = {}
    for _ in range(2000):
        if live and rs.uniform() < 0.45:
            off = list(live)[rs.integers(len(live))]
            a.free(off)
            del live[off]
        else:
            n = int(rs.integers(1, 20000))
            off = a.alloc(n)
            if off is not None:
                live[off] = (n + 255) // 256 * 256
        spans = sorted(live.items())
        for (o1, n1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + n1 <= o2
        assert a.used == sum(live.values())


class _Img:
    def __init__(self, px, tag=None):
        self.size = px
        self.tag = tag


def _sizes(r):
    px = r.bitmap.size
    if r.bitmap.tag == "bad":
        return (0, 0, 0, -6)
    if r.bitmap.tag == "huge":
        return (1 << 40, 1 << 40, 0, -7)
    return (px // 2, px, px // 50, -7)  # before emission the status is "no outputs bound"


def _drive(server, items, arrivals):
    be = server.backend
    reqs, j = [], 0
    for _ in range(1_000_000):
        while j < len(items) and arrivals[j] <= be.now():
            reqs.append(server.submit(items[j][0], items[j][1], arrival=arrivals[j]))
            j += 1
        if j == len(items) and server.idle:
            return reqs
        if not server.step():
            nxt = [arrivals[j]] if j < len(items) else []
            nxt += [t for t in be.busy_until if t > be.now()]
            assert nxt, "scheduler stalled"
            be.clock = min(nxt)
    raise AssertionError("did not finish")


def _trace(n, rate, seed=3):
    rs = np.random.default_rng(seed)
    arr = np.cumsum(rs.exponential(1.0 / rate, n))
    items = [(_Img(int(rs.integers(10_000, 200_000))), float(rs.choice([0.5, 1, 1.5, 2, 4]))) for _ in range(n)]
    return items, arr


def test_every_request_completes_in_fifo_batches():
    items, arr = _trace(400, 2000.0)
    order = []
    srv = Server(MockBackend(_sizes), budget_bytes=1 << 30, streams=2, max_batch=8,
                 on_done=lambda r: order.append(r.rid))
    reqs = _drive(srv, items, arr)
    assert all(r.done and r.status == 0 for r in reqs)
    assert srv.completed == 400 and srv.failed == 0
    assert all(r.t_done >= r.t_admit >= r.arrival for r in reqs)
    # admission is FIFO: admit times never decrease with the request id
    adm = [r.t_admit for r in sorted(reqs, key=lambda r: r.rid)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert srv.arena.used == 0 and srv.arena.peak <= srv.arena.capacity
    # grid edges reach the batch as given (dyadic ones included)
    assert [r.grid_h for r in sorted(reqs, key=lambda r: r.rid)] == [h for _, h in items]


def test_batch_limits():
    items, arr = _trace(200, 1e6)  # everything arrives at once
    sizes = []
    be = MockBackend(_sizes)
    orig = be.new_batch

    def spy(reqs, arena, slot):
        sizes.append((len(reqs), sum(r.pixels for r in reqs)))
        return orig(reqs, arena, slot)

    be.new_batch = spy
    srv = Server(be, budget_bytes=1 << 30, streams=2, max_batch=16, max_batch_pixels=1_000_000)
    _drive(srv, items, arr)
    assert max(n for n, _ in sizes) <= 16
    assert all(px <= 1_000_000 or n == 1 for n, px in sizes)
    assert srv.batches == len(sizes)


def test_budget_bounds_memory_and_forces_waits():
    items, arr = _trace(300, 1e5)
    per_req_out = 16 * 100_000 + 13 * 200_000  # largest possible outputs of one request
    budget = 3 * per_req_out + 64 * 1024
    srv = Server(MockBackend(_sizes), budget_bytes=budget, streams=4, max_batch=4)
    reqs = _drive(srv, items, arr)
    assert all(r.status == 0 for r in reqs)
    assert srv.arena.peak <= budget


def test_streams_overlap():
    items, arr = _trace(300, 1e6)
    done = {}
    for streams in (1, 2, 4):
        srv = Server(MockBackend(_sizes), budget_bytes=1 << 32, streams=streams, max_batch=8)
        reqs = _drive(srv, items, arr)
        done[streams] = max(r.t_done for r in reqs)
    assert done[2] < 0.75 * done[1] and done[4] < done[2]


def test_failures_are_isolated():
    items, arr = _trace(60, 1e4)
    items[10] = (_Img(50_000, "bad"), 1)
    items[20] = (_Img(50_000, "huge"), 2)
    srv = Server(MockBackend(_sizes), budget_bytes=1 << 30, streams=2, max_batch=8)
    reqs = _drive(srv, items, arr)
    st = {r.rid: r.status for r in reqs}
    assert st[10] == -6
    assert st[20] == STATUS_NO_MEMORY
    assert all(s == 0 for rid, s in st.items() if rid not in (10, 20))
    assert srv.completed == 58 and srv.failed == 2


@pytest.mark.parametrize("keep", [False, True])
def test_outputs_kept_until_released(keep):
    items, arr = _trace(20, 1e3)
    srv = Server(MockBackend(_sizes), budget_bytes=1 << 30, streams=2, max_batch=4, keep_outputs=keep)
    reqs = _drive(srv, items, arr)
    if keep:
        assert srv.arena.used > 0 and all(r.outputs is not None for r in reqs)
        for r in reqs:
            srv.release(r)
    assert srv.arena.used == 0
