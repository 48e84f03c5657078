"""Continuous-batching request server over the batched SBMT path.

Requests (a bitmap on the device and its grid edge) arrive at any time.  The
scheduler loop never blocks on the device:

* admission: while a stream slot is free, the oldest arrived requests form
  the next batch, as many as fit ``max_batch`` images, ``max_batch_pixels``
  pixels and the free part of the device-memory budget (the batch workspace
  is carved out of one resident arena);
* each batch is planned asynchronously on its own stream; once its sizes are
  back, its outputs are carved out of the arena (or it waits until memory
  frees) and it is emitted on the same stream, overlapping with the batches
  on the other streams;
* a request completes at the device event that ends its batch; its outputs
  stay in the arena until it is released.

The meshing itself runs in the library's kernels; this module only schedules
and accounts memory.  ``MockBackend`` replaces the device with a simulated
clock so the scheduling logic is testable without a GPU.
"""
from __future__ import annotations

import bisect
import math
import time
from dataclasses import dataclass, field

__all__ = ["Arena", "ArenaFull", "Request", "Server", "STATUS_NO_MEMORY", "GpuBackend", "MockBackend", "run_trace", "run_plain",
           "latency_stats"]

ALIGN = 256
STATUS_NO_MEMORY = -8  # a request whose outputs can never fit the budget


class ArenaFull(Exception):
    pass


class Arena:
    """First-fit allocator of byte ranges of [0, capacity) (host bookkeeping only)."""

    def __init__(self, capacity: int, align: int = ALIGN):
        self.capacity = int(capacity)
        self.align = int(align)
        self._free = [(0, self.capacity)]  # sorted (offset, size), coalesced
        self._used = {}
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int):
        n = max(self.align, (int(nbytes) + self.align - 1) // self.align * self.align)
        for j, (off, size) in enumerate(self._free):
            if size >= n:
                if size == n:
                    self._free.pop(j)
                else:
                    self._free[j] = (off + n, size - n)
                self._used[off] = n
                self.used += n
                self.peak = max(self.peak, self.used)
                return off
        return None

    def free(self, off: int):
        n = self._used.pop(off)
        self.used -= n
        j = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(j, (off, n))
        # coalesce with the neighbours
        if j + 1 < len(self._free) and self._free[j][0] + self._free[j][1] == self._free[j + 1][0]:
            self._free[j] = (off, n + self._free[j + 1][1])
            self._free.pop(j + 1)
        if j > 0 and self._free[j - 1][0] + self._free[j - 1][1] == self._free[j][0]:
            self._free[j - 1] = (self._free[j - 1][0], self._free[j - 1][1] + self._free[j][1])
            self._free.pop(j)

    def largest_free(self) -> int:
        return max((s for _, s in self._free), default=0)


@dataclass
class Request:
    rid: int
    bitmap: object
    grid_h: float
    arrival: float
    pixels: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    status: int | None = None
    sizes: tuple | None = None       # (n_vertices, n_triangles, n_cut)
    outputs: tuple | None = None     # (verts, tris, codes) views, valid until released
    out_offs: list = field(default_factory=list)
    done: bool = False

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class _Run:
    __slots__ = ("reqs", "handle", "ws_off", "slot", "state", "token", "sizes", "n0")

    def __init__(self, reqs, handle, ws_off, slot):
        self.reqs, self.handle, self.ws_off, self.slot = reqs, handle, ws_off, slot
        self.state, self.token, self.sizes = "plan", None, None
        self.n0 = len(reqs)  # images of the batch object (requests may be split off)

    def handle_n(self) -> int:
        return self.n0


def _out_bytes(nv: int, nt: int):
    return (16 * nv, 12 * nt, nt)


class Server:
    """Continuous batching under a device-memory budget (see the module doc)."""

    def __init__(self, backend, budget_bytes: int = 64 << 30, streams: int = 2, max_batch: int = 64,
                 max_batch_pixels: int = 48 << 20, keep_outputs: bool = False, on_done=None):
        if streams < 1:
            raise ValueError("at least one stream")
        self.backend = backend
        self.arena = Arena(budget_bytes)
        backend.attach(self.arena.capacity, streams)
        self.slots = [None] * streams
        self.max_batch = int(max_batch)
        self.max_batch_pixels = int(max_batch_pixels)
        self.keep_outputs = keep_outputs
        self.on_done = on_done
        self.pending = []      # arrived, not admitted (FIFO)
        self.active = []       # _Run in admission order
        self.completed = 0
        self.failed = 0
        self.batches = 0
        self._next_id = 0

    # -- client side -----------------------------------------------------------
    def submit(self, bitmap, grid_h: float, arrival: float | None = None) -> Request:
        r = Request(self._next_id, bitmap, float(grid_h), self.backend.now() if arrival is None else float(arrival))
        r.pixels = int(self.backend.pixels(bitmap))
        self._next_id += 1
        self.pending.append(r)
        return r

    def release(self, r: Request):
        for off in r.out_offs:
            self.arena.free(off)
        r.out_offs = []
        r.outputs = None

    @property
    def idle(self) -> bool:
        return not self.pending and not self.active

    # -- scheduler ---------------------------------------------------------------
    def step(self) -> bool:
        progressed = False
        for run in list(self.active):
            progressed |= self._advance(run)
        progressed |= self._admit()
        return progressed

    def drain(self, sleep: float = 0.0):
        while not self.idle:
            if not self.step() and sleep:
                time.sleep(sleep)

    def _advance(self, run: _Run) -> bool:
        b = self.backend
        moved = False
        if run.state == "plan" and b.ready(run.token):
            run.sizes = b.sizes(run.handle)
            run.state = "wait_mem"
            moved = True
        if run.state == "wait_mem":
            moved |= self._start_emit(run)
        if run.state == "emit" and b.ready(run.token):
            t_done = b.done_time(run.token)
            for r in run.reqs:
                if r.done:
                    continue
                r.t_done = t_done
                r.done = True
                if r.status == 0:
                    self.completed += 1
                else:
                    self.failed += 1
                if self.on_done is not None:
                    self.on_done(r)
                if not self.keep_outputs:
                    self.release(r)
            self._finish(run)
            moved = True
        return moved

    def _start_emit(self, run: _Run) -> bool:
        """Carve the outputs of the batch out of the arena and emit it.  If only
        a prefix of its requests fits, that prefix is emitted and the rest go
        back to the head of the queue; if none fits and nothing in flight can
        free memory, the first request fails with STATUS_NO_MEMORY."""
        for r, (nv, nt, nc, st) in zip(run.reqs, run.sizes):
            r.status = int(st)
            r.sizes = (int(nv), int(nt), int(nc))
        got = []  # (request, offsets) of the fitting prefix
        fits_all = True
        for r in run.reqs:
            if r.status not in (0, -7):  # planning failed for this image: isolate it
                got.append((r, None))
                continue
            offs = []
            for nb in _out_bytes(*r.sizes[:2]):
                off = self.arena.alloc(nb)
                if off is None:
                    break
                offs.append(off)
            if len(offs) < 3:
                for off in offs:
                    self.arena.free(off)
                fits_all = False
                break
            got.append((r, offs))
        if not fits_all:
            n_ok = sum(1 for _, o in got if o is not None)
            in_flight = any(x.state in ("plan", "emit") for x in self.active if x is not run)
            if n_ok == 0:
                for _, o in got:
                    for off in o or ():
                        self.arena.free(off)
                if in_flight:
                    return False  # wait for memory
                first = run.reqs[len(got)]
                first.status = STATUS_NO_MEMORY
                first.t_done = self.backend.now()
                first.done = True
                self.failed += 1
                if self.on_done is not None:
                    self.on_done(first)
                got.append((first, None))
            # keep the prefix, put the rest back at the head of the queue
            rest = run.reqs[len(got):]
            run.reqs = [r for r, _ in got]
            run.sizes = run.sizes[:len(got)]
            for r in rest:
                r.status = None
                r.sizes = None
            self.pending[:0] = rest
        views = []
        for r, offs in got:
            if offs is None or r.done:
                views.append(None)
                continue
            r.out_offs = offs
            r.outputs = self.backend.views(offs, r.sizes)
            r.status = 0
            views.append(r.outputs)
        self.backend.bind_outputs(run.handle, views + [None] * (run.handle_n() - len(views)), run.slot)
        run.token = self.backend.emit(run.handle, run.slot)
        run.state = "emit"
        return True

    def _finish(self, run: _Run):
        self.backend.close(run.handle)
        self.arena.free(run.ws_off)
        self.slots[run.slot] = None
        self.active.remove(run)

    def _admit(self) -> bool:
        admitted = False
        now = self.backend.now()
        while self.pending:
            slot = next((j for j, x in enumerate(self.slots) if x is None), None)
            if slot is None:
                break
            take, px = [], 0
            for r in self.pending:
                if r.arrival > now or len(take) >= self.max_batch:
                    break
                if take and px + r.pixels > self.max_batch_pixels:
                    break
                take.append(r)
                px += r.pixels
            if not take:
                break
            run = None
            while take:
                try:
                    handle, ws_off = self.backend.new_batch(take, self.arena, slot)
                    run = _Run(take, handle, ws_off, slot)
                    break
                except ArenaFull:
                    if len(take) == 1:
                        take = []
                        break
                    take = take[: len(take) // 2]
            if run is None:
                break  # wait until memory frees
            for r in take:
                r.t_admit = now
            del self.pending[: len(take)]
            run.token = self.backend.plan(run.handle, slot)
            self.slots[slot] = run
            self.active.append(run)
            self.batches += 1
            admitted = True
        return admitted


# ---------------------------------------------------------------------------
# Backends.
# ---------------------------------------------------------------------------
class GpuBackend:
    """The library's batched path on one device, with a resident arena tensor."""

    def __init__(self, device: int = 0, tuning=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.tuning = tuning
        self.arena_t = None

    def attach(self, capacity: int, streams: int):
        torch = self.torch
        self.arena_t = torch.empty(capacity, dtype=torch.uint8, device=self.device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        torch.cuda.synchronize(self.device)
        self.t0_ev = torch.cuda.Event(enable_timing=True)
        self.t0_ev.record(self.streams[0])
        self.t0_ev.synchronize()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def pixels(self, bitmap) -> int:
        return int(bitmap.numel())

    def new_batch(self, reqs, arena: Arena, slot: int):
        from .batch import Batch
        offs = []

        def ws(nbytes):
            off = arena.alloc(nbytes)
            if off is None:
                raise ArenaFull()
            offs.append(off)
            return self.arena_t.narrow(0, off, nbytes)

        b = Batch([(r.bitmap, r.grid_h) for r in reqs], tuning=self.tuning, workspace=ws, bind=False)
        try:
            b.bind(None, self.streams[slot])
        except Exception:
            arena.free(offs[0])
            b.close()
            raise
        return b, offs[0]

    def _event(self, slot: int):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.streams[slot])
        return ev

    def plan(self, b, slot: int):
        b.plan_async(self.streams[slot])
        return self._event(slot)

    def ready(self, ev) -> bool:
        return ev.query()

    def sizes(self, b):
        sz, st = b.host_sizes()
        return [(s.n_vertices, s.n_triangles, s.n_cut, int(x)) for s, x in zip(sz, st)]

    def views(self, offs, sizes):
        torch = self.torch
        nv, nt, _ = sizes
        v = self.arena_t.narrow(0, offs[0], 16 * nv).view(torch.float64).view(nv, 2)
        t = self.arena_t.narrow(0, offs[1], 12 * nt).view(torch.int32).view(nt, 3)
        c = self.arena_t.narrow(0, offs[2], nt)
        return (v, t, c)

    def bind_outputs(self, b, views, slot: int):
        torch = self.torch
        empty = (torch.empty((0, 2), dtype=torch.float64, device=self.device),
                 torch.empty((0, 3), dtype=torch.int32, device=self.device),
                 torch.empty((0,), dtype=torch.uint8, device=self.device))
        b.bind([v if v is not None else empty for v in views], self.streams[slot])

    def emit(self, b, slot: int):
        b.emit(self.streams[slot], sizes=False)
        return self._event(slot)

    def done_time(self, ev) -> float:
        return self.t0_ev.elapsed_time(ev) / 1e3

    def close(self, b):
        b.close()


class MockBackend:
    """A simulated device: each batch phase takes a fixed time per pixel and
    phases of different streams overlap.  Sizes come from a callable."""

    def __init__(self, sizes_fn, ws_bytes_fn=lambda reqs: 1024 * len(reqs), plan_s_per_px=1e-9,
                 emit_s_per_px=2e-9):
        self.sizes_fn = sizes_fn
        self.ws_bytes_fn = ws_bytes_fn
        self.plan_s = plan_s_per_px
        self.emit_s = emit_s_per_px
        self.clock = 0.0
        self.bound = {}

    def attach(self, capacity: int, streams: int):
        self.busy_until = [0.0] * streams

    def now(self) -> float:
        return self.clock

    def advance(self, dt: float):
        self.clock += dt

    def pixels(self, bitmap) -> int:
        return int(bitmap.size)

    def new_batch(self, reqs, arena: Arena, slot: int):
        off = arena.alloc(self.ws_bytes_fn(reqs))
        if off is None:
            raise ArenaFull()
        return list(reqs), off

    def _phase(self, reqs, slot, per_px):
        start = max(self.clock, self.busy_until[slot])
        end = start + per_px * sum(r.pixels for r in reqs)
        self.busy_until[slot] = end
        return end

    def plan(self, reqs, slot):
        return self._phase(reqs, slot, self.plan_s)

    def ready(self, t_end) -> bool:
        return self.clock >= t_end

    def sizes(self, reqs):
        return [self.sizes_fn(r) for r in reqs]

    def views(self, offs, sizes):
        return tuple(offs)

    def bind_outputs(self, reqs, views, slot):
        self.bound[id(reqs)] = views

    def emit(self, reqs, slot):
        return self._phase(reqs, slot, self.emit_s)

    def done_time(self, t_end) -> float:
        return t_end

    def close(self, reqs):
        self.bound.pop(id(reqs), None)


# ---------------------------------------------------------------------------
# Drivers for measurements.
# ---------------------------------------------------------------------------
def run_trace(server: Server, items, arrivals, spin: float = 0.0):
    """Submit items [(bitmap, grid_h)] at the given arrival times (s, counted
    from the start of the run) and run the scheduler until all are done."""
    import gc
    reqs = []
    gc_was = gc.isenabled()
    gc.collect()
    gc.disable()  # no collector pauses inside the timed loop
    try:
        _trace_loop(server, items, arrivals, spin, reqs, server.backend.now())
    finally:
        if gc_was:
            gc.enable()
    return reqs


def _trace_loop(server, items, arrivals, spin, reqs, t0):
    j = 0
    n = len(items)
    while j < n or not server.idle:
        now = server.backend.now()
        while j < n and t0 + arrivals[j] <= now:
            bm, gh = items[j]
            reqs.append(server.submit(bm, gh, arrival=t0 + float(arrivals[j])))
            j += 1
        if not server.step() and spin:
            time.sleep(spin)


def run_plain(items, arrivals, device: int = 0):
    """The plain single-image path per request: FIFO, one stream, same arrivals.
    Returns [(arrival, t_done, n_triangles)] on one clock."""
    import torch

    from . import mesh_from_bitmap
    import gc
    out = []
    evs = []
    gc_was = gc.isenabled()
    gc.collect()
    gc.disable()  # no collector pauses inside the timed loop
    s = torch.cuda.current_stream(device)
    torch.cuda.synchronize(device)
    t0_ev = torch.cuda.Event(enable_timing=True)
    t0_ev.record(s)
    t0_ev.synchronize()
    t0 = time.perf_counter()
    try:
        _plain_loop(items, arrivals, t0, s, evs, mesh_from_bitmap)
    finally:
        if gc_was:
            gc.enable()
    torch.cuda.synchronize(device)
    for a, ev, nt in evs:
        out.append((a, t0_ev.elapsed_time(ev) / 1e3, nt))
    return out


def _plain_loop(items, arrivals, t0, s, evs, mesh_from_bitmap):
    import torch
    for (bm, gh), a in zip(items, arrivals):
        while time.perf_counter() - t0 < a:
            pass
        v, t, c = mesh_from_bitmap(bm, gh)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        evs.append((a, ev, int(t.shape[0])))
        del v, t, c


def latency_stats(rows):
    """rows: [(arrival, t_done, n_triangles)] -> p50/p99 latency (ms), throughput."""
    import numpy as np
    lat = np.array([d - a for a, d, _ in rows]) * 1e3
    tri = sum(nt for _, _, nt in rows)
    span = max(d for _, d, _ in rows) - min(a for a, _, _ in rows)
    return {"requests": len(rows), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "tri_per_s": tri / span, "req_per_s": len(rows) / span}
