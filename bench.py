"""Benchmark of the SBMT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints ONE JSON line.  The headline ``value`` is output triangles/s of the
plain single-image path on the largest single-image workload (8192x8192
smoothed noise, sigma 16 px, threshold 0.3 after z-normalisation, grid edge
1 px): one step = plan (coarsen + classify/count + prefix sum + size read-back)
+ run (emit) of that image, inputs resident in HBM, outputs preallocated.

Extra objects on the same line:
  roofline      achieved algorithmic HBM bytes/s of the dominant kernel (k_emit)
                against the MI355X peak, timed with HIP events on its stream
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
  latency       p50/p99 per-image latency (plan + run + sync) of small images
  batch256      the 256-image batch workload: plain per-image loop, the
                batched path (autotuned, replayed as one captured graph) and
                the persistent fused launch at its best tuning (also a graph),
                triangles/s, MPix/s and HBM fraction
  serve         the request stream: plain path per request (FIFO, one stream)
                and the continuous-batching server, same Poisson arrivals,
                p50/p99 latency (arrival -> device completion) and throughput
  post          the consumers of the headline mesh: quality statistics, field
                sampling at the vertices, cotangent-Laplacian assembly and
                explicit heat steps, timed with HIP events, with their
                algorithmic HBM bytes and the oracle on a sample
  preprocess    the geometric preprocessing of Alg. 3 (snap, repel, edge
                elimination at the paper's thresholds) of the headline image:
                one sbmt_preprocess call timed with HIP events, its algorithmic
                HBM bytes, and the oracle's grid on a sample
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _gen_batch_item(j):
    from paper_2602_19474_amd import workloads as wl
    g = wl.rng(3, j)
    w, h = int(g.integers(128, 2049)), int(g.integers(128, 2049))
    gh = int(g.choice([1, 2, 4]))
    return wl.smoothed_noise(w, h, 8.0, 0.0, False, g), gh


def gen_batch(n: int):
    from concurrent.futures import ProcessPoolExecutor
    workers = min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_gen_batch_item, range(n), chunksize=4))


class Plain:
    """Preallocated plan/run of one image on the current stream."""

    def __init__(self, bitmap_gpu, grid_h: int):
        import torch

        import paper_2602_19474_amd as sbmt
        self.sbmt = sbmt
        self.t = bitmap_gpu
        self.h = grid_h
        self.ws = sbmt.workspace(bitmap_gpu, grid_h)
        sz = sbmt.plan(bitmap_gpu, grid_h, self.ws)
        self.sizes = sz
        dev = bitmap_gpu.device
        self.verts = torch.empty((max(sz.n_vertices, 1), 2), dtype=torch.float64, device=dev)
        self.tris = torch.empty((max(sz.n_triangles, 1), 3), dtype=torch.int32, device=dev)
        self.codes = torch.empty((max(sz.n_triangles, 1),), dtype=torch.uint8, device=dev)

    def plan(self):
        return self.sbmt.plan(self.t, self.h, self.ws)

    def run(self):
        self.sbmt.run(self.t, self.h, self.ws, self.verts, self.tris, self.codes)

    def step(self):
        self.plan()
        self.run()

    def alg_bytes(self) -> int:
        H, W = self.t.shape
        return W * H + 16 * self.sizes.n_vertices + 13 * self.sizes.n_triangles


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for fn in ("sbmt.hip", "sbmt_device.h", "sbmt_tables.h"):
        with open(os.path.join(ROOT, "paper_2602_19474_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per k_emit launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "noise8192_hbm_traffic.md")
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", "|", " ")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != kernel_source_sha256():
            return None, "profiles/noise8192_hbm_traffic.md (stale: kernel sources changed)"
        return int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"]), \
            "profiles/noise8192_hbm_traffic.md"
    except (OSError, KeyError, ValueError):
        return None, None


def headline(bm: np.ndarray, steps: int, warmup: int):
    import torch
    t = torch.from_numpy(bm).cuda()
    p = Plain(t, 1)
    for _ in range(warmup):
        p.step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        p.plan()
        ev[k][1].record()
        p.run()
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    plan_ms = float(np.mean([ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]))
    emit_ms = float(np.mean([ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]))
    sz = p.sizes
    return {"bitmap": bm, "plain": p, "wall": wall, "plan_ms": plan_ms, "emit_ms": emit_ms, "sizes": sz}


def async_section(plain, steps: int, warmup: int):
    """The headline image through sbmt_mesh_async: planning and emission queued back
    to back with no host round trip (outputs of the capacity an earlier plan gave,
    sizes left on the device and checked after the timed steps)."""
    import torch
    from paper_2602_19474_amd import _lib
    sd = torch.zeros(_lib.SIZE_WORDS, dtype=torch.int64, device=plain.t.device)

    def f():
        plain.sbmt.mesh_async(plain.t, plain.h, plain.ws, plain.verts, plain.tris, plain.codes, sd)
    for _ in range(warmup):
        f()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        f()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    st = sd.cpu().tolist()
    if st[3] != 0 or st[1] != plain.sizes.n_triangles:
        raise RuntimeError(f"sbmt_mesh_async sizes {st}")
    ms = wall / steps * 1e3
    return {"ms_per_step": ms, "event_ms_per_step": e0.elapsed_time(e1) / steps,
            "triangles_per_s": plain.sizes.n_triangles / (ms * 1e-3),
            "launch": "sbmt_mesh_async: plan and emission queued without a host round trip"}


def _event_ms(fn, reps: int) -> float:
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def post_section(plain, reps: int = 10):
    """Quality statistics, field sampling and heat steps over the headline mesh."""
    import torch

    from paper_2602_19474_amd import post
    nv, nt = plain.sizes.n_vertices, plain.sizes.n_triangles
    v, t = plain.verts[:nv], plain.tris[:nt]
    H, W = plain.t.shape
    ws = torch.empty((post.quality_workspace_bytes(nt),), dtype=torch.uint8, device="cuda")
    out = torch.empty((512,), dtype=torch.uint8, device="cuda")
    q_ms = _event_ms(lambda: post.mesh_quality_async(v, t, ws, out), reps)
    q = post.quality_from_bytes(out)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2602)
    field = torch.randn((H, W), generator=gen, dtype=torch.float32, device="cuda")
    s_ms = _event_ms(lambda: post.sample_field(field, v, t), reps)  # outputs from torch's caching allocator
    q_bytes = 12 * nt + 16 * nv                       # the mesh, read once
    s_bytes = 16 * nv + 4 * W * H + 8 * nv + 20 * nt  # vertices + field -> values; triangles -> means
    from paper_2602_19474_amd.pde import Laplacian
    torch.cuda.synchronize()
    a = time.perf_counter()
    lap = Laplacian(v, t)  # synchronous: assembles and reads back the summary
    asm_ms = (time.perf_counter() - a) * 1e3
    u = lap.heat_init((W - 1) / 2, (H - 1) / 2, min(W, H) / 8, 100.0)
    tmp = torch.empty_like(u)
    dt = 1.9 / (500.0 * lap.info["lambda_bound"])  # alpha = 500 (App. H), Gershgorin-stable step
    h_ms = _event_ms(lambda: lap.heat_steps(u, 500.0, dt, 10, tmp), reps) / 10
    nnz = int(lap.info["nnz"])
    h_bytes = 8 * (nv + 1) + 12 * nnz + 8 * nv + nv + 16 * nv  # operator + masses + flags, u in and out
    del lap, u, tmp
    res = {
        "heat": {"assemble_ms": asm_ms, "step_ms": h_ms, "nnz": nnz, "alg_bytes_per_step": h_bytes,
                 "hbm_frac": h_bytes / (h_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "alpha": 500.0, "dt": dt},
        "quality": {"ms": q_ms, "triangles_per_s": nt / (q_ms * 1e-3), "alg_bytes": q_bytes,
                    "hbm_frac": q_bytes / (q_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "stats": {k: (val.tolist() if k == "angle_hist" else val) for k, val in q.items()}},
        "sampling": {"ms": s_ms, "vertices_per_s": nv / (s_ms * 1e-3), "alg_bytes": s_bytes,
                     "hbm_frac": s_bytes / (s_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    return res


def preprocess_section(bm: np.ndarray, reps: int = 10):
    """Alg. 3 preprocessing (Steps 1-3, the paper's thresholds) of the headline
    image: the whole sbmt_preprocess call timed by events on its stream."""
    import torch

    from paper_2602_19474_amd.preprocess import Preprocessor
    t = torch.from_numpy(bm).cuda()
    pp = Preprocessor(t, 1)
    nv, nt, ns, nr, ni = pp.run()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(reps):
        ev[0].record()
        pp.run()
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    ms = float(np.median(ms))
    alg = bm.size + 17 * nv + 12 * nt  # bitmap in; vertices, on-polyline flags and triangles out
    del pp
    # the mesh of Alg. 3: the grid retriangulated against the polyline
    from paper_2602_19474_amd.preprocess import MeshPreprocessor
    mp = MeshPreprocessor(t, 1)
    mv, mt, mg, mc = mp.run()
    torch.cuda.synchronize()
    mms = []
    for _ in range(max(3, reps // 2)):
        ev[0].record()
        mp.run()
        ev[1].record()
        torch.cuda.synchronize()
        mms.append(ev[0].elapsed_time(ev[1]))
    mms = float(np.median(mms))
    malg = bm.size + 16 * mv + 13 * mt  # bitmap in; vertices, triangles and codes out
    # quality of the mesh of Alg. 3 (the bounds of Sec. 3.3.4 at full size)
    from paper_2602_19474_amd import post
    q = post.mesh_quality(mp.verts[:mv], mp.tris[:mt])
    quality = {k: q[k] for k in ("min_angle_deg", "min_area", "n_slivers", "n_equilateral", "ar_median", "ar_p95",
                                 "ar_max", "n_invalid")}
    del mp, t
    return {"ms": ms, "grid_h": 1, "thresholds": "(0.26, 0.125, 0.183) * h / sqrt(0.45)",
            "vertices": nv, "triangles": nt, "snapped": ns, "repelled": nr, "inserted": ni,
            "triangles_per_s": nt / (ms * 1e-3), "alg_bytes": alg,
            "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "mesh": {"ms": mms, "vertices": mv, "grid_vertices": mg, "triangles": mt, "cut": mc, "quality": quality,
                     "triangles_per_s": mt / (mms * 1e-3), "alg_bytes": malg,
                     "hbm_frac": malg / (mms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "kernels": "profiles/noise8192_preprocess_kernel_stats.md"}


def preprocess_cpu_baseline(bm: np.ndarray, rows: int = 2048):
    """The oracle's preprocessed grid on the first `rows` rows of the headline image."""
    import oracle
    crop = np.ascontiguousarray(bm[:rows])
    a = time.perf_counter()
    g = oracle.preprocessed_grid(crop, 1)
    dt = time.perf_counter() - a
    return {"value": g.tris.shape[0] / dt, "unit": "triangles/s", "cores": 1, "kind": "oracle",
            "sample": f"Steps 1-3 of Alg. 3 on rows 0-{rows - 1} of noise8192 ({crop.shape[1]} px wide)"}


def preprocess_mesh_cpu_baseline(bm: np.ndarray, rows: int = 512):
    """The oracle's mesh of Alg. 3 on the first `rows` rows of the headline image."""
    import oracle
    crop = np.ascontiguousarray(bm[:rows])
    a = time.perf_counter()
    m = oracle.mesh_preprocessed(crop, 1)
    dt = time.perf_counter() - a
    return {"value": m.tris.shape[0] / dt, "unit": "triangles/s", "cores": 1, "kind": "oracle",
            "sample": f"mesh of Alg. 3 on rows 0-{rows - 1} of noise8192 ({crop.shape[1]} px wide, {dt:.1f} s)"}


def post_cpu_baseline(plain, n_tri: int = 4_000_000):
    """The oracle's quality pass over the first n_tri triangles of the headline mesh."""
    import oracle
    nv, nt = plain.sizes.n_vertices, plain.sizes.n_triangles
    t = plain.tris[:min(nt, n_tri)].cpu().numpy()
    v = plain.verts[:nv].cpu().numpy()
    a = time.perf_counter()
    oracle.mesh_quality(v, t)
    dt = time.perf_counter() - a
    return {"value": t.shape[0] / dt, "unit": "triangles/s", "cores": 1, "kind": "oracle",
            "sample": f"quality statistics of the first {t.shape[0]} triangles of the noise8192 mesh"}


def latency(name: str, images, grid_h: int, repeats: int = 1):
    """Per-image latency of mesh_from_bitmap-equivalent plan + run + sync."""
    import torch

    import paper_2602_19474_amd as sbmt
    lat = []
    tri = 0
    gpu = [torch.from_numpy(b).cuda() for b in images]
    plains = [Plain(g, grid_h) for g in gpu]
    for p in plains:  # warm
        p.step()
    torch.cuda.synchronize()
    for _ in range(repeats):
        for p in plains:
            a = time.perf_counter()
            sz = p.plan()
            p.run()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - a)
            tri += sz.n_triangles
    lat = np.array(lat) * 1e3
    del sbmt
    return {"workload": name, "images": len(images), "grid_h": grid_h, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "tri_per_s": float(tri / (lat.sum() / 1e3))}


def batch_section(items, repeats: int = 5):
    import torch

    from paper_2602_19474_amd.batch import Batch
    n = len(items)
    gpu = [(torch.from_numpy(b).cuda(), gh) for b, gh in items]
    px = sum(b.size for b, _ in items)
    out = {"workload": f"batch{n}", "images": n, "mpix": px / 1e6,
           "grid_h_counts": {str(h): sum(1 for _, g in items if g == h) for h in (1, 2, 4)}}
    # plain: one plan + run per image, back to back on one stream
    plains = [Plain(g, gh) for g, gh in gpu]
    for p in plains:
        p.step()
    torch.cuda.synchronize()
    a = time.perf_counter()
    tri = 0
    for p in plains:
        tri += p.plan().n_triangles
        p.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - a
    alg = px + sum(16 * p.sizes.n_vertices + 13 * p.sizes.n_triangles for p in plains)
    out["plain"] = {"tri_per_s": tri / dt, "mpix_per_s": px / 1e6 / dt, "ms": dt * 1e3, "triangles": tri,
                    "hbm_frac": alg / dt / 1e9 / HBM_PEAK_GBS}
    del plains
    torch.cuda.empty_cache()
    # batched: plan once for the sizes, autotune, capture the whole path in a graph;
    # the batch is laid out for the persistent kernel too (records for every owner
    # of a band tile), so that the autotuner's candidates include it
    from paper_2602_19474_amd.batch import Tuning
    b = Batch(gpu, tuning=Tuning(strategy=1, tile_rows=8, groups_per_cu=2))
    sizes = b.plan()
    b.allocate(sizes)
    best, tuned_ms = b.tune(reps=3)
    g = b.capture()
    g.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    w0 = time.perf_counter()
    ev[0].record()
    for _ in range(repeats):
        g.replay()
    ev[1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) / repeats
    ms = ev[0].elapsed_time(ev[1]) / repeats
    st = b.sizes()
    assert all(x[3] == 0 for x in st), "batched path reported a failure"
    btri = sum(x[1] for x in st)
    assert btri == tri, (btri, tri)
    alg = px + sum(16 * x[0] + 13 * x[1] for x in st)
    out["batched"] = {"tri_per_s": tri / (ms * 1e-3), "mpix_per_s": px / 1e6 / (ms * 1e-3), "ms": ms,
                      "wall_ms": wall * 1e3, "triangles": tri, "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "tuning": best.__dict__, "launch": "one hipGraph replay per step",
                      "workspace_gb": b.ws.numel() / 1e9}
    out["speedup"] = out["batched"]["tri_per_s"] / out["plain"]["tri_per_s"]
    # the persistent fused launch (coarsening, then one classify-scan-emit
    # kernel): the best of its tunings, replayed as a graph like the above
    from paper_2602_19474_amd import SbmtError
    try:
        trials = []
        for rows in (4, 8):
            for gpc in (1, 2, 3):
                b.tuning = Tuning(strategy=1, tile_rows=rows, groups_per_cu=gpc)
                b.mesh()
                torch.cuda.synchronize()
                ev[0].record()
                for _ in range(2):
                    b.mesh()
                ev[1].record()
                torch.cuda.synchronize()
                trials.append((ev[0].elapsed_time(ev[1]) / 2, rows, gpc))
        _, rows, gpc = min(trials)
        b.tuning = Tuning(strategy=1, tile_rows=rows, groups_per_cu=gpc)
        gf = b.capture()
        gf.replay()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(repeats):
            gf.replay()
        ev[1].record()
        torch.cuda.synchronize()
        fms = ev[0].elapsed_time(ev[1]) / repeats
        st = b.sizes()
        assert all(x[3] == 0 for x in st) and sum(x[1] for x in st) == tri, "fused path differs"
        out["fused"] = {"ms": fms, "tri_per_s": tri / (fms * 1e-3), "mpix_per_s": px / 1e6 / (fms * 1e-3),
                        "tuning": {"tile_rows": rows, "groups_per_cu": gpc},
                        "launch": "coarsening + one persistent classify-scan-emit kernel, one hipGraph replay",
                        "vs_batched": fms / ms,
                        "trials_ms": {f"rows{r}_gpc{q}": t for t, r, q in trials}}
        del gf
    except SbmtError as e:  # the batch does not fit the persistent kernel's limits
        out["fused"] = {"skipped": str(e)}
    del b, g
    torch.cuda.empty_cache()
    return out


def _gen_serve_item(j):
    from paper_2602_19474_amd import workloads as wl
    return wl.serve_request(j)


def gen_serve_pool(n: int):
    from concurrent.futures import ProcessPoolExecutor
    workers = min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_gen_serve_item, range(n), chunksize=1))


def serve_section(pool, n_requests: int, rates=(0.5, 0.8, 1.0), budget_gb: float = 64.0, streams: int = 3):
    """Request stream over a pool of pre-generated requests sampled with replacement."""
    import torch

    from paper_2602_19474_amd import workloads as wl
    from paper_2602_19474_amd.serve import GpuBackend, Server, latency_stats, run_plain, run_trace
    gpu_pool = [(torch.from_numpy(b).cuda(), gh) for b, gh in pool]
    pick = wl.rng(7, 0).integers(0, len(pool), size=n_requests)
    items = [gpu_pool[j] for j in pick]
    px = [gpu_pool[j][0].numel() for j in pick]
    res = {"workload": f"serve{n_requests}", "requests": n_requests, "pool": len(pool),
           "mean_mpix": float(np.mean(px)) / 1e6, "budget_gb": budget_gb, "streams": streams}
    # plain saturation: back-to-back requests (all arrivals at 0)
    warm = run_plain(items[:20], np.zeros(20))
    sat = latency_stats(run_plain(items, np.zeros(n_requests)))
    r_sat = sat["req_per_s"]
    res["plain_saturation"] = {"req_per_s": r_sat, "tri_per_s": sat["tri_per_s"]}
    log(f"serve: plain saturation {r_sat:.0f} req/s")
    srv = Server(GpuBackend(0), budget_bytes=int(budget_gb * (1 << 30)), streams=streams, max_batch=64)
    run_trace(srv, items[:64], np.zeros(64))  # warm-up
    torch.cuda.synchronize()
    for f in rates:
        arr = wl.poisson_arrivals(n_requests, f * r_sat, item=int(f * 100))
        plain = latency_stats(run_plain(items, arr))
        reqs = run_trace(srv, items, arr)
        rows = [(r.arrival, r.t_done, r.sizes[1]) for r in reqs]
        served = latency_stats(rows)
        served["batches"] = srv.batches
        served["arena_peak_gb"] = srv.arena.peak / 1e9
        res[f"rate_{f:.1f}"] = {"qps": f * r_sat, "plain": plain, "served": served}
        log(f"serve: rate {f:.1f} R_sat plain p99 {plain['p99_ms']:.2f} ms served p99 {served['p99_ms']:.2f} ms")
    # served saturation
    reqs = run_trace(srv, items, np.zeros(n_requests))
    sat_s = latency_stats([(r.arrival, r.t_done, r.sizes[1]) for r in reqs])
    res["served_saturation"] = {"req_per_s": sat_s["req_per_s"], "tri_per_s": sat_s["tri_per_s"]}
    del srv
    torch.cuda.empty_cache()
    return res


def _oracle_tris(item):
    import oracle
    bm, gh = item
    return int(oracle.mesh_from_bitmap(bm, gh).tris.shape[0])


def cpu_baseline_pool(items, seconds: float = 15.0, what: str = "batch workload"):
    """The oracle over a process pool on all host cores (a sample of a many-image workload)."""
    from concurrent.futures import ProcessPoolExecutor
    cores = os.cpu_count() or 1
    done_tri, done_px, n = 0, 0, 0
    a = time.perf_counter()
    with ProcessPoolExecutor(cores) as ex:
        for j in range(0, len(items), cores):
            chunk = items[j:j + cores]
            done_tri += sum(ex.map(_oracle_tris, chunk))
            done_px += sum(b.size for b, _ in chunk)
            n += len(chunk)
            if time.perf_counter() - a > seconds:
                break
    dt = time.perf_counter() - a
    return {"value": done_tri / dt, "unit": "triangles/s", "mpix_per_s": done_px / 1e6 / dt, "cores": cores,
            "kind": "oracle", "sample": f"first {n} images of the {what}, one process per core"}


def cpu_baseline_images(name: str, images, grid_h: int, seconds: float = 5.0):
    """The oracle on one core over the latency workload's images, one after the other."""
    import oracle
    lat, tri, px = [], 0, 0
    a = time.perf_counter()
    for bm in images:
        b = time.perf_counter()
        tri += oracle.mesh_from_bitmap(bm, grid_h).tris.shape[0]
        lat.append(time.perf_counter() - b)
        px += bm.size
        if time.perf_counter() - a > seconds:
            break
    dt = time.perf_counter() - a
    lat = np.array(lat) * 1e3
    return {"value": tri / dt, "unit": "triangles/s", "mpix_per_s": px / 1e6 / dt, "cores": 1, "kind": "oracle",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "sample": f"first {len(lat)} images of the {name} workload, one after the other, single thread"}


def cpu_baseline(full: np.ndarray):
    import oracle
    bm = np.ascontiguousarray(full[:4096])
    a = time.perf_counter()
    m = oracle.mesh_from_bitmap(bm, 1)
    dt = time.perf_counter() - a
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": m.tris.shape[0] / dt, "unit": "triangles/s", "cores": 1, "kind": "oracle",
            "sample": f"top 4096x8192 band of the noise8192 workload, grid_h=1, one pass, single thread "
                      f"({m.tris.shape[0]} triangles in {dt:.2f}s; host {model or platform.processor()}, "
                      f"{os.cpu_count()} logical CPUs)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-pool", type=int, default=48)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-latency", action="store_true", help="skip the per-image latency sections")
    ap.add_argument("--no-post", action="store_true", help="skip the mesh-consumer section")
    ap.add_argument("--no-preprocess", action="store_true", help="skip the Alg. 3 preprocessing section")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (one process, one MI355X); --gpus {args.gpus} is not supported. "
              "Images are independent work units, so N GPUs would each mesh their own share.", file=sys.stderr)
        sys.exit(2)
    # every input is generated before the GPU is initialised (the batch uses a
    # process pool, whose workers must not inherit a GPU context)
    from paper_2602_19474_amd import workloads as wl
    t0 = time.time()
    noise = wl.noise8192()
    log(f"noise8192 generated in {time.time() - t0:.1f}s")
    extras = None
    if not args.no_extras:
        t0 = time.time()
        extras = {"disk64": [wl.disk(item=j) for j in range(1000)],
                  "ellipses1024": [wl.ellipses(item=j) for j in range(8)],
                  "batch": gen_batch(args.batch)}
        if not args.no_serve:
            extras["serve"] = gen_serve_pool(args.serve_pool)
        log(f"extra workloads generated in {time.time() - t0:.1f}s")
    import torch
    torch.cuda.set_device(0)
    import paper_2602_19474_amd  # noqa: F401  (fails loudly if the HIP library is missing)

    if args.copy_ref:
        # a plain elementwise kernel reading and writing exactly 1 GiB each
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    H = headline(noise, args.steps, args.warmup)
    sz = H["sizes"]
    ms = H["wall"] / args.steps * 1e3
    bm = H["bitmap"]
    emit_bytes = 16 * sz.n_vertices + 13 * sz.n_triangles
    achieved = emit_bytes / (H["emit_ms"] * 1e-3) / 1e9
    path_bytes = H["plain"].alg_bytes()
    traffic, traffic_src = measured_traffic()
    res = {
        "metric": "output triangles/s (plain single image; batched and latency below)",
        "value": sz.n_triangles / (ms * 1e-3),
        "unit": "triangles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/f64",
        "data": "synthetic",
        "config": {"workload": "noise8192", "width": int(bm.shape[1]), "height": int(bm.shape[0]), "grid_h": 1,
                   "fg_only": True, "generator": "N(0,1) -> Gaussian sigma 16 -> z-score -> > 0.3, seed 4/0"},
        "mpix_per_s": bm.size / 1e6 / (ms * 1e-3),
        "mesh": {"vertices": sz.n_vertices, "triangles": sz.n_triangles, "cut": sz.n_cut,
                 "boundary_segments": sz.n_segments},
        "plan_ms": H["plan_ms"],
        "emit_ms": H["emit_ms"],
        "path_hbm_frac": path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": "k_emit", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": traffic_src, "alg_bytes_per_launch": emit_bytes},
        "async": async_section(H["plain"], args.steps, args.warmup),
    }
    if not args.no_preprocess:
        log("preprocess section")
        res["preprocess"] = preprocess_section(noise)
        if not args.no_cpu_baseline:
            res["preprocess"]["cpu_baseline"] = preprocess_cpu_baseline(noise)
            res["preprocess"]["mesh"]["cpu_baseline"] = preprocess_mesh_cpu_baseline(noise)
    if not args.no_post:
        log("post section")
        res["post"] = post_section(H["plain"])
        if not args.no_cpu_baseline:
            res["post"]["quality"]["cpu_baseline"] = post_cpu_baseline(H["plain"])
    del H
    if extras is not None:
        if not args.no_latency:
            log("latency sections")
            res["latency"] = [
                latency("disk64", extras["disk64"], 1),
                latency("ellipses1024", extras["ellipses1024"], 2, repeats=10),
            ]
        log("batch section")
        res["batch"] = batch_section(extras["batch"])
        if "serve" in extras:
            log("serve section")
            res["serve"] = serve_section(extras["serve"], args.serve_requests)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline(noise)
        if extras is not None and not args.no_latency:
            res["latency"][0]["cpu_baseline"] = cpu_baseline_images("disk64", extras["disk64"], 1)
            res["latency"][1]["cpu_baseline"] = cpu_baseline_images("ellipses1024", extras["ellipses1024"], 2)
        if extras is not None:
            res["batch"]["cpu_baseline"] = cpu_baseline_pool(extras["batch"])
            if "serve" in extras:
                res["serve"]["cpu_baseline"] = cpu_baseline_pool(extras["serve"], what="serving request pool")
    res["inputs_sha256"] = {"noise8192": wl.sha256(noise)}
    if extras is not None:
        import hashlib
        hb = hashlib.sha256()
        for b, gh in extras["batch"]:
            hb.update(wl.sha256(b).encode())
            hb.update(bytes([gh]))
        res["inputs_sha256"]["batch"] = hb.hexdigest()
        if "serve" in extras:
            hs = hashlib.sha256()
            for b, gh in extras["serve"]:
                hs.update(wl.sha256(b).encode())
                hs.update(bytes([gh]))
            res["inputs_sha256"]["serve_pool"] = hs.hexdigest()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
