"""The benchmark's contract on the CPU: refusal of several GPUs, seeded inputs,
and the rule that ties the roofline's measured traffic to the kernel sources.
"""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np

from paper_2602_19474_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_before_any_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_inputs_are_seeded_and_shaped():
    import bench
    a, b = bench._gen_batch_item(5), bench._gen_batch_item(5)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and a[1] in (1, 2, 4)
    for j in range(6):
        bm, gh = bench._gen_batch_item(j)
        assert bm.dtype == np.uint8 and 128 <= bm.shape[0] <= 2048 and 128 <= bm.shape[1] <= 2048
        assert 0.3 < bm.mean() < 0.7  # threshold 0 of smoothed noise: about half foreground
    d = wl.disk(item=3)
    assert d.shape == (64, 64) and wl.sha256(d) == wl.sha256(wl.disk(item=3)) != wl.sha256(wl.disk(item=4))
    e = wl.ellipses(item=1)
    assert e.shape == (1024, 1024) and 0.05 < e.mean() < 0.95
    bm, gh = wl.serve_request(7)
    assert bm.shape[0] == bm.shape[1] and 256 <= bm.shape[0] <= 4096 and gh in (1, 2, 4)
    arr = wl.poisson_arrivals(1000, 500.0)
    assert np.all(np.diff(arr) > 0) and abs(arr[-1] / 1000 - 1 / 500.0) < 0.2 / 500.0


def test_traffic_is_reported_only_for_the_profiled_sources():
    import bench
    path = os.path.join(ROOT, "profiles", "noise8192_hbm_traffic.md")
    recorded = None
    with open(path) as f:
        for line in f:
            if line.startswith("source_sha256:"):
                recorded = line.split(":", 1)[1].strip()
    assert recorded and len(recorded) == 64
    traffic, src = bench.measured_traffic()
    if recorded == bench.kernel_source_sha256():
        assert traffic is not None and traffic > 1e9 and src.endswith("noise8192_hbm_traffic.md")
    else:
        assert traffic is None and "stale" in src
