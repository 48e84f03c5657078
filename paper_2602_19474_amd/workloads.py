"""Seeded synthetic bitmaps for the SBMT workloads.

This module holds no meshing arithmetic: it only draws random binary images.
Tests, the oracle checks and the benchmark all take their inputs from here.

Every generator is seeded with ``numpy.random.default_rng([260219474, cfg, item])``
(PCG64), so the same (cfg, item) gives the same bitmap on every machine.

Workloads (one per configuration the measurements are quoted on):

1. ``disk64``       64x64, one filled disk of radius 20 px, centre offset U(-2, 2) px
                    from the image centre; grid edge 1 px.
2. ``ellipses1024`` 1024x1024, union of 32 ellipses (centres uniform over the image,
                    semi-axes U(20, 150) px, rotation U(0, pi)), XOR 16 disks
                    (radius U(5, 30) px); grid edge 2 px.
3. ``batch256``     256 images, each side U{128..2048} px, iid N(0,1) noise smoothed
                    by a Gaussian of sigma 8 px, thresholded at 0; grid edge drawn
                    from {1, 2, 4} per image.
4. ``noise8192``    8192x8192 N(0,1) noise smoothed with sigma 16 px, z-normalised,
                    thresholded at 0.3; grid edge 1 px.
5. ``serve``        request stream: side round(exp(U(ln 256, ln 4096))), square, content
                    50/50 from the ellipse and smoothed-noise generators, grid edge
                    from {1, 2, 4}, Poisson arrivals.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

SEED_BASE = 260219474


def rng(cfg: int, item: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(cfg), int(item)])


def sha256(bitmap: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(bitmap, dtype=np.uint8).tobytes()).hexdigest()


def disk(size: int = 64, radius: float = 20.0, item: int = 0) -> np.ndarray:
    g = rng(1, item)
    cx = (size - 1) / 2.0 + g.uniform(-2.0, 2.0)
    cy = (size - 1) / 2.0 + g.uniform(-2.0, 2.0)
    yy, xx = np.mgrid[0:size, 0:size]
    return (((xx - cx) ** 2 + (yy - cy) ** 2) <= radius * radius).astype(np.uint8)


def ellipses(width: int = 1024, height: int | None = None, n_ellipses: int = 32, n_holes: int = 16,
             g: np.random.Generator | None = None, item: int = 0) -> np.ndarray:
    height = width if height is None else height
    g = rng(2, item) if g is None else g
    out = np.zeros((height, width), dtype=bool)
    for _ in range(n_ellipses):
        cx, cy = g.uniform(0, width), g.uniform(0, height)
        a, b = g.uniform(20, 150), g.uniform(20, 150)
        th = g.uniform(0, math.pi)
        c, s = math.cos(th), math.sin(th)
        x0, x1 = max(0, int(cx - max(a, b)) - 1), min(width, int(cx + max(a, b)) + 2)
        y0, y1 = max(0, int(cy - max(a, b)) - 1), min(height, int(cy + max(a, b)) + 2)
        if x0 >= x1 or y0 >= y1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dx, dy = xx - cx, yy - cy
        u = (dx * c + dy * s) / a
        v = (-dx * s + dy * c) / b
        out[y0:y1, x0:x1] |= (u * u + v * v) <= 1.0
    for _ in range(n_holes):
        cx, cy, r = g.uniform(0, width), g.uniform(0, height), g.uniform(5, 30)
        x0, x1 = max(0, int(cx - r) - 1), min(width, int(cx + r) + 2)
        y0, y1 = max(0, int(cy - r) - 1), min(height, int(cy + r) + 2)
        if x0 >= x1 or y0 >= y1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        out[y0:y1, x0:x1] ^= ((xx - cx) ** 2 + (yy - cy) ** 2) <= r * r
    return out.astype(np.uint8)


def smoothed_noise(width: int, height: int, sigma: float, threshold: float, zscore: bool,
                   g: np.random.Generator) -> np.ndarray:
    """iid N(0,1) -> separable Gaussian (truncate 4 sigma, reflect) -> threshold."""
    from scipy.ndimage import gaussian_filter

    x = g.standard_normal((height, width), dtype=np.float32)
    x = gaussian_filter(x, sigma=sigma, mode="reflect", truncate=4.0)
    if zscore:
        x = (x - x.mean(dtype=np.float64)) / x.std(dtype=np.float64)
    return (x > threshold).astype(np.uint8)


def noise8192(size: int = 8192, item: int = 0) -> np.ndarray:
    return smoothed_noise(size, size, 16.0, 0.3, True, rng(4, item))


def batch256(n: int = 256, lo: int = 128, hi: int = 2048, item0: int = 0):
    """List of (bitmap, grid_h) pairs; sizes and grid edges are seeded per image."""
    out = []
    for j in range(n):
        g = rng(3, item0 + j)
        w, h = int(g.integers(lo, hi + 1)), int(g.integers(lo, hi + 1))
        gh = int(g.choice([1, 2, 4]))
        out.append((smoothed_noise(w, h, 8.0, 0.0, False, g), gh))
    return out


def batch_shapes(n: int = 256, lo: int = 128, hi: int = 2048, item0: int = 0):
    """The (width, height, grid_h) of ``batch256`` without drawing the images."""
    out = []
    for j in range(n):
        g = rng(3, item0 + j)
        w, h = int(g.integers(lo, hi + 1)), int(g.integers(lo, hi + 1))
        out.append((w, h, int(g.choice([1, 2, 4]))))
    return out


def serve_request(item: int, lo: int = 256, hi: int = 4096):
    """One serving request: (bitmap, grid_h)."""
    g = rng(5, item)
    side = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
    gh = int(g.choice([1, 2, 4]))
    if g.uniform() < 0.5:
        bm = ellipses(side, side, g=g)
    else:
        bm = smoothed_noise(side, side, 8.0, 0.0, False, g)
    return bm, gh


def poisson_arrivals(n: int, qps: float, item: int = 0) -> np.ndarray:
    """Arrival times (s) of n requests at rate qps."""
    g = rng(6, item)
    return np.cumsum(g.exponential(1.0 / qps, size=n))
