"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds only image generators (random numbers, rectangles, step
edges, noise).  It contains none of the operator's arithmetic and imports
neither the GPU library nor the oracle.

The paper evaluates on photographs that are not available; these generators
stand in for them with the structure an edge detector meets: flat regions
(exact zero response), axis-aligned and diagonal step edges, smooth gradients
and noise.
"""
from __future__ import annotations

import math

import numpy as np

STEP_ANGLES_DEG = (0.0, 30.0, 45.0, 60.0, 90.0, 135.0)


def rect_image(h: int, w: int, seed: int, n_rects: int = 20) -> np.ndarray:
    """Uniform-random uint8 base overlaid with filled rectangles.

    Each of ``n_rects`` rectangles is painted in order, axis-aligned or rotated
    by 45 degrees with probability 1/2 each; its centre is uniform over the
    image, each side is uniform in [8, max(8, w/4)] and its intensity is
    uniform in {0..255}.
    """
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    smax = max(8.0, w / 4.0)
    for _ in range(n_rects):
        rotated = rng.random() < 0.5
        cy = rng.uniform(0, h)
        cx = rng.uniform(0, w)
        a = rng.uniform(8.0, smax)
        b = rng.uniform(8.0, smax)
        val = np.uint8(rng.integers(0, 256))
        if not rotated:
            y0 = int(max(0, math.floor(cy - a / 2)))
            y1 = int(min(h, math.ceil(cy + a / 2)))
            x0 = int(max(0, math.floor(cx - b / 2)))
            x1 = int(min(w, math.ceil(cx + b / 2)))
            if y1 > y0 and x1 > x0:
                img[y0:y1, x0:x1] = val
        else:
            r = (a + b) / (2.0 * math.sqrt(2.0)) + 1.0
            y0 = int(max(0, math.floor(cy - r)))
            y1 = int(min(h, math.ceil(cy + r)))
            x0 = int(max(0, math.floor(cx - r)))
            x1 = int(min(w, math.ceil(cx + r)))
            if y1 <= y0 or x1 <= x0:
                continue
            yy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
            xx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
            u = (xx + yy) / math.sqrt(2.0)
            v = (xx - yy) / math.sqrt(2.0)
            mask = (np.abs(u) <= a / 2) & (np.abs(v) <= b / 2)
            img[y0:y1, x0:x1][mask] = val
    return img


def field_image(h: int, w: int, seed: int, noise_sigma: float = 8.0) -> np.ndarray:
    """Smooth low-frequency field plus step edges at six angles plus Gaussian noise.

    The field is the bilinear upsampling of a 9x9 grid of values uniform in
    [32, 224]; one straight step edge per angle in ``STEP_ANGLES_DEG`` passes
    through a uniform random point with height +-U[20, 80]; noise is N(0,
    noise_sigma^2).  Values are rounded half-to-even and clamped to [0, 255].
    """
    rng = np.random.default_rng(seed)
    grid = rng.uniform(32.0, 224.0, size=(9, 9))
    gy = np.linspace(0.0, 8.0, h)
    gx = np.linspace(0.0, 8.0, w)
    iy = np.minimum(np.floor(gy).astype(np.int64), 7)
    ix = np.minimum(np.floor(gx).astype(np.int64), 7)
    fy = (gy - iy)[:, None]
    fx = (gx - ix)[None, :]
    g00 = grid[iy][:, ix]
    g01 = grid[iy][:, ix + 1]
    g10 = grid[iy + 1][:, ix]
    g11 = grid[iy + 1][:, ix + 1]
    field = (g00 * (1 - fy) * (1 - fx) + g01 * (1 - fy) * fx
             + g10 * fy * (1 - fx) + g11 * fy * fx)
    yy = np.arange(h, dtype=np.float64)[:, None]
    xx = np.arange(w, dtype=np.float64)[None, :]
    for ang in STEP_ANGLES_DEG:
        py = rng.uniform(0, h)
        px = rng.uniform(0, w)
        height = rng.uniform(20.0, 80.0) * (1.0 if rng.random() < 0.5 else -1.0)
        t = math.radians(ang)
        # the edge line runs along direction t; one side gets the step
        side = (xx - px) * (-math.sin(t)) + (yy - py) * math.cos(t)
        field = field + np.where(side > 0, height, 0.0)
    field = field + rng.normal(0.0, noise_sigma, size=(h, w))
    return np.clip(np.rint(field), 0, 255).astype(np.uint8)


def batch_sizes(count: int, seed: int, lo: int = 128, hi: int = 4096):
    """(height, width) pairs, each side uniform in {lo..hi}."""
    rng = np.random.default_rng(seed)
    hs = rng.integers(lo, hi + 1, size=count)
    ws = rng.integers(lo, hi + 1, size=count)
    return [(int(a), int(b)) for a, b in zip(hs, ws)]


def batch_images(count: int = 256, size_seed: int = 77, lo: int = 128, hi: int = 4096,
                 content_seed0: int = 1000):
    """Mixed-size batch: image i is rect_image of a random size with seed content_seed0+i."""
    return [rect_image(h, w, content_seed0 + i)
            for i, (h, w) in enumerate(batch_sizes(count, size_seed, lo, hi))]


def float_batch(b: int = 32, h: int = 1024, w: int = 1024, seed0: int = 2000) -> np.ndarray:
    """float32 (b, h, w) batch with values k/255 from rect_image with seeds seed0+i."""
    out = np.empty((b, h, w), np.float32)
    for i in range(b):
        out[i] = rect_image(h, w, seed0 + i).astype(np.float32) / np.float32(255.0)
    return out


def round_up(v: int, m: int) -> int:
    return (v + m - 1) // m * m


def pitched(img: np.ndarray, pitch: int) -> np.ndarray:
    """Copy a (h, w) uint8 image into rows of ``pitch`` bytes; returns the (h, w) view.

    The padding bytes are filled with a sentinel pattern so that any read of
    them would show in the results.
    """
    h, w = img.shape
    if pitch < w:
        raise ValueError("pitch < width")
    buf = np.full((h, pitch), 0xA5, dtype=np.uint8)
    buf[:, :w] = img
    return buf[:, :w]
