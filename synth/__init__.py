"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only *makes inputs*; it holds none of the reconstruction's
arithmetic, and neither the oracle nor the GPU library imports the other
through it.

The paper's workload is 4K x 4K tiles cut from glioblastoma whole-slide images
(Sec. V-A).  That dataset is not available, so nuclei-like tiles stand in for
it: a sum of isotropic 2-D Gaussians (bright blobs of nucleus size) over a
background with uniform integer noise, clipped to uint8.  Markers follow the
h-dome form ``max(I - h, 0)`` used for nucleus candidates; fill-holes runs on a
thresholded binary copy.  Adversarial "spiral corridor" masks (one 1-pixel
wide corridor winding to the centre) give the longest propagation chain a
tile of a given size can have.

Recipe (all draws from ``numpy.random.default_rng(seed)``, PCG64, in this
order): centres y ~ U[0, H), x ~ U[0, W) (vectors of length n), then sigma ~
U[s_lo, s_hi], then amplitude ~ U[a_lo, a_hi]; each Gaussian is accumulated
in float64 over a window of +-ceil(4 sigma) pixels around its centre; the sum
is rounded (numpy.rint), the background added, then integer noise
``rng.integers(n_lo, n_hi + 1)`` per pixel, and the result clipped to 0..255.
"""
from __future__ import annotations

import math

import numpy as np

SIZES_CFG4 = tuple(range(512, 4096 + 1, 256))  # 512, 768, ..., 4096 (15 values)


def seed_for(config: int, index: int) -> int:
    """Seed of tile ``index`` of workload ``config`` (1-based config number)."""
    return 1_000_000 * int(config) + int(index)


def gaussian_tile(h: int, w: int, n_gauss: int, sigma=(4.0, 12.0), amp=(40.0, 200.0),
                  background: int = 0, noise=(-8, 8), seed: int = 0) -> np.ndarray:
    """Sum of ``n_gauss`` random Gaussians plus background and noise, as uint8 (h, w)."""
    rng = np.random.default_rng(seed)
    cy = rng.uniform(0.0, h, size=n_gauss)
    cx = rng.uniform(0.0, w, size=n_gauss)
    sg = rng.uniform(sigma[0], sigma[1], size=n_gauss)
    am = rng.uniform(amp[0], amp[1], size=n_gauss)
    acc = np.zeros((h, w), dtype=np.float64)
    for i in range(n_gauss):
        r = int(math.ceil(4.0 * sg[i]))
        y0 = max(int(math.floor(cy[i])) - r, 0)
        y1 = min(int(math.floor(cy[i])) + r + 1, h)
        x0 = max(int(math.floor(cx[i])) - r, 0)
        x1 = min(int(math.floor(cx[i])) + r + 1, w)
        if y0 >= y1 or x0 >= x1:
            continue
        gy = np.exp(-((np.arange(y0, y1) - cy[i]) ** 2) / (2.0 * sg[i] ** 2))
        gx = np.exp(-((np.arange(x0, x1) - cx[i]) ** 2) / (2.0 * sg[i] ** 2))
        acc[y0:y1, x0:x1] += am[i] * np.outer(gy, gx)
    img = np.rint(acc).astype(np.int32) + int(background)
    img += rng.integers(noise[0], noise[1] + 1, size=(h, w), dtype=np.int32)
    return np.clip(img, 0, 255).astype(np.uint8)


def hdome_marker(mask: np.ndarray, h: int) -> np.ndarray:
    """Marker ``max(I - h, 0)`` as uint8."""
    return np.clip(mask.astype(np.int32) - int(h), 0, 255).astype(np.uint8)


# ---- the five workloads -------------------------------------------------------

def config1_tile(seed: int = seed_for(1, 0)):
    """512 x 512 tile: 40 Gaussians, sigma U[4,12], amplitude U[40,200], noise [-8,8].

    Returns (marker, mask) with marker = max(I - 30, 0); 8-connectivity."""
    mask = gaussian_tile(512, 512, 40, (4.0, 12.0), (40.0, 200.0), 0, (-8, 8), seed)
    return hdome_marker(mask, 30), mask


def scaled_config1_tile(h: int, w: int, seed: int):
    """The 512 x 512 generator scaled to an h x w tile (Gaussian count ~ area)."""
    n = int(round(40.0 * h * w / (512.0 * 512.0)))
    return gaussian_tile(h, w, n, (4.0, 12.0), (40.0, 200.0), 0, (-8, 8), seed)


def config2_tile(seed: int = seed_for(2, 0), size: int = 4096, n_gauss: int = 3000):
    """4096 x 4096 nuclei-like tile: ~3000 Gaussians, sigma U[3,8], amplitude U[60,220],
    background 30, noise [-10,10].

    Returns (marker, mask, binary) with marker = max(I - 20, 0) and
    binary = 255 * (I > 120) for fill-holes.  ``size``/``n_gauss`` shrink it
    at constant density for quick tests."""
    mask = gaussian_tile(size, size, n_gauss, (3.0, 8.0), (60.0, 220.0), 30, (-10, 10), seed)
    binary = np.where(mask > 120, 255, 0).astype(np.uint8)
    return hdome_marker(mask, 20), mask, binary


def spiral_path(h: int, w: int) -> np.ndarray:
    """Cells (y, x) of a one-pixel corridor spiralling clockwise from (0, 0) inwards.

    Consecutive rings are two pixels apart (one-pixel walls).  The path is a
    single chain under both 4- and 8-connectivity: no two cells three or more
    steps apart along it are 8-adjacent (checked here; the path is cut before
    the first cell that would break this near the centre)."""
    segs = []
    k = 0
    while True:
        xs = 0 if k == 0 else k - 1
        xe = w - 1 - k
        if k > h - 1 - k or xe < xs:
            break
        segs.append(np.stack([np.full(xe - xs + 1, k), np.arange(xs, xe + 1)], 1))
        ys, ye = k + 1, h - 1 - k
        if ye < ys:
            break
        segs.append(np.stack([np.arange(ys, ye + 1), np.full(ye - ys + 1, xe)], 1))
        xs2, xe2 = xe - 1, k
        if xs2 < xe2:
            break
        segs.append(np.stack([np.full(xs2 - xe2 + 1, ye), np.arange(xs2, xe2 - 1, -1)], 1))
        ys3, ye3 = ye - 1, k + 2
        if ys3 < ye3:
            break
        segs.append(np.stack([np.arange(ys3, ye3 - 1, -1), np.full(ys3 - ye3 + 1, k)], 1))
        k += 2
    path = np.concatenate(segs, 0).astype(np.int64)
    # Cut the path before the first cell that touches an earlier, non-adjacent cell.
    idx = np.full((h + 2, w + 2), -1, dtype=np.int64)
    cut = len(path)
    order = np.arange(len(path))
    # duplicates: keep the first visit only
    flat = path[:, 0] * w + path[:, 1]
    _, first = np.unique(flat, return_index=True)
    if len(first) != len(path):
        dup = np.setdiff1d(order, first)
        cut = min(cut, int(dup.min()))
    idx[path[:cut, 0] + 1, path[:cut, 1] + 1] = order[:cut]
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            nb = idx[path[:cut, 0] + 1 + dy, path[:cut, 1] + 1 + dx]
            bad = (nb >= 0) & (np.abs(nb - order[:cut]) >= 3)
            if bad.any():
                cut = min(cut, int(np.maximum(nb[bad], order[:cut][bad]).min()))
    return path[:cut]


def spiral_tile(h: int, w: int, seed_at: str = "outer"):
    """Spiral corridor mask (255 on the corridor, 0 elsewhere) and a marker that is
    0 except one 255 pixel at the corridor's ``outer`` or ``inner`` end.

    Returns (marker, mask, path_length)."""
    path = spiral_path(h, w)
    mask = np.zeros((h, w), dtype=np.uint8)
    mask[path[:, 0], path[:, 1]] = 255
    marker = np.zeros((h, w), dtype=np.uint8)
    end = path[0] if seed_at == "outer" else path[-1]
    marker[end[0], end[1]] = 255
    return marker, mask, len(path)


def config3_batch(n_tiles: int = 64, size: int = 4096, seed_base: int = seed_for(3, 0)):
    """Batch of ``n_tiles`` size x size tiles from the scaled 512-px generator with
    marker max(I - 30, 0), 8-connectivity; tiles i = 7 (mod 8) are spiral
    corridors, seeded at the outer end when i = 7 (mod 16) and at the inner end
    when i = 15 (mod 16).  Returns a list of task dicts."""
    tasks = []
    for i in range(n_tiles):
        if i % 8 == 7:
            marker, mask, _ = spiral_tile(size, size, "outer" if i % 16 == 7 else "inner")
            kind = "spiral"
        else:
            mask = scaled_config1_tile(size, size, seed_base + i)
            marker = hdome_marker(mask, 30)
            kind = "nuclei"
        tasks.append({"op": "dilate", "marker": marker, "mask": mask, "conn": 8, "kind": kind})
    return tasks


def config4_shapes(n_tiles: int = 256, seed: int = seed_for(4, 999_999)):
    """Shapes, connectivities and h values of the uneven batch: H and W drawn
    independently from {512, 768, ..., 4096}, conn 4 or 8 with p = 1/2,
    h ~ integers[10, 40]."""
    rng = np.random.default_rng(seed)
    hs = rng.choice(SIZES_CFG4, size=n_tiles)
    ws = rng.choice(SIZES_CFG4, size=n_tiles)
    conns = np.where(rng.random(n_tiles) < 0.5, 4, 8)
    hvals = rng.integers(10, 41, size=n_tiles)
    return [(int(a), int(b), int(c), int(d)) for a, b, c, d in zip(hs, ws, conns, hvals)]


def config4_batch(n_tiles: int = 256, config: int = 4, scale: float = 1.0):
    """Uneven batch: per tile the scaled 512-px generator at its own size, marker
    max(I - h, 0).  ``scale`` < 1 shrinks every side (for quick tests)."""
    tasks = []
    for i, (h, w, conn, hv) in enumerate(config4_shapes(n_tiles, seed_for(config, 999_999))):
        h = max(1, int(h * scale))
        w = max(1, int(w * scale))
        mask = scaled_config1_tile(h, w, seed_for(config, i))
        tasks.append({"op": "dilate", "marker": hdome_marker(mask, hv), "mask": mask,
                      "conn": conn, "kind": "uneven", "h": hv})
    return tasks


def random_pair(rng: np.random.Generator, h: int, w: int, levels: int = 256):
    """Random (marker, mask) with values in [0, levels) (few levels force plateaus)."""
    mask = rng.integers(0, levels, size=(h, w)).astype(np.uint8)
    marker = rng.integers(0, levels, size=(h, w)).astype(np.uint8)
    return marker, mask
