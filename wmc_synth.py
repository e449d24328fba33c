"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws images only; it holds none of the method's arithmetic and
imports neither the oracle nor the HIP binding.

The paper's workloads (natural photographs, BSDS500 patches, a circle grid
whose parameters are not given) are not available, so these stand in for
them: piecewise-smooth images -- a linear ramp with eight hard-edged disks or
convex polygons painted over it -- plus clipped i.i.d. Gaussian noise.  They
contain what the discrete operator distinguishes: straight edges, corners,
curved edges, smooth ramps and noise.

Recipe (numpy PCG64 ``default_rng(seed)``, draws in this order, FP64, cast to
FP32 last; x = column, y = row, values in [0, 1]):

1. ramp  r = a0 + ax * x/(W-1) + ay * y/(H-1),  a0 ~ U[0.30, 0.50],
   ax, ay ~ U[-0.15, 0.15];
2. eight shapes painted in order (later ones on top), each: disk with
   probability 1/2 else convex polygon; centre ~ U[0,W) x U[0,H);
   s = min(H, W); disk radius ~ U[0.04, 0.20] s; polygon: k ~ U{3..6}
   vertices at sorted angles ~ U[0, 2 pi) with radii ~ U[0.05, 0.25] s,
   then their convex hull; per-channel intensity ~ U[0, 1]; inside tests
   at integer pixel coordinates (no anti-aliasing);
3. noisy = clip(clean + sigma N(0, 1), 0, 1), one field per channel.
"""
from __future__ import annotations

import numpy as np


def _hull(pts):
    """Convex hull of a few 2-D points (monotone chain), counter-clockwise."""
    pts = sorted(map(tuple, pts))
    if len(pts) <= 2:
        return pts

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return lower[:-1] + upper[:-1]


def piecewise_smooth(h: int, w: int, channels: int, rng: np.random.Generator) -> np.ndarray:
    """Clean image, shape (channels, h, w), float64 in [0, 1]."""
    a0 = rng.uniform(0.30, 0.50)
    ax = rng.uniform(-0.15, 0.15)
    ay = rng.uniform(-0.15, 0.15)
    ys = np.arange(h, dtype=np.float64)[:, None]
    xs = np.arange(w, dtype=np.float64)[None, :]
    ramp = a0 + ax * xs / max(w - 1, 1) + ay * ys / max(h - 1, 1)
    img = np.broadcast_to(ramp, (channels, h, w)).copy()
    s = float(min(h, w))
    for _ in range(8):
        is_disk = rng.uniform() < 0.5
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        if is_disk:
            rad = rng.uniform(0.04, 0.20) * s
            y0, y1 = max(0, int(np.floor(cy - rad))), min(h, int(np.ceil(cy + rad)) + 1)
            x0, x1 = max(0, int(np.floor(cx - rad))), min(w, int(np.ceil(cx + rad)) + 1)
            yy = np.arange(y0, y1, dtype=np.float64)[:, None]
            xx = np.arange(x0, x1, dtype=np.float64)[None, :]
            mask = (xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad
        else:
            k = int(rng.integers(3, 7))
            ang = np.sort(rng.uniform(0, 2 * np.pi, size=k))
            rr = rng.uniform(0.05, 0.25, size=k) * s
            verts = np.stack([cx + rr * np.cos(ang), cy + rr * np.sin(ang)], axis=1)
            hull = _hull(verts)
            hx = [p[0] for p in hull]
            hy = [p[1] for p in hull]
            y0, y1 = max(0, int(np.floor(min(hy)))), min(h, int(np.ceil(max(hy))) + 1)
            x0, x1 = max(0, int(np.floor(min(hx)))), min(w, int(np.ceil(max(hx))) + 1)
            yy = np.arange(y0, y1, dtype=np.float64)[:, None]
            xx = np.arange(x0, x1, dtype=np.float64)[None, :]
            mask = np.ones((max(y1 - y0, 0), max(x1 - x0, 0)), dtype=bool)
            n = len(hull)
            if n < 3:
                mask[:] = False
            for i in range(n):
                (px, py), (qx, qy) = hull[i], hull[(i + 1) % n]
                mask &= (qx - px) * (yy - py) - (qy - py) * (xx - px) >= 0
        inten = rng.uniform(0.0, 1.0, size=channels)
        if y1 > y0 and x1 > x0:
            for c in range(channels):
                img[c, y0:y1, x0:x1][mask] = inten[c]
    return img


def add_noise(clean: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    return np.clip(clean + sigma * rng.standard_normal(clean.shape), 0.0, 1.0)


def image(h: int, w: int, channels: int, sigma: float, seed: int):
    """(noisy, clean) float32 arrays of shape (channels, h, w)."""
    rng = np.random.default_rng(seed)
    clean = piecewise_smooth(h, w, channels, rng)
    noisy = add_noise(clean, sigma, rng)
    return noisy.astype(np.float32), clean.astype(np.float32)


# ---- the five workloads -------------------------------------------------------------
# C1: 1x1x256x256, sigma 0.05, lam 1, 50 iterations (parity against the oracle).
# C2: 1x1x4096x4096, sigma 0.1, lam 1, 200 iterations (solver throughput).
# C3: 64 images x 3 channels, sides U{128..2048}, sigma U[0.02, 0.15], 100 iterations.
# C4: 16x1x512x512, sigma 0.1, K = 20 (differentiable layer).
# C5: 32x1x256x256, sigma U[0.02, 0.20], K = 30 (learned lam).

def c1():
    noisy, clean = image(256, 256, 1, 0.05, seed=0)
    return noisy, clean


def c2(side: int = 4096, seed: int = 1):
    noisy, clean = image(side, side, 1, 0.1, seed=seed)
    return noisy, clean


def c3_sizes(n_images: int = 64, seed: int = 2):
    """Per-image (h, w, sigma) for the uneven batch."""
    rng = np.random.default_rng(seed)
    hs = rng.integers(128, 2049, size=n_images)
    ws = rng.integers(128, 2049, size=n_images)
    sig = rng.uniform(0.02, 0.15, size=n_images)
    return [(int(h), int(w), float(s)) for h, w, s in zip(hs, ws, sig)]


def c3_image(b: int, h: int, w: int, sigma: float):
    return image(h, w, 3, sigma, seed=1000 + b)


def c4(batch: int = 16, side: int = 512):
    noisy = np.empty((batch, 1, side, side), np.float32)
    clean = np.empty_like(noisy)
    for b in range(batch):
        noisy[b], clean[b] = image(side, side, 1, 0.1, seed=2000 + b)
    return noisy, clean


def c5_batch(seed: int, batch: int = 32, side: int = 256):
    """(noisy, clean, sigma) for one learned-lam training or eval batch."""
    rng = np.random.default_rng(seed)
    sig = rng.uniform(0.02, 0.20, size=batch)
    noisy = np.empty((batch, 1, side, side), np.float32)
    clean = np.empty_like(noisy)
    for b in range(batch):
        noisy[b], clean[b] = image(side, side, 1, float(sig[b]), seed=seed * 1000 + b)
    return noisy, clean, sig.astype(np.float32)


def random_unit(h: int, w: int, seed: int) -> np.ndarray:
    """i.i.d. U[0, 1) plane, float32 (unstructured parity input)."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(h, w)).astype(np.float32)


def shapes(side: int = 128) -> np.ndarray:
    """Piecewise-constant edge test image for the curvature-flow study, float32
    (side, side): background 0.2, an axis-aligned cross (0.6) in the upper
    left quadrant, a 45-degree diamond |x-cx| + |y-cy| <= r (0.8) in the upper
    right, a disk (0.4) in the lower left and an axis-aligned square (0.9) in
    the lower right.  No randomness."""
    q = side // 4
    ys = np.arange(side, dtype=np.float64)[:, None]
    xs = np.arange(side, dtype=np.float64)[None, :]
    img = np.full((side, side), 0.2)
    r = 0.6 * q
    arm = max(1, q // 4)
    cross = ((np.abs(xs - q) <= arm) & (np.abs(ys - q) <= r)) | \
            ((np.abs(ys - q) <= arm) & (np.abs(xs - q) <= r))
    img[cross] = 0.6
    img[np.abs(xs - 3 * q) + np.abs(ys - q) <= r] = 0.8
    img[(xs - q) ** 2 + (ys - 3 * q) ** 2 <= r * r] = 0.4
    img[(np.abs(xs - 3 * q) <= r) & (np.abs(ys - 3 * q) <= r)] = 0.9
    return img.astype(np.float32)
