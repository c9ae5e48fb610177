"""Seeded image generator and workload definitions.

Images: a constant background, star-shaped polygons painted in order with
even-odd fill, an optional smooth gradient, additive N(0, 10^2) noise, then
clipping to [0, 255] and rounding (half to even) to integer gray levels,
stored as float32.  Every draw comes from ``numpy.random.Generator(PCG64)``
with an explicit seed, so the same call returns the same bytes on any host.

Polygon size is tied to an object scale S = min(H, W, 512) (the paper's test
image is 512 x 512), and the polygon count is 10 H W / (pi (0.2 S)^2); star
polygons cover roughly a third of their bounding disc, so the painted area is
about three times the image area at every size, which keeps the density of
edges per pixel similar from 256^2 up to 8192^2.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _fill_polygon(img: np.ndarray, xs: np.ndarray, ys: np.ndarray, value: float) -> None:
    """Paint one closed polygon (vertices xs, ys in pixel units) with even-odd
    fill, sampling at pixel centres (c + 0.5, r + 0.5)."""
    H, W = img.shape
    r0 = max(0, int(math.floor(ys.min() - 0.5)))
    r1 = min(H, int(math.ceil(ys.max() + 0.5)) + 1)
    c0 = max(0, int(math.floor(xs.min() - 0.5)))
    c1 = min(W, int(math.ceil(xs.max() + 0.5)) + 1)
    if r1 <= r0 or c1 <= c0:
        return
    yc = (np.arange(r0, r1, dtype=np.float64) + 0.5)[:, None]
    xa, ya = xs[None, :], ys[None, :]
    xb, yb = np.roll(xs, -1)[None, :], np.roll(ys, -1)[None, :]
    cross = ((ya <= yc) & (yc < yb)) | ((yb <= yc) & (yc < ya))
    dy = np.where(cross, yb - ya, 1.0)
    xc = xa + (yc - ya) * (xb - xa) / dy
    # first pixel column whose centre lies right of the crossing
    col = np.ceil(xc - 0.5) - c0
    rr, ee = np.nonzero(cross)
    bw = c1 - c0
    cc = np.clip(col[rr, ee], 0, bw).astype(np.int64)
    toggles = np.zeros((r1 - r0, bw + 1), dtype=np.uint8)
    np.add.at(toggles, (rr, cc), 1)
    inside = np.bitwise_xor.accumulate(toggles & 1, axis=1)[:, :bw].astype(bool)
    sub = img[r0:r1, c0:c1]
    sub[inside] = value


def polygon_image(height: int, width: int, seed: int, gradient: bool = False,
                  noise_sd: float = 10.0) -> np.ndarray:
    """One H x W float32 image of integer gray levels in [0, 255]."""
    H, W = int(height), int(width)
    rng = _rng(seed)
    img = np.full((H, W), rng.uniform(0.0, 255.0), dtype=np.float64)
    S = float(min(H, W, 512))
    mean_area = math.pi * (0.2 * S) ** 2
    n_poly = max(8, int(round(10.0 * H * W / mean_area)))
    for _ in range(n_poly):
        cx = rng.uniform(0.0, W)
        cy = rng.uniform(0.0, H)
        radius = rng.uniform(0.05, 0.35) * S
        nv = int(rng.integers(3, 9))
        ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, nv))
        rad = radius * rng.uniform(0.4, 1.0, nv)
        value = rng.uniform(0.0, 255.0)
        _fill_polygon(img, cx + rad * np.cos(ang), cy + rad * np.sin(ang), value)
    if gradient:
        a, b = rng.uniform(-60.0, 60.0, 2)
        c = rng.uniform(0.0, 30.0)
        u, v = rng.uniform(0.5, 2.0, 2)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        x = (np.arange(W, dtype=np.float64) / W)[None, :]
        y = (np.arange(H, dtype=np.float64) / H)[:, None]
        img += a * (x - 0.5) + b * (y - 0.5) + c * np.sin(2.0 * math.pi * (u * x + v * y) + ph)
    img += rng.normal(0.0, noise_sd, size=(H, W))
    np.clip(img, 0.0, 255.0, out=img)
    np.rint(img, out=img)
    return img.astype(np.float32)


def frames(n: int, height: int, width: int, seed0: int, gradient: bool = True) -> List[np.ndarray]:
    """n frames, frame j drawn with seed seed0 + j."""
    return [polygon_image(height, width, seed0 + j, gradient=gradient) for j in range(n)]


def batch_specs(n: int = 64, seed: int = 404, min_side: int = 256, max_side: int = 4096) -> List[Dict]:
    """Per-image sizes and filter parameters of the mixed batch.

    Each side is round(exp(U[ln min_side, ln max_side])) drawn independently
    (so most images are not square); sigma_s ~ U[2, 16] with W = ceil(3 sigma_s);
    sigma_r ~ U[10, 80]; range kernel Gaussian or exponential by a fair coin.
    Image i is drawn with seed 100 * seed + i.
    """
    rng = _rng(seed)
    out = []
    lo, hi = math.log(min_side), math.log(max_side)
    for i in range(n):
        h = int(round(math.exp(rng.uniform(lo, hi))))
        w = int(round(math.exp(rng.uniform(lo, hi))))
        sigma_s = float(rng.uniform(2.0, 16.0))
        sigma_r = float(rng.uniform(10.0, 80.0))
        rk = "gaussian" if rng.uniform() < 0.5 else "exponential"
        out.append(dict(height=h, width=w, sigma_s=sigma_s, W=int(math.ceil(3.0 * sigma_s)),
                        sigma_r=sigma_r, range_kind=rk, seed=100 * seed + i))
    return out


# Workload definitions: sizes, kernels and fit settings (data only).
WORKLOADS: Dict[str, Dict] = {
    "gauss_256": dict(n=1, height=256, width=256, seed=101, gradient=False,
                      spatial="gaussian", sigma_s=3.0, W=9,
                      range_kind="gaussian", sigma_r=30.0, T=255, eps=1e-2, K_max=255),
    "exp_2048": dict(n=1, height=2048, width=2048, seed=202, gradient=False,
                     spatial="gaussian", sigma_s=5.0, W=15,
                     range_kind="exponential", sigma_r=20.0, T=255, eps=1e-2, K_max=24),
    "exp_2048_box": dict(n=1, height=2048, width=2048, seed=202, gradient=False,
                         spatial="box", sigma_s=0.0, W=15,
                         range_kind="exponential", sigma_r=20.0, T=255, eps=1e-2, K_max=24),
    "gauss_8192": dict(n=1, height=8192, width=8192, seed=303, gradient=False,
                       spatial="gaussian", sigma_s=10.0, W=30,
                       range_kind="gaussian", sigma_r=10.0, T=255, eps=0.0, K_max=40),
    # the exponential kernel at the number of harmonics where eq. (9) comes
    # within half a gray level of eq. (1) on this image (its kink at t = 0
    # makes the cosine series converge slowly)
    "exp_2048_k128": dict(n=1, height=2048, width=2048, seed=202, gradient=False,
                          spatial="gaussian", sigma_s=5.0, W=15,
                          range_kind="exponential", sigma_r=20.0, T=255, eps=0.0, K_max=128),
    "exp_2048_box_k160": dict(n=1, height=2048, width=2048, seed=202, gradient=False,
                              spatial="box", sigma_s=0.0, W=15,
                              range_kind="exponential", sigma_r=20.0, T=255, eps=0.0, K_max=160),
    # range kernels given only by samples phi(0..T) (see range_table)
    "tukey_2048": dict(n=1, height=2048, width=2048, seed=202, gradient=False,
                       spatial="gaussian", sigma_s=5.0, W=15,
                       range_kind="table", table="tukey", sigma_r=0.0, T=255, eps=1e-3, K_max=128),
    "cauchy_2048": dict(n=1, height=2048, width=2048, seed=202, gradient=False,
                        spatial="gaussian", sigma_s=5.0, W=15,
                        range_kind="table", table="cauchy", sigma_r=0.0, T=255, eps=1e-3, K_max=128),
    "batch64_mixed": dict(n=64, seed=404, T=255, eps=1e-2, K_max=40, spatial="gaussian"),
    "frames32_2160x3840": dict(n=32, height=2160, width=3840, seed=50500, gradient=True,
                               spatial="gaussian", sigma_s=8.0, W=24,
                               range_kind="gaussian", sigma_r=15.0, T=255, eps=0.0, K_max=32),
}


def workload_images(name: str, limit: int | None = None) -> List[np.ndarray]:
    """The input images of a named workload (optionally only the first `limit`)."""
    wl = WORKLOADS[name]
    if name == "batch64_mixed":
        specs = batch_specs(wl["n"], wl["seed"])
        if limit is not None:
            specs = specs[:limit]
        return [polygon_image(s["height"], s["width"], s["seed"]) for s in specs]
    n = wl["n"] if limit is None else min(wl["n"], limit)
    if wl["n"] == 1:
        return [polygon_image(wl["height"], wl["width"], wl["seed"], wl["gradient"])]
    return frames(n, wl["height"], wl["width"], wl["seed"], wl["gradient"])


def range_table(name: str, T: int = 255) -> np.ndarray:
    """Samples phi(0..T) of the sampled range kernels used as inputs: Tukey's
    biweight with support 40, the Cauchy (Lorentzian) kernel of scale 12, and
    a hard window of half-width 20."""
    t = np.arange(T + 1, dtype=np.float64)
    if name == "tukey":
        return np.where(t < 40.0, (1.0 - (t / 40.0) ** 2) ** 2, 0.0)
    if name == "cauchy":
        return 1.0 / (1.0 + (t / 12.0) ** 2)
    if name == "window":
        return (t <= 20).astype(np.float64)
    raise KeyError(name)
