"""Seeded synthetic inputs shaped like the filter's workloads.

This module only draws numbers: it holds none of the filter's arithmetic, so both
the HIP path and the CPU oracle can be fed from it.  Images are row-major
``[H, W]`` (k1 = column, contiguous); scale fields are float32 ``[H, W, 4]``
holding the per-pixel scale vector (a1, a2, a3, a4) in the paper's units (the
support length of each generating segment, Section 4).

Recipes
-------
* ``unit_grid_image``: i.i.d. U{0 .. 2^24-1} / 2^24 -- "uniform[0, 1]" pixels that
  are exact in float32 and float64.
* ``blurred_u8_image``: U[0,1) noise, Gaussian blur (sigma, reflect, truncate 4),
  min-max rescale to [0, 255], round half to even, uint8.
* ``integer_scales``: every entry i.i.d. uniform on the integers lo..hi.
* ``uniform_scales``: every entry i.i.d. real U[lo, hi].
* ``smooth_scales``: four independent fields, U[0,1) noise blurred with
  (sigma, wrap, truncate 4), min-max to t in [0, 1], a = lo + (hi - lo) t.
* ``smooth_scales_1d``: per signal, U[0,1) knots every ``period`` samples joined by
  smoothstep interpolation, min-max per signal to t in [0, 1], a = lo + (hi - lo) t:
  float32 [count, length] scales of the one-dimensional filter.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "unit_grid_image", "blurred_u8_image", "integer_scales", "uniform_scales",
    "smooth_scales", "smooth_scales_1d", "Job", "config_job", "batch_jobs", "serving_requests", "CONFIGS",
    "rect_workload",
]


def unit_grid_image(rng: np.random.Generator, h: int, w: int, dtype=np.float64) -> np.ndarray:
    return (rng.integers(0, 1 << 24, size=(h, w), dtype=np.int64).astype(np.float64)
            / float(1 << 24)).astype(dtype)


def _gaussian(noise: np.ndarray, sigma: float, mode: str) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(noise, sigma=sigma, mode=mode, truncate=4.0)


def blurred_u8_image(rng: np.random.Generator, h: int, w: int, sigma: float = 3.0) -> np.ndarray:
    b = _gaussian(rng.random((h, w)), sigma, "reflect")
    b = (b - b.min()) / (b.max() - b.min()) * 255.0
    return np.rint(b).astype(np.uint8)


def integer_scales(rng: np.random.Generator, h: int, w: int, lo: int = 1, hi: int = 8) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=(h, w, 4)).astype(np.float32)


def uniform_scales(rng: np.random.Generator, h: int, w: int, lo: float, hi: float) -> np.ndarray:
    return rng.uniform(lo, hi, size=(h, w, 4)).astype(np.float32)


def smooth_scales(rng: np.random.Generator, h: int, w: int, lo: float = 1.0, hi: float = 16.0,
                  sigma: float = 32.0) -> np.ndarray:
    out = np.empty((h, w, 4), np.float32)
    for d in range(4):
        b = _gaussian(rng.random((h, w)), sigma, "wrap")
        t = (b - b.min()) / (b.max() - b.min())
        out[..., d] = (lo + (hi - lo) * t).astype(np.float32)
    return out


@dataclass
class Job:
    """One filter request: image [H, W], scales [H, W, 4] float32, order n, path."""
    image: np.ndarray
    scales: np.ndarray
    order: int
    path: str = "f64"
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def pixels(self) -> int:
        return int(self.image.shape[0] * self.image.shape[1])


def smooth_scales_1d(rng: np.random.Generator, count: int, length: int, lo: float = 1.0, hi: float = 16.0,
                     period: int = 256) -> np.ndarray:
    nk = length // period + 2
    knots = rng.random((count, nk))
    pos = np.arange(length, dtype=np.float64) / period
    i = np.floor(pos).astype(np.int64)
    u = pos - i
    u = u * u * (3.0 - 2.0 * u)  # smoothstep between neighbouring knots
    b = knots[:, i] * (1.0 - u) + knots[:, i + 1] * u
    bmin, bmax = b.min(axis=1, keepdims=True), b.max(axis=1, keepdims=True)
    t = (b - bmin) / np.maximum(bmax - bmin, 1e-300)
    return np.ascontiguousarray((lo + (hi - lo) * t).astype(np.float32))


# The five workload shapes.  "small" is the parity case the oracle finishes in
# seconds; "plain" is the throughput workload; the others are the precision,
# batched and serving forms.
CONFIGS = {
    "small": dict(desc="256x256 f64 unit-grid pixels, integer scales U{1..8}, order 1", seed=1),
    "plain": dict(desc="2048x2048 uint8 blurred(sigma=3) noise, smooth real scales [1,16] "
                       "(sigma=32 fields), order 2", seed=2),
    "precision": dict(desc="4096x4096 f32 unit-grid pixels, i.i.d. real scales U[1,32], order 2", seed=3),
    "batched": dict(desc="64 images, sides U{256..2048 step 64}, f32 unit-grid pixels, integer "
                         "scales U{1..8}, orders U{1,2,3}", seed=4),
    "serving": dict(desc="Poisson stream, square sides log-uniform [128,4096], f32/f64 50/50, "
                         "integer scales U{1..8}, orders U{1,2,3}", seed=5),
    "ellipse": dict(desc="2048x2048 ellipse field: smooth s_major in [1,8], elongation in [1,4], "
                         "orientation in [0,pi) (sigma=32 fields), order 2", seed=6),
    "signal1d": dict(desc="1024 signals x 65536 samples, f32 unit-grid samples, smooth real scales "
                          "[1,16] (knots every 256 samples), order 3, impulse model, clamp", seed=7),
    "rect": dict(desc="2048x2048 uint8 blurred(sigma=3) noise, two smooth real scale fields [1,16] "
                      "(sigma=32), two-direction (rect) box spline, order 2, impulse model", seed=8),
}


def ellipse_field(rng: np.random.Generator, h: int, w: int, s_lo: float = 1.0, s_hi: float = 8.0,
                  elong_hi: float = 4.0, sigma: float = 32.0) -> np.ndarray:
    """[h, w, 3] float32 (s_major, s_minor, phi) of an adaptive elliptical filter: three
    independent smooth fields (U[0,1) noise, Gaussian sigma, wrap, min-max) mapped to
    s_major in [s_lo, s_hi], elongation s_major/s_minor in [1, elong_hi] and orientation in
    [0, pi)."""
    t = []
    for _ in range(3):
        b = _gaussian(rng.random((h, w)), sigma, "wrap")
        t.append((b - b.min()) / max(b.max() - b.min(), 1e-300))
    out = np.empty((h, w, 3), np.float32)
    out[..., 0] = s_lo + (s_hi - s_lo) * t[0]
    out[..., 1] = out[..., 0] / (1.0 + (elong_hi - 1.0) * t[1])
    out[..., 2] = np.pi * t[2]
    return out


def rect_workload(size: tuple[int, int] = (2048, 2048), seed: int | None = None):
    """(image [H, W] uint8, scales [H, W, 2] float32) of the two-direction workload: the plain
    workload's image recipe, and two of its smooth scale fields (a1 along x, a2 along y)."""
    rng = np.random.default_rng(CONFIGS["rect"]["seed"] if seed is None else seed)
    h, w = size
    img = blurred_u8_image(rng, h, w, 3.0)
    sc = np.ascontiguousarray(smooth_scales(rng, h, w, 1.0, 16.0, 32.0)[..., :2])
    return img, sc


def config_job(name: str, size: tuple[int, int] | None = None, seed: int | None = None) -> Job:
    """Full-size (or resized, same recipe) job for one of the single-image configs."""
    cfg = CONFIGS[name]
    rng = np.random.default_rng(cfg["seed"] if seed is None else seed)
    if name == "small":
        h, w = size or (256, 256)
        img = unit_grid_image(rng, h, w, np.float64)
        sc = integer_scales(rng, h, w, 1, 8)
        return Job(img, sc, 1, "f64", name)
    if name == "plain":
        h, w = size or (2048, 2048)
        img = blurred_u8_image(rng, h, w, 3.0)
        sc = smooth_scales(rng, h, w, 1.0, 16.0, 32.0)
        return Job(img, sc, 2, "f64", name)
    if name == "precision":
        h, w = size or (4096, 4096)
        img = unit_grid_image(rng, h, w, np.float32)
        sc = uniform_scales(rng, h, w, 1.0, 32.0)
        return Job(img, sc, 2, "f32tiled", name)
    raise KeyError(name)


def batch_jobs(count: int = 64, seed: int | None = None, side_lo: int = 256, side_hi: int = 2048,
               step: int = 64, scale_hi: int = 8) -> list[Job]:
    rng = np.random.default_rng(CONFIGS["batched"]["seed"] if seed is None else seed)
    sides = np.arange(side_lo, side_hi + 1, step)
    jobs = []
    for i in range(count):
        w = int(rng.choice(sides))
        h = int(rng.choice(sides))
        n = int(rng.integers(1, 4))
        img = unit_grid_image(rng, h, w, np.float32)
        sc = integer_scales(rng, h, w, 1, scale_hi)
        jobs.append(Job(img, sc, n, "f32tiled", f"batch{i}"))
    return jobs


def serving_requests(duration_s: float, rate_hz: float, seed: int | None = None,
                     side_lo: int = 128, side_hi: int = 4096) -> list[tuple[float, Job]]:
    """(arrival time, job) pairs of a Poisson stream."""
    rng = np.random.default_rng(CONFIGS["serving"]["seed"] if seed is None else seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        s = int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
        f64 = bool(rng.integers(0, 2))
        n = int(rng.integers(1, 4))
        img = unit_grid_image(rng, s, s, np.float64 if f64 else np.float32)
        sc = integer_scales(rng, s, s, 1, 8)
        out.append((t, Job(img, sc, n, "f64" if f64 else "f32tiled", f"req{len(out)}")))
    return out
