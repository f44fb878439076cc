"""Conditioning of the two-stage method at a pixel (Section 7), for reporting beside errors.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP path.

The two-stage method reaches s[m] as a signed sum of large terms (eq. final_eqn, generalised
to order n as the n-fold self-convolution):
    s[m] = 2^n sum_{k in {0..n}^4} c_k sum_j g[j] B_b(p_k - j),
    c_k = (a1 a2 a3 a4)^-n (-1)^|k| prod_d C(n, k_d)            (eq. FD, per direction),
    p_k = m + n tau - sum_d k_d a_d r_d,                       (Table 1 for n = 1)
    tau = ((a1 + a2' - a4' - 1)/2, (a2' + a3 + a4' - 3)/2),  a_j' = a_j / sqrt2,
with g the unit-weight n-fold running sums of eq. RS (the sqrt2 weights of the two diagonal
steps give the factor 2^n) and B_b the order-n box spline at the integration scale
b = (1, sqrt2, 1, sqrt2).  Its rounding error is about kappa(m) eps with
    kappa(m) = 2^n sum_k |c_k| sum_j |g[j] B_b(p_k - j)| / |s[m]|.
This module evaluates both sums for a pixel on its own restart window: the box
[m1 - R1 - 2n - 1, m1 + R1 + n + 1] x [m2 - R2 - 3n - 1, m2 + R2 + 1], R1 = (n/2)(a1 + a2' + a4'),
R2 = (n/2)(a3 + a2' + a4'), which holds the pixel's support and every point its taps read; g
comes from the oracle's exact recursion (``oracle.preintegrate``), B_b from the oracle's
box-spline evaluator.  The signed sum must reproduce the oracle's direct s[m] to within the
rounding of its terms, which checks the geometry above.  kappa for tile windows (what a
GPU tile faces) is larger; the per-pixel window gives the method's own floor.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import box_spline, preintegrate

SQRT2 = math.sqrt(2.0)
B_SCALE = (1.0, SQRT2, 1.0, SQRT2)


def _window(img, x0, x1, y0, y1, border):
    H, W = img.shape
    ys = np.arange(y0, y1 + 1)
    xs = np.arange(x0, x1 + 1)
    win = np.asarray(img, np.float64)[np.ix_(np.clip(ys, 0, H - 1), np.clip(xs, 0, W - 1))].copy()
    if border == "zero":
        win[(ys < 0) | (ys >= H), :] = 0.0
        win[:, (xs < 0) | (xs >= W)] = 0.0
    return win


def two_stage_terms(img, scales, n: int, m1: int, m2: int, border: str = "clamp"):
    """(signed sum, sum of magnitudes) of the two-stage evaluation of s[m] at pixel (m1, m2),
    from exact integer running sums (samples must be integers or on the 2^-24 grid)."""
    a1, a2, a3, a4 = (float(v) for v in np.asarray(scales, np.float32)[m2, m1])
    a2p, a4p = a2 / SQRT2, a4 / SQRT2
    R1 = 0.5 * n * (a1 + a2p + a4p)
    R2 = 0.5 * n * (a3 + a2p + a4p)
    x0, x1 = m1 - math.ceil(R1) - 2 * n - 1, m1 + math.ceil(R1) + n + 1
    y0, y1 = m2 - math.ceil(R2) - 3 * n - 1, m2 + math.ceil(R2) + 1
    win = _window(img, x0, x1, y0, y1, border)
    scale = 1.0 if np.all(win == np.round(win)) else 2.0 ** 24
    wi = win * scale
    if not np.all(wi == np.round(wi)):
        raise ValueError("samples must be integers or lie on the 2^-24 grid")
    g = preintegrate(wi.astype(np.int64), n)  # rows: k2 = y0 + r, columns: k1 = x0 + c
    tx = 0.5 * n * (a1 + a2p - a4p - 1.0)
    ty = 0.5 * n * (a2p + a3 + a4p - 3.0)
    inv = (a1 * a2 * a3 * a4) ** (-n)
    reach = 1.5 * n
    terms = []
    for k in itertools.product(range(n + 1), repeat=4):
        ck = inv * (-1) ** sum(k) * math.prod(math.comb(n, kd) for kd in k)
        px = m1 + tx - (k[0] * a1 + k[1] * a2p - k[3] * a4p)
        py = m2 + ty - (k[1] * a2p + k[2] * a3 + k[3] * a4p)
        for j2 in range(math.ceil(py - reach), math.floor(py + reach) + 1):
            for j1 in range(math.ceil(px - reach), math.floor(px + reach) + 1):
                d1, d2 = px - j1, py - j2
                if abs(d1 + d2) >= 2 * n or abs(d1 - d2) >= 2 * n:
                    continue  # outside the octagonal support
                w = box_spline(d1, d2, B_SCALE, n)
                if w == 0.0:
                    continue
                gv = int(g[j2 - y0, j1 - x0])
                terms.append(ck * w * gv)
    f = 2.0 ** n / scale
    return math.fsum(terms) * f, math.fsum(abs(t) for t in terms) * f


def kappa(img, scales, n: int, pixels, s_direct, border: str = "clamp"):
    """kappa(m) for the flat pixel indices ``pixels`` (row-major), given the direct values
    s_direct (the oracle's filter) at those pixels; also returns the largest mismatch between
    the two-stage sum and s_direct relative to the sum of magnitudes (a check of the terms)."""
    H, W = np.asarray(img).shape
    ks, worst = [], 0.0
    for p, s in zip(pixels, s_direct):
        m2, m1 = divmod(int(p), W)
        signed, mag = two_stage_terms(img, scales, n, m1, m2, border)
        worst = max(worst, abs(signed - s) / mag)
        ks.append(mag / abs(s) if s != 0 else math.inf)
    return np.array(ks), worst
