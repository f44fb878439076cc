"""Oracle for the two-direction (rect) space-variant box-spline filter.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP path and
never imports it.

What is computed.  Section 4, eq. def with directional order N = 2 (angles 0 and pi/2): the
box spline of scale vector (a1, a2) is the convolution of a segment of length a1 along the
first lattice axis (x, columns) with one of length a2 along the second (y, rows),
    beta^2_(a1,a2)(x) = beta_a1(x1) beta_a2(x2),
rect = beta^2_(1,1) being the most elementary one.  Order n is the n-fold self-convolution
(closing remark of Section 4): beta_a1^{n-1}(x1) beta_a2^{n-1}(x2).  Section 6 projects the
continuous model f(x) = sum_k c[k] phi(x - k) onto it at every pixel m with that pixel's own
scales, here with phi = beta^{n1} (x) beta^{n1} (model degree n1 in {-1, 0, 1, 2, 3}; n1 = -1
is phi = delta, Section 7's choice), and c = f_ext * (b^{n1} (x) b^{n1})^{-1}, the
interpolating coefficients (c = f_ext for n1 <= 1).  The result is separable per pixel:
    s[m] = sum_k c[k] K_{a1(m)}(m1 - k1) K_{a2(m)}(m2 - k2),   K_a = beta^{n1} * beta_a^{n-1},
with K_a the one-dimensional model kernel of Section 3 (``oracle.filter1d``: exact rationals
from the truncated-power form) and f_ext the image extended by clamp or zero.

The inverse of the separable interpolation filter is the one-dimensional inverse along rows,
then along columns: each row of f_ext (rows outside the image follow the border rule) is
solved exactly on a block reaching PREFILTER_MARGIN samples past the needed columns, then each
needed column of the result likewise (``oracle.filter1d.solve_block``; truncation below 1e-30).

``filter_rect_exact`` returns Fractions (small images); ``filter_rect`` rounds c and K to
float64 and sums each pixel's terms with numpy, which for the non-negative kernels and the
bounded coefficients here is accurate to a few ulps of the output's magnitude.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import filter1d as F1

BORDERS = ("clamp", "zero")


def _check(img, scales, n, n1, border):
    img = np.asarray(img)
    scales = np.asarray(scales, dtype=np.float32)
    if img.ndim != 2 or scales.shape != img.shape + (2,):
        raise ValueError("expected img [H, W] and scales [H, W, 2]")
    if n < 1 or n1 not in F1.MODELS or border not in BORDERS:
        raise ValueError("order >= 1, model in -1..3, border clamp/zero")
    return img, scales


def _ext_row(img, k2: int, border: str):
    """Row k2 of f_ext as a 1-D signal (its own extension along k1 is done by filter1d)."""
    H, W = img.shape
    if 0 <= k2 < H:
        return img[k2]
    if border == "clamp":
        return img[min(max(k2, 0), H - 1)]
    return np.zeros(W, dtype=img.dtype)


def coefficients_2d(img, n1: int, border: str, y0: int, y1: int, x0: int, x1: int) -> list[list[Fraction]]:
    """c[k2][k1] for k2 in [y0, y1), k1 in [x0, x1) (rows of Fractions)."""
    if n1 <= 1:
        return [F1.coefficients(_ext_row(img, k2, border), n1, border, x0, x1) for k2 in range(y0, y1)]
    M = F1.PREFILTER_MARGIN
    # along rows: every row the column solves reach
    rows = [F1.coefficients(_ext_row(img, k2, border), n1, border, x0, x1) for k2 in range(y0 - M, y1 + M)]
    out = [[Fraction(0)] * (x1 - x0) for _ in range(y1 - y0)]
    for i in range(x1 - x0):
        col = F1.solve_block([r[i] for r in rows], n1)[M:M + (y1 - y0)]
        for r in range(y1 - y0):
            out[r][i] = col[r]
    return out


def _kernel(a, n, n1):
    R = int(math.floor(F1.support_radius(a, n, n1)))
    nums, den = F1.kernel_numerators(list(range(-R, R + 1)), a, n, n1)
    return R, [Fraction(v) / den for v in nums]


def _reach(scales, n, n1):
    return int(math.floor(F1.support_radius(float(np.max(scales)), n, n1)))


def filter_rect_exact(img, scales, n: int, n1: int = -1, border: str = "clamp", pixels=None) -> list[Fraction]:
    """Exact s[m] (Fractions) for the flat pixel indices ``pixels`` (default: all, row-major)."""
    img, scales = _check(img, scales, n, n1, border)
    H, W = img.shape
    pix = range(H * W) if pixels is None else [int(p) for p in pixels]
    R = _reach(scales, n, n1)
    c = coefficients_2d(img, n1, border, -R, H + R, -R, W + R)
    out = []
    for p in pix:
        m2, m1 = divmod(p, W)
        a1, a2 = scales[m2, m1]
        R1, K1 = _kernel(a1, n, n1)
        R2, K2 = _kernel(a2, n, n1)
        acc = Fraction(0)
        for i2, w2 in enumerate(K2):
            if not w2:
                continue
            row = c[m2 + R2 - i2 + R]  # k2 = m2 - (i2 - R2)
            inner = Fraction(0)
            for i1, w1 in enumerate(K1):
                if w1:
                    inner += w1 * row[m1 + R1 - i1 + R]
            acc += w2 * inner
        out.append(acc)
    return out


def filter_rect(img, scales, n: int, n1: int = -1, border: str = "clamp", pixels=None) -> np.ndarray:
    """s[m] in float64 ([H, W], or the flat indices ``pixels``)."""
    img, scales = _check(img, scales, n, n1, border)
    H, W = img.shape
    R = _reach(scales, n, n1)
    if n1 <= 1:
        ys = np.clip(np.arange(-R, H + R), 0, H - 1)
        xs = np.clip(np.arange(-R, W + R), 0, W - 1)
        c = np.asarray(img, np.float64)[np.ix_(ys, xs)].copy()
        if border == "zero":
            inside_y = (np.arange(-R, H + R) >= 0) & (np.arange(-R, H + R) < H)
            inside_x = (np.arange(-R, W + R) >= 0) & (np.arange(-R, W + R) < W)
            c[~inside_y, :] = 0.0
            c[:, ~inside_x] = 0.0
    else:
        c = np.array([[float(v) for v in row] for row in coefficients_2d(img, n1, border, -R, H + R, -R, W + R)])
    pix = np.arange(H * W) if pixels is None else np.asarray(pixels, dtype=np.int64)
    cache = {}

    def kern(a):
        key = float(a)
        if key not in cache:
            Rk, K = _kernel(a, n, n1)
            cache[key] = (Rk, np.array([float(v) for v in K]))
        return cache[key]

    out = np.empty(len(pix), np.float64)
    for i, p in enumerate(pix):
        m2, m1 = divmod(int(p), W)
        R1, K1 = kern(scales[m2, m1, 0])
        R2, K2 = kern(scales[m2, m1, 1])
        # window rows m2 + R2 .. m2 - R2 (k2 = m2 - (i2 - R2)), columns likewise
        win = c[m2 - R2 + R:m2 + R2 + R + 1, m1 - R1 + R:m1 + R1 + R + 1]
        out[i] = K2[::-1] @ (win @ K1[::-1])
    return out.reshape(H, W) if pixels is None else out
