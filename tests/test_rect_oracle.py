"""Pins of the two-direction (rect) oracle against facts that do not come from it.

* rect = beta^2_(1,1) (Section 4): at unit scales and order 1 the filter is the identity;
* order 1 at integer scales is the moving average over the half-open box (Section 2's
  beta^0 on (-a/2, a/2]), by brute force;
* an image constant along its columns reduces to the one-dimensional filter of Section 3
  along its rows (the column kernel sums to one at integer scales);
* constant scales make the filter shift-invariant and separable: the one-dimensional oracle
  along rows, then along columns;
* the impulse response is the tensor product of scipy's B-spline basis elements;
* the projection of a reproduced polynomial (model degree 2, 3) follows from the B-spline's
  moments alone; transpose and mirror symmetries.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle.filter1d as F1
import oracle.rect as R


def test_unit_rect_is_the_identity():
    rng = np.random.default_rng(3000)
    img = rng.standard_normal((9, 11))
    sc = np.ones((9, 11, 2), np.float32)
    for border in ("clamp", "zero"):
        out = R.filter_rect_exact(img, sc, 1, -1, border)
        assert out == [Fraction(float(v)) for v in img.reshape(-1)]


def test_order_one_is_the_box_average():
    rng = np.random.default_rng(3001)
    H, W = 10, 13
    img = rng.standard_normal((H, W))
    sc = rng.integers(1, 6, size=(H, W, 2)).astype(np.float32)
    out = R.filter_rect_exact(img, sc, 1, -1, "zero")
    for p, v in enumerate(out):
        m2, m1 = divmod(p, W)
        a1, a2 = (Fraction(float(x)) for x in sc[m2, m1])
        acc = Fraction(0)
        for k2 in range(H):
            for k1 in range(W):
                if -a1 / 2 < m1 - k1 <= a1 / 2 and -a2 / 2 < m2 - k2 <= a2 / 2:
                    acc += Fraction(float(img[k2, k1]))
        assert v == acc / (a1 * a2), (m1, m2)


@pytest.mark.parametrize("n,n1", [(1, -1), (2, -1), (3, 0), (2, 1), (2, 2), (1, 3)])
def test_column_constant_image_is_the_1d_filter(n, n1):
    rng = np.random.default_rng(3002 + 7 * n + n1)
    H, W = 7, 30
    row = rng.standard_normal(W)
    img = np.tile(row, (H, 1))
    sc = np.empty((H, W, 2), np.float32)
    sc[..., 0] = rng.uniform(0.5, 6.0, size=(H, W))
    sc[..., 1] = rng.integers(1, 5, size=(H, W))  # the column kernel sums to one
    pix = list(range(0, H * W, 5))
    out = R.filter_rect_exact(img, sc, n, n1, "clamp", pix)
    for p, v in zip(pix, out):
        m2, m1 = divmod(p, W)
        sc1 = sc[m2, :, 0]
        ref = F1.filter1d_exact(row, sc1, n, n1, "clamp", [m1])[0]
        assert abs(v - ref) < Fraction(1, 10 ** 30), (p, float(v - ref))


@pytest.mark.parametrize("n,n1", [(1, -1), (2, -1), (3, -1), (2, 0), (3, 1)])
def test_constant_scales_are_two_1d_passes(n, n1):
    rng = np.random.default_rng(3003 + n + n1)
    H, W = 12, 15
    img = rng.standard_normal((H, W))
    a1, a2 = np.float32(2.75), np.float32(1.5)
    sc = np.empty((H, W, 2), np.float32)
    sc[..., 0], sc[..., 1] = a1, a2
    out = np.array(R.filter_rect_exact(img, sc, n, n1, "zero"), dtype=object).reshape(H, W)
    # rows with a1, then columns with a2, both through the 1-D oracle (zero border)
    rows = [F1.filter1d_exact(img[k2], np.full(W, a1), n, n1, "zero") for k2 in range(H)]
    for m1 in range(W):
        colx = [rows[k2][m1] for k2 in range(H)]
        # exact column pass: the 1-D oracle's kernel on the exact row results
        Rr, K = R._kernel(a2, n, n1)
        for m2 in range(H):
            acc = Fraction(0)
            for i, w in enumerate(K):
                k2 = m2 - (i - Rr)
                if 0 <= k2 < H and w:
                    acc += w * colx[k2]
            assert out[m2, m1] == acc, (m1, m2)


@pytest.mark.parametrize("n", [2, 3])
def test_impulse_response_is_the_tensor_bspline(n):
    H, W = 21, 23
    img = np.zeros((H, W))
    img[10, 11] = 1.0
    a1, a2 = 3.25, 2.5
    sc = np.empty((H, W, 2), np.float32)
    sc[..., 0], sc[..., 1] = a1, a2
    out = R.filter_rect(img, sc, n, -1, "zero")

    def bs(x, a):
        N = n - 1
        B = BSpline.basis_element(a * (np.arange(N + 2) - (N + 1) / 2), extrapolate=False)
        return np.nan_to_num(B(np.asarray(x, float))) / a

    ref = np.outer(bs(np.arange(H) - 10, a2), bs(np.arange(W) - 11, a1))
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n,n1", [(1, 2), (2, 2), (3, 3), (2, 3)])
def test_prefiltered_polynomials(n, n1):
    """p(k1, k2) of degree <= n1 in each variable is its own model; its projection is
    p(m) + (p_11 Var1 + p_22 Var2) / 2, Var_i = n a_i^2 / 12, away from the borders."""
    rng = np.random.default_rng(3004 + 5 * n + n1)
    H, W = 125, 126  # the clamped border's effect on c dies off like |z|^60 < 1e-34 at the centre
    cf = {(0, 0): Fraction(2), (1, 0): Fraction(-1), (0, 1): Fraction(3, 2), (2, 0): Fraction(1, 4),
          (1, 1): Fraction(-1, 8), (0, 2): Fraction(3, 16)}

    def p(x, y):
        return sum(c * Fraction(x) ** i * Fraction(y) ** j for (i, j), c in cf.items())

    img = np.array([[float(p(k1, k2)) for k1 in range(W)] for k2 in range(H)])
    sc = rng.uniform(0.5, 3.0, size=(H, W, 2)).astype(np.float32)
    pix = [k2 * W + k1 for k2 in range(61, 64) for k1 in range(62, 65)]
    out = R.filter_rect_exact(img, sc, n, n1, "clamp", pix)
    for q, v in zip(pix, out):
        m2, m1 = divmod(q, W)
        a1, a2 = (Fraction(float(x)) for x in sc[m2, m1])
        want = p(m1, m2) + (2 * cf[(2, 0)] * n * a1 * a1 + 2 * cf[(0, 2)] * n * a2 * a2) / 24
        assert abs(v - want) < Fraction(1, 10 ** 25), (m1, m2, float(v - want))


def test_transpose_and_mirror_symmetry():
    rng = np.random.default_rng(3005)
    H, W = 9, 12
    img = rng.standard_normal((H, W))
    sc = rng.uniform(0.5, 4.0, size=(H, W, 2)).astype(np.float32)
    for n, n1 in [(2, -1), (3, 0), (1, 2)]:
        out = np.array(R.filter_rect_exact(img, sc, n, n1, "clamp"), dtype=object).reshape(H, W)
        t = np.array(R.filter_rect_exact(img.T.copy(), sc.transpose(1, 0, 2)[..., ::-1].copy(), n, n1, "clamp"),
                     dtype=object).reshape(W, H)
        assert (t.T == out).all()
        # mirror along x: kernels are even for n >= 2 or a continuous model
        mir = np.array(R.filter_rect_exact(img[:, ::-1].copy(), sc[:, ::-1].copy(), n, n1, "clamp"),
                       dtype=object).reshape(H, W)
        assert (mir[:, ::-1] == out).all()


def test_float_and_exact_agree():
    rng = np.random.default_rng(3006)
    H, W = 14, 17
    img = rng.uniform(0, 1, (H, W))
    sc = rng.uniform(0.5, 5.0, size=(H, W, 2)).astype(np.float32)
    for n, n1, border in [(2, -1, "clamp"), (3, 1, "zero"), (2, 2, "clamp"), (1, 3, "zero")]:
        ex = np.array([float(v) for v in R.filter_rect_exact(img, sc, n, n1, border)]).reshape(H, W)
        fl = R.filter_rect(img, sc, n, n1, border)
        assert np.abs(ex - fl).max() <= 1e-15 * np.abs(ex).max()
        pix = np.array([0, 5, W * H - 1, 3 * W + 7])
        np.testing.assert_array_equal(R.filter_rect(img, sc, n, n1, border, pix), fl.reshape(-1)[pix])
