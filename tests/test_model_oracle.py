"""Pins of the continuous-model oracle (Section 6 with phi = beta^{n1} (x) beta^{n1}) for the
four-direction box spline, against facts that do not come from it:

* n1 = -1 (phi = delta) is the Section 7 oracle itself;
* phi * B_a at sample points against a direct two-dimensional quadrature of
  phi(y) B_a(x - y) over the support of phi (scipy's B-spline basis elements for phi);
* unit mass, and the covariance Cov(B_a) + (n1+1)/12 I (a convolution adds covariances;
  Cov(B_a) = n sum_d a_d^2/12 r_d r_d^T, Section 4);
* a constant image is reproduced at any scales (the model of a constant is that constant);
  a linear image is reproduced for n1 >= 1; a quadratic one projects to p(m) + tr(H Sigma)/2
  for n1 >= 2 with Sigma = Cov(B_a) alone (the interpolating model is the polynomial itself,
  so phi's own spread must not appear -- which pins the prefilter);
* an image constant along its columns reduces to the one-dimensional filter of Section 3
  (oracle.filter1d) with the box spline's marginal along x.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

import oracle.filter1d as F1

S2 = math.sqrt(2.0)
R = [np.array([1.0, 0.0]), np.array([1.0, 1.0]) / S2, np.array([0.0, 1.0]), np.array([-1.0, 1.0]) / S2]


def test_delta_model_is_the_section7_oracle(oracle_mod):
    rng = np.random.default_rng(7000)
    for n in (1, 2, 3):
        a = rng.uniform(0.6, 3.0, 4)
        for _ in range(6):
            x = rng.uniform(-3, 3, 2)
            assert abs(oracle_mod.box_spline_model(x[0], x[1], a, n, -1) - oracle_mod.box_spline(x[0], x[1], a, n)) \
                < 1e-15
    img = rng.uniform(0, 1, (12, 13))
    sc = rng.uniform(1, 3, (12, 13, 4)).astype(np.float32)
    for border in ("clamp", "zero"):
        np.testing.assert_allclose(oracle_mod.filter_model(img, sc, 2, -1, border), oracle_mod.filter(img, sc, 2, border),
                                   rtol=0, atol=1e-15)


def _bs(N, y):
    B = BSpline.basis_element(np.arange(N + 2) - (N + 1) / 2, extrapolate=False)
    return float(np.nan_to_num(B(y)))


@pytest.mark.parametrize("n1", [0, 1])
def test_phi_convolution_against_direct_quadrature(oracle_mod, n1):
    a = [1.7, 2.3, 1.2, 1.9]
    rng = np.random.default_rng(7010 + n1)
    h = 0.5 * (n1 + 1)
    knots = [-h + i for i in range(n1 + 2)]
    for _ in range(2):
        x = rng.uniform(-1.5, 1.5, 2)

        def inner(y2):
            return integrate.quad(lambda y1: _bs(n1, y1) * _bs(n1, y2) * oracle_mod.box_spline(x[0] - y1, x[1] - y2, a, 1),
                                  -h, h, points=knots[1:-1] or None, limit=200, epsabs=1e-12)[0]

        ref = integrate.quad(inner, -h, h, points=knots[1:-1] or None, limit=200, epsabs=1e-11)[0]
        got = oracle_mod.box_spline_model(x[0], x[1], a, 1, n1)
        assert abs(got - ref) < 2e-7, (x, got, ref)


@pytest.mark.parametrize("n,n1", [(1, 0), (1, 1), (1, 3), (2, 1)])
def test_mass_and_covariance(oracle_mod, n, n1):
    a = [1.3, 2.1, 0.9, 1.6]
    h = 1.0 / 16
    e = 0.5 * (n1 + 1)
    R1 = 0.5 * n * (a[0] + (a[1] + a[3]) / S2) + e
    R2 = 0.5 * n * (a[2] + (a[1] + a[3]) / S2) + e
    xs = np.arange(-R1 - h / 2, R1 + h, h)
    ys = np.arange(-R2 - h / 2, R2 + h, h)
    m0, M = 0.0, np.zeros((2, 2))
    for x in xs:
        for y in ys:
            v = oracle_mod.box_spline_model(x, y, a, n, n1)
            if v:
                m0 += v
                M += v * np.outer([x, y], [x, y])
    m0 *= h * h
    M *= h * h
    C = n * sum(ad * ad / 12.0 * np.outer(rd, rd) for ad, rd in zip(a, R)) + (n1 + 1) / 12.0 * np.eye(2)
    assert abs(m0 - 1.0) < 1e-9
    np.testing.assert_allclose(M, C, atol=2e-3)


@pytest.mark.parametrize("n1", [0, 1, 2, 3])
def test_constant_image_at_real_scales(oracle_mod, n1):
    rng = np.random.default_rng(7020 + n1)
    img = np.full((9, 10), 0.625)
    sc = rng.uniform(0.5, 2.5, (9, 10, 4)).astype(np.float32)
    out = oracle_mod.filter_model(img, sc, 1, n1, "clamp", pixels=np.array([0, 17, 44, 89]))
    np.testing.assert_allclose(out, 0.625, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n1", [1, 2, 3])
def test_polynomials_project_by_moments(oracle_mod, n1):
    rng = np.random.default_rng(7030 + n1)
    H, W = 96, 97  # the clamped border's effect on c dies off like |z|^45 at the centre
    al, be, ga = (0.25, -0.125, 0.1875) if n1 >= 2 else (0.0, 0.0, 0.0)
    k1, k2 = np.meshgrid(np.arange(W, dtype=float), np.arange(H, dtype=float))
    img = 2.0 - 0.75 * k1 + 0.5 * k2 + al * k1 * k1 + be * k1 * k2 + ga * k2 * k2
    sc = rng.uniform(0.5, 2.0, (H, W, 4)).astype(np.float32)
    pix = np.array([47 * W + 48, 48 * W + 47, 46 * W + 49])
    out = oracle_mod.filter_model(img, sc, 1, n1, "clamp", pixels=pix)
    for p, v in zip(pix, out):
        m2, m1 = divmod(int(p), W)
        a = sc[m2, m1].astype(np.float64)
        # the model is the polynomial itself, so only the box spline's moments enter (phi's
        # smoothing is undone by the interpolating coefficients)
        C = sum(ad * ad / 12.0 * np.outer(rd, rd) for ad, rd in zip(a, R))
        want = img[m2, m1] + al * C[0, 0] + be * C[0, 1] + ga * C[1, 1]
        assert abs(v - want) < 1e-11 * np.abs(img).max(), (n1, p, v - want)


@pytest.mark.parametrize("n1", [0, 1, 3])
def test_column_constant_image_is_the_1d_filter(oracle_mod, n1):
    """Sum over rows of (phi * B_a) at integer offsets is its marginal along x exactly for
    n1 >= 0 (the integer translates of beta^{n1} sum to one); with a1 = a2/sqrt2 = a4/sqrt2 = c
    that marginal is beta^{n1} * beta_c^2 (order 1: three boxes of width c), the 1-D model kernel
    of order 3 (up to the float32 rounding of sqrt2 c)."""
    rng = np.random.default_rng(7040 + n1)
    H, W = 8, 40
    row = rng.uniform(0, 1, W)
    img = np.tile(row, (H, 1))
    c = np.float32(1.75)
    sc = np.empty((H, W, 4), np.float32)
    sc[..., 0] = c
    sc[..., 1] = np.float32(S2 * float(c))
    sc[..., 2] = rng.uniform(0.5, 3.0, (H, W))
    sc[..., 3] = np.float32(S2 * float(c))
    pix = np.array([3 * W + 20, 4 * W + 5, 2 * W + 33])
    out = oracle_mod.filter_model(img, sc, 1, n1, "clamp", pixels=pix)
    for p, v in zip(pix, out):
        m1 = int(p) % W
        ref = F1.filter1d(row, np.full(W, c), 3, n1, "clamp", [m1])[0]
        assert abs(v - ref) < 1e-6, (n1, p, v, ref)
