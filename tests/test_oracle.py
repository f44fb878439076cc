"""Pins for the CPU oracle: closed forms, identities and library routines.

None of these re-types the oracle's own formula.  They check it against facts the
paper and the mathematics fix:
* hand-worked closed-form values of the order-1 element at the integration
  scale (tests/golden/box_spline_values.json, Section 7);
* the partition of unity that holds for integer a1, a3 (Poisson summation: the
  Fourier transform, a product of sinc powers, vanishes on the dual lattice);
* the 1-D marginal, which must be a B-spline of degree 3n-1 (SciPy's basis
  element is the independent routine);
* mass, covariance and symmetries of a convolution of segments (Section 4,
  Thm 4.3 uses the covariance sum_d a_d^2/12 r_d r_d^T);
* for stage 1, brute-force enumeration of the running-sum cone and the lattice
  finite differences that invert it.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import BSpline

S2 = math.sqrt(2.0)
B = [1.0, S2, 1.0, S2]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "box_spline_values.json")


def test_closed_form_values(oracle_mod):
    spec = json.load(open(GOLDEN))
    for case in spec["cases"]:
        c = 1.0 if case["a"] == "b" else 2.0
        a = [c * v for v in B]
        got = oracle_mod.box_spline(case["x"][0], case["x"][1], a, spec["order"])
        want = float(Fraction(case["value"]))
        assert abs(got - want) < 1e-15, (case, got)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_partition_of_unity_integer_axis_scales(oracle_mod, n):
    rng = np.random.default_rng(10 + n)
    for _ in range(4 if n < 3 else 2):
        a = [float(rng.integers(1, 4)), rng.uniform(0.6, 3.0), float(rng.integers(1, 4)), rng.uniform(0.6, 3.0)]
        x = rng.uniform(-0.5, 0.5, size=2)
        R = int(math.ceil(0.5 * n * (max(a[0], a[2]) + (a[1] + a[3]) / S2))) + 1
        tot = sum(oracle_mod.box_spline(x[0] - k1, x[1] - k2, a, n)
                  for k1 in range(-R, R + 1) for k2 in range(-R, R + 1))
        assert abs(tot - 1.0) < 1e-13, (a, x, tot)


def test_partition_of_unity_fails_for_fractional_axis_scale(oracle_mod):
    # the identity really needs integer a1, a3: a fractional a1 must leave a ripple
    a = [1.5, 1.3, 1.0, 1.1]
    tot = sum(oracle_mod.box_spline(0.1 - k1, 0.1 - k2, a, 1) for k1 in range(-4, 5) for k2 in range(-4, 5))
    assert abs(tot - 1.0) > 1e-5


@pytest.mark.parametrize("n", [1, 2, 3])
def test_marginal_is_bspline(oracle_mod, n):
    """sum over k2 at integer a3 is the x1-marginal: the convolution of the three
    projected segment sums, a B-spline of degree 3n-1 when a1 = a2/sqrt2 = a4/sqrt2 = c."""
    for c in (0.8, 1.7):
        a = [c, c * S2, 2.0, c * S2]
        knots = c * (np.arange(3 * n + 1) - 1.5 * n)
        ref = BSpline.basis_element(knots, extrapolate=False)
        R = int(math.ceil(0.5 * n * (2.0 + 2 * c))) + 2
        for x1 in (-1.3 * c, -0.2, 0.0, 0.37, 1.1 * c):
            x2 = 0.3
            tot = sum(oracle_mod.box_spline(x1, x2 - k2, a, n) for k2 in range(-R, R + 1))
            want = float(np.nan_to_num(ref(x1))) / c
            assert abs(tot - want) < 1e-12, (n, c, x1, tot, want)
    # the same along x2 with the roles of a1 and a3 exchanged
    c = 1.3
    a = [3.0, c * S2, c, c * S2]
    knots = c * (np.arange(3 * n + 1) - 1.5 * n)
    ref = BSpline.basis_element(knots, extrapolate=False)
    for x2 in (-0.9, 0.0, 0.6):
        tot = sum(oracle_mod.box_spline(0.2 - k1, x2, a, n) for k1 in range(-12, 13))
        assert abs(tot - float(np.nan_to_num(ref(x2))) / c) < 1e-12


@pytest.mark.parametrize("n", [1, 2])
def test_mass_and_covariance(oracle_mod, n):
    """Midpoint-rule moments on a fine grid: unit mass and covariance
    n * sum_d a_d^2/12 r_d r_d^T (the segment sums are independent)."""
    a = [1.3, 2.1, 0.9, 1.6]
    h = 1.0 / 24
    R1 = 0.5 * n * (a[0] + (a[1] + a[3]) / S2)
    R2 = 0.5 * n * (a[2] + (a[1] + a[3]) / S2)
    xs = np.arange(-R1 - h / 2, R1 + h, h)
    ys = np.arange(-R2 - h / 2, R2 + h, h)
    m0 = 0.0
    M = np.zeros((2, 2))
    for x in xs:
        for y in ys:
            v = oracle_mod.box_spline(x, y, a, n)
            if v:
                m0 += v
                M += v * np.outer([x, y], [x, y])
    m0 *= h * h
    M *= h * h
    r = [np.array([1.0, 0.0]), np.array([1.0, 1.0]) / S2, np.array([0.0, 1.0]), np.array([-1.0, 1.0]) / S2]
    C = n * sum(ad * ad / 12.0 * np.outer(rd, rd) for ad, rd in zip(a, r))
    assert abs(m0 - 1.0) < 2e-3
    assert np.abs(M - C).max() < 5e-3 * np.abs(C).max()
    # the off-diagonal entry separates a2 from a4
    assert abs(M[0, 1] - n * (a[1] ** 2 - a[3] ** 2) / 24.0) < 5e-3


@pytest.mark.parametrize("n", [1, 2, 3])
def test_symmetries_and_scaling(oracle_mod, n):
    rng = np.random.default_rng(3 * n)
    for _ in range(6):
        a = list(rng.uniform(0.7, 2.5, size=4))
        x1, x2 = rng.uniform(-2.0, 2.0, size=2)
        v = oracle_mod.box_spline(x1, x2, a, n)
        assert abs(v - oracle_mod.box_spline(-x1, -x2, a, n)) < 1e-15
        # mirror x1 -> -x1 exchanges the two diagonal directions
        assert abs(v - oracle_mod.box_spline(-x1, x2, [a[0], a[3], a[2], a[1]], n)) < 1e-15
        # transpose exchanges the two axis directions
        assert abs(v - oracle_mod.box_spline(x2, x1, [a[2], a[1], a[0], a[3]], n)) < 1e-15
        # scaling of a convolution of segments: B_{ca}(x) = B_a(x/c)/c^2
        c = 1.75
        assert abs(oracle_mod.box_spline(c * x1, c * x2, [c * t for t in a], n) - v / c ** 2) < 1e-15


def test_filter_constant_image(oracle_mod):
    rng = np.random.default_rng(5)
    H, W = 9, 11
    sc = rng.uniform(1.0, 3.0, size=(H, W, 4)).astype(np.float32)
    sc[..., 0] = np.round(sc[..., 0])
    sc[..., 2] = np.round(sc[..., 2])
    for n in (1, 2):
        s = oracle_mod.filter(np.full((H, W), 3.25), sc, n, "clamp")
        assert np.abs(s - 3.25).max() < 1e-13


@pytest.mark.parametrize("n", [1, 2])
def test_filter_rows_reduce_to_bspline_convolution(oracle_mod, n):
    """An image constant along k2 with integer a3 is filtered by the 1-D marginal."""
    rng = np.random.default_rng(7)
    H, W = 7, 23
    h = rng.uniform(0, 1, size=W)
    img = np.tile(h, (H, 1))
    c = 1.4
    sc = np.empty((H, W, 4), np.float32)
    sc[...] = [c, c * S2, 2.0, c * S2]
    a = sc[0, 0].astype(np.float64)
    s = oracle_mod.filter(img, sc, n, "clamp")
    c1, c2 = a[0], a[1] / S2
    # the float32 scales make a1, a2/sqrt2, a4/sqrt2 differ in the last bits; use the
    # exact 1-D density of the three projected sums, evaluated with SciPy B-splines
    from scipy.integrate import quad
    def b(deg, width, y):
        kn = width * (np.arange(deg + 2) - (deg + 1) / 2)
        return float(np.nan_to_num(BSpline.basis_element(kn, extrapolate=False)(y))) / width
    def kernel(x):
        if n == 1:
            # conv of three boxes: integrate box(c1) * box(c2) against box(c2)
            g = lambda y: quad(lambda z: b(0, c1, x - y - z) * b(0, c2, z), -c2 / 2, c2 / 2,
                               points=[x - y - c1 / 2, x - y + c1 / 2])[0]
            return quad(lambda y: g(y) * b(0, c2, y), -c2 / 2, c2 / 2, limit=200)[0]
        knots = c * (np.arange(3 * n + 1) - 1.5 * n)
        return float(np.nan_to_num(BSpline.basis_element(knots, extrapolate=False)(x))) / c
    for m1 in (3, 11, 19):
        want = 0.0
        for k1 in range(m1 - 8, m1 + 9):
            want += h[min(max(k1, 0), W - 1)] * kernel(m1 - k1)
        tol = 1e-7 if n == 1 else 2e-6
        assert abs(s[3, m1] - want) < tol, (m1, s[3, m1], want)


def test_filter_mirror_and_transpose(oracle_mod):
    rng = np.random.default_rng(9)
    H, W = 8, 10
    img = rng.uniform(0, 1, size=(H, W))
    sc = rng.uniform(1, 3, size=(H, W, 4)).astype(np.float32)
    for n in (1, 2):
        s = oracle_mod.filter(img, sc, n)
        sm = oracle_mod.filter(img[:, ::-1].copy(), sc[:, ::-1][..., [0, 3, 2, 1]].copy(), n)
        assert np.abs(sm[:, ::-1] - s).max() < 1e-14
        st = oracle_mod.filter(img.T.copy(), sc.transpose(1, 0, 2)[..., [2, 1, 0, 3]].copy(), n)
        assert np.abs(st.T - s).max() < 1e-14
        # zero border differs from clamp near the edge only
        sz = oracle_mod.filter(img, sc, n, "zero")
        assert np.abs(sz - s).max() > 1e-3


@pytest.mark.parametrize("n", [1, 2, 3])
def test_zero_border_is_clamp_on_a_zero_frame(oracle_mod, n):
    """The zero border rule, pinned through the clamp rule: embedding the image in a frame of
    zeros wider than every pixel's support makes clamp-to-edge read zeros wherever the zero
    rule would, and only there.  A wrong edge index, a one-sided or off-by-one zero region in
    the zero branch, would break the equality (it is exact: the same terms in the same order)."""
    rng = np.random.default_rng(40 + n)
    H, W = 9, 11
    img = rng.uniform(0.5, 1.5, size=(H, W))
    sc = rng.uniform(0.5, 3.5, size=(H, W, 4)).astype(np.float32)
    R = int(math.ceil(0.5 * n * (3.5 + 2 * 3.5 / S2))) + 2   # beyond every support radius
    big = np.zeros((H + 2 * R, W + 2 * R))
    big[R:R + H, R:R + W] = img
    bsc = np.ones((H + 2 * R, W + 2 * R, 4), np.float32)
    bsc[R:R + H, R:R + W] = sc
    sz = oracle_mod.filter(img, sc, n, "zero")
    sc_frame = oracle_mod.filter(big, bsc, n, "clamp")[R:R + H, R:R + W]
    assert np.array_equal(sz, sc_frame)
    # and the zero rule really differs from clamp at the edges (so the frame matters)
    assert np.abs(sz - oracle_mod.filter(img, sc, n, "clamp")).max() > 1e-2


def test_zero_border_mirror_and_transpose(oracle_mod):
    """The symmetries of the filter hold under the zero rule too: mirroring k1 swaps the two
    diagonal scales, transposing swaps a1 and a3 (the direction set maps onto itself); the
    zero frame is symmetric, so an asymmetric zero region would break them."""
    rng = np.random.default_rng(44)
    H, W = 7, 10
    img = rng.uniform(0, 1, size=(H, W))
    sc = rng.uniform(0.5, 3, size=(H, W, 4)).astype(np.float32)
    for n in (1, 2, 3):
        s = oracle_mod.filter(img, sc, n, "zero")
        sm = oracle_mod.filter(img[:, ::-1].copy(), sc[:, ::-1][..., [0, 3, 2, 1]].copy(), n, "zero")
        assert np.abs(sm[:, ::-1] - s).max() < 1e-14
        st = oracle_mod.filter(img.T.copy(), sc.transpose(1, 0, 2)[..., [2, 1, 0, 3]].copy(), n, "zero")
        assert np.abs(st.T - s).max() < 1e-14
        s180 = oracle_mod.filter(img[::-1, ::-1].copy(), sc[::-1, ::-1].copy(), n, "zero")
        assert np.abs(s180[::-1, ::-1] - s).max() < 1e-14


def test_filter_sampled_pixels_match_full(oracle_mod):
    rng = np.random.default_rng(11)
    img = rng.uniform(0, 1, size=(12, 13))
    sc = rng.uniform(1, 4, size=(12, 13, 4)).astype(np.float32)
    full = oracle_mod.filter(img, sc, 2)
    pix = np.array([0, 5, 77, 155])
    assert np.array_equal(oracle_mod.filter(img, sc, 2, pixels=pix), full.reshape(-1)[pix])


# ----------------------------------------------------------------------------
# stage 1 (eq. RS): the n-fold running sums along l1..l4
# ----------------------------------------------------------------------------
STEPS = [(1, 0), (1, 1), (0, 1), (-1, 1)]


def cone_weights(v, n):
    """Number of weighted ways to write v = sum_d t_d l_d (t_d >= 0); an n-fold
    running sum weights t steps by C(t + n - 1, n - 1)."""
    v1, v2 = v
    tot = 0
    for t2 in range(0, v2 + 1):
        for t4 in range(0, v2 - t2 + 1):
            t3 = v2 - t2 - t4
            t1 = v1 - t2 + t4
            if t1 < 0:
                continue
            w = 1
            for t in (t1, t2, t3, t4):
                w *= math.comb(t + n - 1, n - 1)
            tot += w
    return tot


@pytest.mark.parametrize("n", [1, 2, 3])
def test_preintegrate_brute_force_cone(oracle_mod, n):
    rng = np.random.default_rng(20 + n)
    Hq, Wq = 5, 6
    win = rng.integers(-50, 200, size=(Hq, Wq))
    g = oracle_mod.preintegrate(win, n)
    for r in range(Hq):
        for c in range(Wq):
            want = sum(int(win[rs, cs]) * cone_weights((c - cs, r - rs), n)
                       for rs in range(Hq) for cs in range(Wq) if rs <= r)
            assert g[r, c] == want, (r, c)


@pytest.mark.parametrize("n", [1, 2])
def test_preintegrate_lattice_differences_invert(oracle_mod, n):
    """prod_d (1 - E^{l_d})^n g = f wherever every difference stays in the window."""
    rng = np.random.default_rng(30 + n)
    Hq, Wq = 9, 10
    win = rng.integers(0, 256, size=(Hq, Wq))
    g = oracle_mod.preintegrate(win, n).astype(object)
    d = g
    for (s1, s2) in STEPS:
        for _ in range(n):
            nd = np.zeros_like(d)
            for r in range(Hq):
                for c in range(Wq):
                    rr, cc = r - s2, c - s1
                    prev = d[rr, cc] if (0 <= rr < Hq and 0 <= cc < Wq) else None
                    nd[r, c] = None if (d[r, c] is None or prev is None) else d[r, c] - prev
            d = nd
    checked = 0
    for r in range(Hq):
        for c in range(Wq):
            if d[r, c] is not None:
                assert d[r, c] == win[r, c]
                checked += 1
    assert checked > 10


def test_preintegrate_extension_matches_large_zero_padding(oracle_mod):
    """The right-hand triangle makes the window result equal to the one on a far larger domain."""
    rng = np.random.default_rng(41)
    Hq, Wq = 6, 7
    win = rng.integers(0, 256, size=(Hq, Wq))
    big = np.zeros((Hq, Wq + 40), np.int64)
    big[:, :Wq] = win
    gb = oracle_mod.preintegrate(big, 2)
    assert np.array_equal(oracle_mod.preintegrate(win, 2), gb[:, :Wq])


def test_preintegrate_wrap_is_exact_modulo_2_64(oracle_mod):
    """Stage 1 is linear and homogeneous: scaling the input by 2^s scales every exact value by
    2^s, so the wrapped result of 2^s x must be (exact result of x) * 2^s modulo 2^64."""
    rng = np.random.default_rng(43)
    Hq, Wq, n, s = 40, 45, 3, 30
    win = rng.integers(0, 256, size=(Hq, Wq))
    exact = oracle_mod.preintegrate(win, n)  # fits int64
    with pytest.raises(OverflowError):
        oracle_mod.preintegrate(win << s, n)
    wrapped = oracle_mod.preintegrate(win << s, n, wrap=True)
    expect = (exact.astype(np.uint64) << np.uint64(s)).view(np.int64)
    assert np.array_equal(wrapped, expect)
