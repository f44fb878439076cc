"""Pins of the one-dimensional oracle (Section 3) against facts that do not come from it.

* scipy's B-spline basis elements (a library evaluation of beta_a^N, Section 2 eq. definition);
* numerical quadrature of the model convolution beta^{n1} * beta_a^{n-1};
* Proposition 3.1 itself, the two steps (running sums, then the finite-difference mask on the
  B-spline-interpolated running sums), in exact rational arithmetic with the B-splines from the
  Cox-de Boor recursion -- a different algorithm from the oracle's truncated-power closed form;
* partition of unity and reproduction of linear signals at integer scales, a moving-average
  brute force for the box (n = 1), and symmetry under reversal;
* for the prefiltered models (n1 = 2, 3): the closed-form impulse response of the inverse
  interpolation filter, rho z^|k| (high-precision mpmath), scipy's B-spline prefilter in the
  interior of a long signal, and the projection of a reproduced polynomial, whose value
  follows from the moments of the B-spline alone (p(m) + p''(m) n a^2 / 24).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

import oracle.filter1d as F

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def scipy_bspline(x, a, N):
    """beta_a^N(x) from scipy's basis element on the knots a (j - (N+1)/2), j = 0..N+1.

    A basis element on N+2 knots spanning a(N+1) integrates to a, so beta_a^N = B / a."""
    knots = a * (np.arange(N + 2) - (N + 1) / 2)
    B = BSpline.basis_element(knots, extrapolate=False)
    v = B(np.asarray(x, dtype=np.float64))
    return np.nan_to_num(v) / a


@pytest.mark.parametrize("n", [2, 3, 4])
def test_impulse_model_kernel_is_scipy_bspline(n):
    rng = np.random.default_rng(10 + n)
    for a in list(rng.uniform(0.5, 12.0, 6).astype(np.float32)) + [np.float32(1), np.float32(4)]:
        R = int(F.support_radius(a, n, -1)) + 1
        xs = np.arange(-R, R + 1)
        ours = np.array([float(F.kernel_value(int(x), a, n, -1)) for x in xs])
        ref = scipy_bspline(xs, float(a), n - 1)
        np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-14 / float(a))


def test_box_is_half_open():
    # beta_a^0 = 1/a on (-a/2, a/2] (Section 2): a = 2 covers offsets 0 and 1, not -1
    assert [F.kernel_value(x, 2.0, 1) for x in (-1, 0, 1, 2)] == [0, Fraction(1, 2), Fraction(1, 2), 0]
    assert [F.kernel_value(x, 3.0, 1) for x in (-2, -1, 0, 1, 2)] == [0] + [Fraction(1, 3)] * 3 + [0]
    # a = 2.5: (-1.25, 1.25] holds -1, 0, 1
    assert [F.kernel_value(x, 2.5, 1) for x in (-2, -1, 0, 1, 2)] == [0] + [Fraction(2, 5)] * 3 + [0]


@pytest.mark.parametrize("n1,n", [(0, 1), (0, 2), (1, 1), (1, 3), (0, 3), (2, 1), (2, 3), (3, 2)])
def test_model_kernel_is_the_convolution(n1, n):
    rng = np.random.default_rng(20 + 3 * n1 + n)
    for a in rng.uniform(0.5, 6.0, 4).astype(np.float32):
        a = float(a)
        R = int(F.support_radius(a, n, n1)) + 1
        for x in range(-R, R + 1):
            # (beta^{n1} * beta_a^{n-1})(x) = int beta^{n1}(y) beta_a^{n-1}(x - y) dy
            lo, hi = -(n1 + 1) / 2, (n1 + 1) / 2
            brk = sorted(set([lo + i for i in range(n1 + 2)] +
                             [x + a * (j - n / 2) for j in range(n + 1)]))
            brk = [b for b in brk if lo < b < hi]
            val, _ = integrate.quad(lambda y: scipy_bspline(y, 1.0, n1) * scipy_bspline(x - y, a, n - 1),
                                    lo, hi, points=brk or None, epsabs=1e-15, epsrel=1e-13, limit=200)
            assert abs(float(F.kernel_value(x, a, n, n1)) - val) < 1e-12, (a, x)


# --- Proposition 3.1, two steps, exact -------------------------------------------------------

def cox_de_boor(x: Fraction, D: int) -> Fraction:
    """beta^D(x), unit scale, by the Cox-de Boor recursion on the knots -(D+1)/2 + i."""
    knots = [Fraction(-(D + 1), 2) + i for i in range(D + 2)]
    # degree-0 pieces on half-open intervals (t_i, t_{i+1}] (the box convention of Section 2)
    B = [Fraction(1) if knots[i] < x <= knots[i + 1] else Fraction(0) for i in range(D + 1)]
    for d in range(1, D + 1):
        B = [(x - knots[i]) / d * B[i] + (knots[i + d + 1] - x) / d * B[i + 1] for i in range(D + 1 - d)]
    return B[0]


def prop31(f, scales, n, n1, m_list):
    """s[m] by Proposition 3.1 with zero extension: g = n-fold running sum (u_1^n) of c,
    F(x) = sum_k g[k] beta^{n1+n}(x + tau - k), s[m] = Delta_a^n F(m), tau = (a-1) n / 2.
    c = f for n1 <= 1; for n1 >= 2 the oracle's coefficients (their own pins are below)."""
    L = len(f)
    D = n1 + n
    pad = 64
    if n1 >= 2:
        c = F.coefficients(f, n1, "zero", -pad, L + pad)
    else:
        c = [Fraction(0)] * pad + [Fraction(float(v)) for v in f] + [Fraction(0)] * pad
    g = c
    for _ in range(n):
        acc, out = Fraction(0), []
        for v in g:
            acc += v
            out.append(acc)
        g = out
    res = []
    for m in m_list:
        a = Fraction(float(np.float32(scales[m])))
        tau = (a - 1) * n / 2
        s = Fraction(0)
        for j in range(n + 1):
            x = m - a * j + tau
            Fx = Fraction(0)
            for k in range(math.floor(x - (D + 1) / 2) - 1, math.ceil(x + (D + 1) / 2) + 2):
                w = cox_de_boor(x - k, D)
                if w:
                    Fx += g[k + pad] * w
            s += (-1) ** j * math.comb(n, j) * Fx
        res.append(s / a ** n)
    return res


@pytest.mark.parametrize("n1,n", [(-1, 1), (-1, 2), (-1, 3), (0, 1), (0, 2), (1, 2), (1, 3), (2, 1), (2, 2),
                                  (3, 1), (3, 3)])
def test_oracle_equals_proposition_31_exactly(n1, n):
    rng = np.random.default_rng(30 + 4 * n1 + n)
    L = 24
    f = rng.integers(-9, 10, L).astype(np.float64)
    # exact binary fractions, non-integer and integer, above and below 1
    scales = rng.choice([0.5, 0.75, 1.0, 1.25, 2.0, 2.375, 3.0, 3.5, 4.125, 5.0], L).astype(np.float32)
    ms = list(range(8, 16))
    ref = prop31(f, scales, n, n1, ms)
    ours = F.filter1d_exact(f, scales, n, n1, "zero", ms)
    if n1 <= 1:
        assert ours == ref
    else:  # the two prefilter blocks are truncated differently (far below 1e-30)
        assert all(abs(o - r) < Fraction(1, 10 ** 30) for o, r in zip(ours, ref))


# --- invariants -------------------------------------------------------------------------------

@pytest.mark.parametrize("n1,n", [(-1, 1), (-1, 2), (-1, 3), (0, 2), (1, 3)])
def test_constants_and_ramps_are_reproduced_at_integer_scales(n1, n):
    rng = np.random.default_rng(40 + n)
    L = 80
    sc = rng.integers(1, 7, L).astype(np.float32)
    ms = list(range(30, 50))
    assert all(v == 1 for v in F.filter1d_exact(np.ones(L), sc, n, n1, "clamp", ms))
    if n1 == -1 and n == 1:
        ms = [m for m in ms if sc[m] % 2 == 1]   # the half-open box shifts even widths by 1/2
    ramp = np.arange(L, dtype=np.float64)
    assert F.filter1d_exact(ramp, sc, n, n1, "clamp", ms) == [Fraction(m) for m in ms]


def test_box_is_the_moving_average():
    rng = np.random.default_rng(50)
    L = 60
    f = rng.standard_normal(L)
    sc = rng.uniform(0.5, 9.0, L).astype(np.float32)
    ours = F.filter1d_exact(f, sc, 1, -1, "zero")
    for m in range(L):
        a = Fraction(float(sc[m]))
        ks = [k for k in range(m - 10, m + 11) if -a / 2 < m - k <= a / 2 and 0 <= k < L]
        assert ours[m] == sum(Fraction(float(f[k])) for k in ks) / a


@pytest.mark.parametrize("n1,n", [(-1, 2), (-1, 3), (0, 2), (1, 1)])
def test_reversal_symmetry(n1, n):
    rng = np.random.default_rng(60 + n)
    L = 50
    f = rng.standard_normal(L)
    sc = rng.uniform(0.5, 7.0, L).astype(np.float32)
    fwd = F.filter1d_exact(f, sc, n, n1, "clamp")
    bwd = F.filter1d_exact(f[::-1].copy(), sc[::-1].copy(), n, n1, "clamp")
    assert fwd == bwd[::-1]


def test_rounding_and_batch():
    rng = np.random.default_rng(70)
    sig = rng.standard_normal((3, 40))
    sc = rng.uniform(1, 5, (3, 40)).astype(np.float32)
    full = F.filter1d_batch(sig, sc, 2, 0, "clamp")
    assert full.shape == (3, 40)
    pts = [(0, 3), (2, 39), (1, 0)]
    np.testing.assert_array_equal(F.filter1d_batch(sig, sc, 2, 0, "clamp", pts),
                                  [full[b, m] for b, m in pts])
    ex = F.filter1d_exact(sig[1], sc[1], 2, 0, "clamp", [7])[0]
    assert full[1, 7] == float(ex)


# --- the prefiltered models (n1 = 2, 3) --------------------------------------------------------

@pytest.mark.parametrize("n1", [2, 3])
def test_prefilter_impulse_response_is_the_two_sided_exponential(n1):
    """The inverse of b^{n1} = (b1, b0, b1) is rho z^|k|: z the root inside the unit circle of
    b1 z^2 + b0 z + b1 (z = 2 sqrt2 - 3, sqrt3 - 2) and rho = 1 / (b1 (z - 1/z))."""
    import mpmath
    mpmath.mp.dps = 60
    b0, b1 = (mpmath.mpf(3) / 4, mpmath.mpf(1) / 8) if n1 == 2 else (mpmath.mpf(2) / 3, mpmath.mpf(1) / 6)
    z = (-b0 + mpmath.sqrt(b0 * b0 - 4 * b1 * b1)) / (2 * b1)
    rho = 1 / (b1 * (z - 1 / z))
    assert abs(rho - (mpmath.sqrt(2) if n1 == 2 else mpmath.sqrt(3))) < mpmath.mpf(10) ** -50
    L = 121
    f = np.zeros(L)
    f[60] = 1.0
    c = F.coefficients(f, n1, "zero", 20, 101)
    for k in range(20, 101):
        exact = rho * z ** abs(k - 60)
        assert abs(mpmath.mpf(c[k - 20].numerator) / c[k - 20].denominator - exact) < mpmath.mpf(10) ** -30, k


@pytest.mark.parametrize("n1", [2, 3])
def test_prefilter_interior_matches_scipy(n1):
    from scipy import ndimage
    rng = np.random.default_rng(80 + n1)
    L = 400
    f = rng.standard_normal(L)
    ours = np.array([float(v) for v in F.coefficients(f, n1, "clamp", 100, 300)])
    ref = ndimage.spline_filter1d(f, order=n1, mode="mirror")[100:300]
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n1,n", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_prefiltered_model_projects_polynomials_by_their_moments(n1, n):
    """A polynomial of degree <= n1 is its own model; its projection onto beta_a^{n-1} is
    p(m) + p''(m) Var/2 with Var = n a^2 / 12 (odd moments vanish), away from the ends."""
    rng = np.random.default_rng(90 + 4 * n1 + n)
    L = 300
    coef = [Fraction(3), Fraction(-2), Fraction(1, 2), Fraction(1, 64) if n1 == 3 else Fraction(0)]
    p = lambda x: sum(c * Fraction(x) ** i for i, c in enumerate(coef))  # noqa: E731
    p2 = lambda x: 2 * coef[2] + 6 * coef[3] * x  # noqa: E731
    f = np.array([float(p(k)) for k in range(L)])
    assert all(Fraction(float(f[k])) == p(k) for k in range(L))  # exact in float64
    sc = rng.uniform(0.5, 9.0, L).astype(np.float32)
    ms = list(range(120, 180, 3))
    ours = F.filter1d_exact(f, sc, n, n1, "clamp", ms)
    for m, v in zip(ms, ours):
        a = Fraction(float(sc[m]))
        want = p(m) + p2(m) * n * a * a / 24
        assert abs(v - want) < Fraction(1, 10 ** 25), (m, float(v - want))


@pytest.mark.parametrize("n1", [2, 3])
def test_prefiltered_constant_is_reproduced_at_any_scale(n1):
    rng = np.random.default_rng(100 + n1)
    L = 40
    sc = rng.uniform(0.5, 7.0, L).astype(np.float32)
    for n in (1, 2, 3):
        out = F.filter1d_exact(np.full(L, 2.5), sc, n, n1, "clamp")
        assert all(abs(v - Fraction(5, 2)) < Fraction(1, 10 ** 30) for v in out)
