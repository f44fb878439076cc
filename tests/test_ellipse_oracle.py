"""Pins of the ellipse -> scale-vector oracle (oracle/ellipse.py) against facts it does not
compute itself: the box spline's own moments, Theorem 4.3's isotropic scales, a library
bounded least-squares solver, and the symmetries of the direction set."""
import math
import warnings

import numpy as np
import pytest

from oracle import ellipse as E

S2 = math.sqrt(2.0)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_isotropic_scales_follow_theorem_4_3(n):
    """Sigma = sigma^2 I: every a_k = sigma sqrt(24/N) / sqrt(n) with N = 4 directions
    (Theorem 4.3's scales, the variance spread over the n convolution factors)."""
    for sigma in (1.0, 2.5, 7.0):
        for phi in (0.0, 0.4, 2.0):
            a = E.scales_from_ellipse(sigma, sigma, phi, n)
            assert np.allclose(a, sigma * math.sqrt(24.0 / 4.0 / n), rtol=1e-12)


@pytest.mark.parametrize("n,ell", [(1, (2.2, 1.4, 0.35)), (2, (1.8, 1.3, 2.1)), (3, (1.5, 1.1, -0.7))])
def test_box_spline_of_the_scales_has_the_target_covariance(oracle_mod, n, ell):
    """Midpoint-rule second moments of B_a (the C oracle's box spline) equal the ellipse's
    covariance R diag(s_major^2, s_minor^2) R^T for a reachable ellipse."""
    a = E.scales_from_ellipse(*ell, n)
    assert np.all(a > 0.5)  # an interior solution
    h = 1.0 / 20
    R1 = 0.5 * n * (a[0] + (a[1] + a[3]) / S2)
    R2 = 0.5 * n * (a[2] + (a[1] + a[3]) / S2)
    xs = np.arange(-R1 - h / 2, R1 + h, h)
    ys = np.arange(-R2 - h / 2, R2 + h, h)
    m0, M = 0.0, np.zeros((2, 2))
    for x in xs:
        for y in ys:
            v = oracle_mod.box_spline(x, y, a, n)
            if v:
                m0 += v
                M += v * np.outer([x, y], [x, y])
    m0 *= h * h
    M *= h * h
    target = E.target_covariance(*ell)
    assert abs(m0 - 1.0) < 2e-3
    assert np.abs(M - target).max() < 5e-3 * np.abs(target).max()


def test_unreachable_ellipses_are_projected_in_the_frobenius_norm():
    """An elongated ellipse between lattice directions (or one smaller than the smallest
    admissible kernel) has no exact scale vector; the oracle's residual equals that of a
    bounded least-squares solver (scipy.optimize.lsq_linear)."""
    from scipy.optimize import lsq_linear
    rng = np.random.default_rng(7)
    for _ in range(40):
        n = int(rng.integers(1, 4))
        s1 = float(rng.uniform(0.1, 12.0))
        s2 = s1 * float(rng.uniform(0.05, 0.5))
        phi = float(rng.uniform(0, math.pi))
        a = E.scales_from_ellipse(s1, s2, phi, n)
        S = E.target_covariance(s1, s2, phi)
        C = E.covariance_of_scales(a, n)
        res = float(np.sum((C - S) ** 2))
        t = (n / 12.0) * E.direction_tensors()
        wgt = np.array([1.0, S2, 1.0])
        A = t * wgt[:, None]
        b = np.array([S[0, 0], S[0, 1], S[1, 1]]) * wgt
        lib = lsq_linear(A, b, bounds=(0.25, np.inf), method="bvls", tol=1e-14)
        ref = float(np.sum((A @ lib.x - b) ** 2))
        assert res <= ref + 1e-9 * (1.0 + float(np.sum(b * b))), (s1, s2, phi, n, res, ref)
        assert np.all(a >= 0.5 - 1e-15)


def test_reachable_ellipses_are_reproduced_exactly():
    rng = np.random.default_rng(8)
    for _ in range(40):
        n = int(rng.integers(1, 4))
        s1 = float(rng.uniform(2.0, 10.0))
        s2 = s1 * float(rng.uniform(0.85, 1.0))  # mild elongation: always reachable
        phi = float(rng.uniform(0, math.pi))
        a = E.scales_from_ellipse(s1, s2, phi, n)
        C = E.covariance_of_scales(a, n)
        S = E.target_covariance(s1, s2, phi)
        assert np.abs(C - S).max() < 1e-12 * np.abs(S).max()


def test_symmetries_of_the_direction_set():
    """Swapping the two lattice axes maps phi to pi/2 - phi and the directions (0, 45, 90,
    135 degrees) to (90, 45, 0, 135): a -> (a3, a2, a1, a4).  phi and phi + pi describe the
    same ellipse."""
    rng = np.random.default_rng(9)
    for _ in range(20):
        n = int(rng.integers(1, 4))
        s1 = float(rng.uniform(0.3, 9.0))
        s2 = s1 * float(rng.uniform(0.1, 1.0))
        phi = float(rng.uniform(0, math.pi))
        a = E.scales_from_ellipse(s1, s2, phi, n)
        b = E.scales_from_ellipse(s1, s2, math.pi / 2 - phi, n)
        c = E.scales_from_ellipse(s1, s2, phi + math.pi, n)
        assert np.allclose(b, [a[2], a[1], a[0], a[3]], rtol=1e-9, atol=1e-12)
        assert np.allclose(c, a, rtol=1e-9, atol=1e-12)


def test_tie_break_least_sum_of_fourth_powers_on_anisotropic_ellipses():
    """A reachable ellipse fixes three moments of four scales: the exact solutions form a
    segment (one free parameter, t = (w2 + w4)/2 in w = a^2).  The oracle must return the
    point of that segment with the least sum a_k^4 = sum w_k^2, subject to a_k >= 0.5.  Pinned
    against a general-purpose constrained minimiser (SciPy SLSQP on sum w^2 under the three
    moment equalities and the bounds), on anisotropic ellipses at many angles, including ones
    where the bound a_k >= 0.5 is active and ones where it is not."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(10)
    checked = active = 0
    for _ in range(60):
        n = int(rng.integers(1, 4))
        s1 = float(rng.uniform(1.0, 9.0))
        s2 = s1 * float(rng.uniform(0.35, 0.95))
        phi = float(rng.uniform(0, math.pi))
        S = E.target_covariance(s1, s2, phi)
        t = (n / 12.0) * E.direction_tensors()
        b = np.array([S[0, 0], S[0, 1], S[1, 1]])
        a = E.scales_from_ellipse(s1, s2, phi, n)
        C = E.covariance_of_scales(a, n)
        if np.abs(C - S).max() > 1e-10 * np.abs(S).max():
            continue  # not reachable: the projection is pinned elsewhere
        # in units of the target's size, so that the solver's tolerances are relative
        unit = float(np.trace(S)) * 12.0 / n
        tt, bb = t * 12.0 / n, b * 12.0 / (n * unit)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)  # SLSQP clips its trial steps to the bounds
            res = minimize(lambda w: float(np.dot(w, w)), np.full(4, 0.5), jac=lambda w: 2.0 * w, method="SLSQP",
                           bounds=[(0.25 / unit, None)] * 4,
                           constraints=[{"type": "eq", "fun": lambda w: tt @ w - bb, "jac": lambda w: tt}],
                           options={"ftol": 1e-14, "maxiter": 1000})
        assert res.success, res.message
        assert np.abs(tt @ res.x - bb).max() < 1e-9
        w = a * a / unit
        assert np.allclose(w, res.x, rtol=1e-6, atol=1e-7), (s1, s2, phi, n, w, res.x)
        checked += 1
        active += int(np.min(a) < 0.5 * (1 + 1e-9))
    assert checked >= 30 and active >= 1 and checked - active >= 5, (checked, active)
