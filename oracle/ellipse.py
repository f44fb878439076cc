"""Oracle for the scale field of an elliptical window (the step before the filter).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it; it shares no code with the HIP path.

The paper shapes every pixel's window through the covariance of the four-direction box
spline (Section 4: the covariance is controlled by the scale vector; Theorem 4.3 with
a_k = sigma sqrt(24/N) for the isotropic limit) and leaves the construction of the
scale map from the desired ellipse open (Section 8).  The definition used here:

* A unit segment of length a along r_theta is a uniform density with variance a^2/12 along
  r_theta, so the order-n box spline with scales a (directions theta_k = (k-1) pi/4) has the
  covariance  C(a) = (n/12) sum_k a_k^2 r_k r_k^T  (the n-fold self-convolution adds n
  copies).
* The target is the covariance of the ellipse, Sigma = R_phi diag(s_major^2, s_minor^2) R_phi^T
  (phi from the first lattice axis toward the second).
* The scales are  a_k = sqrt(w_k),  w the minimiser of  ||C(sqrt w) - Sigma||_F  over
  w_k >= a_min^2 (the filter's smallest admissible scale), and among the minimisers the
  one with the least sum_k w_k^2.  For Sigma = sigma^2 I this gives a_k = sigma sqrt(6/n):
  Theorem 4.3's sqrt(24/N) sigma at N = 4, spread over n convolution factors.

It is computed here by brute force: for every set of coordinates held at the bound, the
least-squares problem in the others (numpy's minimum-norm lstsq), keeping the feasible
candidates; the answer is the candidate with the smallest residual, then the smallest
norm.  Plain float64, a pixel at a time.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

A_MIN = 0.5


def direction_tensors() -> np.ndarray:
    """r_k r_k^T as the 3-vectors (xx, xy, yy) for theta_k = (k-1) pi/4, k = 1..4."""
    out = []
    for k in range(4):
        th = k * math.pi / 4
        c, s = math.cos(th), math.sin(th)
        out.append((c * c, c * s, s * s))
    return np.array(out).T  # 3 x 4


def target_covariance(s_major: float, s_minor: float, phi: float) -> np.ndarray:
    c, s = math.cos(phi), math.sin(phi)
    R = np.array([[c, -s], [s, c]])
    return R @ np.diag([s_major ** 2, s_minor ** 2]) @ R.T


def covariance_of_scales(a, n: int) -> np.ndarray:
    """C(a) = (n/12) sum_k a_k^2 r_k r_k^T (Section 4, the n-fold box spline)."""
    t = direction_tensors()
    v = (n / 12.0) * (t @ (np.asarray(a, dtype=np.float64) ** 2))
    return np.array([[v[0], v[1]], [v[1], v[2]]])


def _frobenius_system(n: int):
    # rows (xx, sqrt2 * xy, yy): the Frobenius norm counts the off-diagonal twice
    t = (n / 12.0) * direction_tensors()
    wgt = np.array([1.0, math.sqrt(2.0), 1.0])
    return t * wgt[:, None], wgt


def scales_from_ellipse(s_major: float, s_minor: float, phi: float, n: int, a_min: float = A_MIN) -> np.ndarray:
    """The scale vector (a1..a4) of one pixel (float64)."""
    M, wgt = _frobenius_system(n)
    S = target_covariance(s_major, s_minor, phi)
    b = np.array([S[0, 0], S[0, 1], S[1, 1]]) * wgt
    lb = a_min * a_min
    best = None
    for k in range(5):
        for fixed in itertools.combinations(range(4), k):
            free = [i for i in range(4) if i not in fixed]
            w = np.full(4, lb)
            rhs = b - M[:, list(fixed)].sum(axis=1) * lb if fixed else b.copy()
            if free:
                sol, *_ = np.linalg.lstsq(M[:, free], rhs, rcond=None)
                w[free] = sol
            if np.any(w < lb * (1 - 1e-12) - 1e-15):
                continue
            w = np.maximum(w, lb)
            res = float(np.sum((M @ w - b) ** 2))
            norm = float(np.sum(w * w))
            key = (res, norm)
            if best is None or _better(key, best[0], scale=float(np.sum(b * b)) + 1.0):
                best = (key, w)
    return np.sqrt(best[1])


def _better(key, ref, scale):
    res, norm = key
    rres, rnorm = ref
    tol = 1e-12 * scale
    if res < rres - tol:
        return True
    if res > rres + tol:
        return False
    return norm < rnorm


def scales_from_ellipses(ell: np.ndarray, n: int, a_min: float = A_MIN) -> np.ndarray:
    """[..., 3] (s_major, s_minor, phi) -> [..., 4] float64 scales, pixel by pixel."""
    ell = np.asarray(ell, dtype=np.float64)
    out = np.empty(ell.shape[:-1] + (4,))
    flat_in = ell.reshape(-1, 3)
    flat_out = out.reshape(-1, 4)
    for i, (s1, s2, ph) in enumerate(flat_in):
        flat_out[i] = scales_from_ellipse(s1, s2, ph, n, a_min)
    return out
