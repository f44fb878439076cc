"""The conditioning instrumentation (oracle/kappa.py): its two-stage sum -- exact running
sums of eq. RS on the pixel's own window, taps and shift of eq. final_eqn at order n, the
box spline at the integration scale -- must reproduce the oracle's direct projection to within
the rounding of its terms, at interior, edge and corner pixels, both borders, orders 1-3.
A wrong shift, tap position, coefficient sign or window would leave an O(1) mismatch."""
import numpy as np
import pytest

import oracle
from oracle import kappa as K
from paper_0908_3861_amd import synth


@pytest.mark.parametrize("n,border", [(1, "clamp"), (1, "zero"), (2, "clamp"), (2, "zero"), (3, "clamp")])
def test_two_stage_sum_reproduces_the_projection(n, border):
    rng = np.random.default_rng(6000 + 10 * n + len(border))
    H, W = 24, 27
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = synth.uniform_scales(rng, H, W, 1.0, 3.0 if n < 3 else 1.5)
    pix = np.array([12 * W + 13, 0, W - 1, (H - 1) * W, 5 * W + 20] if n < 3 else [12 * W + 13])
    s = oracle.filter(img, sc, n, border, pixels=pix)
    k, worst = K.kappa(img, sc, n, pix, s, border)
    print(f"n={n} {border}: kappa {k}, mismatch {worst:.2e}")
    assert worst < 1e-15
    assert np.all(k >= 1.0)


def test_kappa_grows_as_scales_shrink():
    """Smaller scales cancel more (the mask's gain (a1a2a3a4)^-n meets the same sums)."""
    rng = np.random.default_rng(6100)
    img = synth.unit_grid_image(rng, 20, 20, np.float64)
    ks = []
    for a in (4.0, 2.0, 1.0):
        sc = np.full((20, 20, 4), a, np.float32)
        p = np.array([10 * 20 + 10])
        ks.append(K.kappa(img, sc, 2, p, oracle.filter(img, sc, 2, pixels=p))[0][0])
    assert ks[0] < ks[1] < ks[2]


def _regrouped_sum(img, scales, n, m1, m2, border):
    """The two-stage sum with the taps of each pair (k2, k4) regrouped: the window combined with
    the finite-difference weights along r1 and r3 at integer shifts (k1 a1, k3 a3), then one
    interpolant per pair at the (k1, k3) = (0, 0) tap's position -- the GPU's combined-tap form,
    written out from the identity on the oracle's own primitives."""
    import itertools
    import math
    a1, a2, a3, a4 = (float(v) for v in np.asarray(scales, np.float32)[m2, m1])
    i1, i3 = int(a1), int(a3)
    a2p, a4p = a2 / K.SQRT2, a4 / K.SQRT2
    R1, R2 = 0.5 * n * (a1 + a2p + a4p), 0.5 * n * (a3 + a2p + a4p)
    x0, y0 = m1 - math.ceil(R1) - 2 * n - 1, m2 - math.ceil(R2) - 3 * n - 1
    x1, y1 = m1 + math.ceil(R1) + n + 1, m2 + math.ceil(R2) + 1
    win = K._window(img, x0, x1, y0, y1, border)
    g = oracle.preintegrate(np.rint(win * 2.0 ** 24).astype(np.int64), n)
    tx, ty = 0.5 * n * (a1 + a2p - a4p - 1.0), 0.5 * n * (a2p + a3 + a4p - 3.0)
    total, mag = 0.0, 0.0
    for k2, k4 in itertools.product(range(n + 1), repeat=2):
        c24 = (-1) ** (k2 + k4) * math.comb(n, k2) * math.comb(n, k4)
        px = m1 + tx - (k2 * a2p - k4 * a4p)
        py = m2 + ty - (k2 * a2p + k4 * a4p)
        for j2 in range(math.ceil(py - 1.5 * n), math.floor(py + 1.5 * n) + 1):
            for j1 in range(math.ceil(px - 1.5 * n), math.floor(px + 1.5 * n) + 1):
                w = oracle.box_spline(px - j1, py - j2, K.B_SCALE, n)
                if w == 0.0:
                    continue
                h = 0
                for k1, k3 in itertools.product(range(n + 1), repeat=2):
                    r, c = j2 - k3 * i3 - y0, j1 - k1 * i1 - x0
                    assert 0 <= r < g.shape[0] and 0 <= c < g.shape[1]  # inside the pixel's window
                    h += (-1) ** (k1 + k3) * math.comb(n, k1) * math.comb(n, k3) * int(g[r, c])
                total += c24 * w * h
                mag += abs(c24 * w * h)
    f = 2.0 ** n / (a1 * a2 * a3 * a4) ** n / 2.0 ** 24
    return total * f, mag * f


@pytest.mark.parametrize("n,border", [(1, "clamp"), (2, "zero"), (3, "clamp")])
def test_integer_a1_a3_regrouping_reproduces_the_projection(n, border):
    """With integer a1 and a3 the (k1, k3) taps of a pair share one cell, and the regrouped sum
    equals the oracle's direct projection to the rounding of its terms; with a1 off the integers
    the same regrouping is wrong by O(1) (so the test would catch a form taken where it does not
    hold)."""
    rng = np.random.default_rng(6200 + n)
    H, W = 22, 23
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = synth.uniform_scales(rng, H, W, 1.0, 2.5 if n < 3 else 1.6)
    sc[..., 0] = rng.integers(1, 4 if n < 3 else 3, size=(H, W))
    sc[..., 2] = rng.integers(1, 4 if n < 3 else 3, size=(H, W))
    for (m1, m2) in [(11, 10), (0, 0), (W - 1, 5)]:
        s = oracle.filter(img, sc, n, border, pixels=np.array([m2 * W + m1]))[0]
        r, mag = _regrouped_sum(img, sc, n, m1, m2, border)
        assert abs(r - s) <= 1e-14 * mag, (n, m1, m2, r, s)
    sc2 = sc.copy()
    sc2[10, 11, 0] += 0.37
    s = oracle.filter(img, sc2, n, border, pixels=np.array([10 * W + 11]))[0]
    r, mag = _regrouped_sum(img, sc2, n, 11, 10, border)
    assert abs(r - s) > 1e-6 * max(abs(s), 1e-300)
