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
