"""GPU parity of the two-direction (rect, N = 2) filter (bsf_filter_rect) with its oracle
(oracle/rect.py), through the C ABI.

Error measure: rel_max = max|s - O| / max|O| over the compared pixels; bar 1e-12 on the float64
path (the oracle is accurate to a few ulps), 1e-5 on the float32-output path.  Sizes span
several tiles with ragged edges.
"""
import numpy as np
import pytest

import oracle.rect as R
from paper_0908_3861_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
F32_TOL = 1e-5
ALL = [(n, n1) for n in (1, 2, 3) for n1 in (-1, 0, 1, 2, 3)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_max(s, o):
    s, o = np.asarray(s, np.float64), np.asarray(o, np.float64)
    return float(np.abs(s - o).max() / max(np.abs(o).max(), 1e-300))


def run(torch, img, sc, n, n1, path="f64", border="clamp", a_max=None, check=True):
    from paper_0908_3861_amd import binding
    dev = torch.device("cuda:0")
    out = binding.filter_rect(torch.from_numpy(np.ascontiguousarray(img)).to(dev),
                              torch.from_numpy(np.ascontiguousarray(sc)).to(dev), n, n1, path, border, a_max,
                              check=check)
    return out.cpu().numpy().astype(np.float64)


def scales2(rng, H, W, lo, hi):
    return rng.uniform(lo, hi, size=(H, W, 2)).astype(np.float32)


@pytest.mark.parametrize("n,n1", ALL)
def test_parity_every_order_and_model(torch_dev, n, n1):
    rng = np.random.default_rng(4000 + 10 * n + n1)
    H, W = (70, 83) if n1 <= 1 else (37, 45)
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = scales2(rng, H, W, 0.5, 8.0)
    o = R.filter_rect(img, sc, n, n1, "clamp")
    s = run(torch_dev, img, sc, n, n1)
    s32 = run(torch_dev, img, sc, n, n1, path="f32tiled")
    err, err32 = rel_max(s, o), rel_max(s32, o)
    print(f"rect order {n} model {n1}: rel_max f64 {err:.2e}, f32 {err32:.2e}")
    assert err < TOL and err32 < F32_TOL


@pytest.mark.parametrize("n,n1", [(1, -1), (2, 0), (3, 1), (2, 2), (1, 3)])
def test_zero_border_and_dtypes(torch_dev, n, n1):
    rng = np.random.default_rng(4100 + 10 * n + n1)
    H, W = 35, 41
    for dtype in (np.uint8, np.float32, np.float64):
        if dtype == np.uint8:
            img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
        else:
            img = synth.unit_grid_image(rng, H, W, dtype)
        sc = scales2(rng, H, W, 0.5, 6.0)
        o = R.filter_rect(img.astype(np.float64), sc, n, n1, "zero")
        assert rel_max(run(torch_dev, img, sc, n, n1, border="zero"), o) < TOL, dtype


def test_edge_cases(torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(4200)
    for (H, W) in [(1, 1), (1, 9), (7, 1), (32, 32), (33, 31), (8, 64)]:
        img = synth.unit_grid_image(rng, H, W, np.float64)
        sc = scales2(rng, H, W, 0.5, 3.0)
        sc[0, 0] = 0.5
        for n, n1, border in [(1, -1, "clamp"), (3, -1, "zero"), (2, 1, "clamp"), (2, 3, "zero")]:
            o = R.filter_rect(img, sc, n, n1, border)
            assert rel_max(run(torch, img, sc, n, n1, border=border), o) < TOL, (H, W, n, n1, border)
    # unit scales at order 1: the identity (rect = beta^2_(1,1))
    img = synth.unit_grid_image(rng, 40, 50, np.float64)
    sc = np.ones((40, 50, 2), np.float32)
    assert np.array_equal(run(torch, img, sc, 1, -1), img)


def test_scale_errors(torch_dev):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(4300)
    H, W = 30, 40
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = scales2(rng, H, W, 1.0, 4.0)
    sc[3, 4, 0] = np.nan
    sc[10, 20, 1] = 0.25
    sc[20, 30, 0] = 5.0  # above the bound given below
    ctx = binding.default_context(0)
    out = run(torch, img, sc, 2, -1, a_max=4.0, check=False)
    assert ctx.device_error() == 5 and ctx.device_error() == 0
    bad = np.zeros((H, W), bool)
    bad[3, 4] = bad[10, 20] = bad[20, 30] = True
    assert np.all(np.isnan(out[bad])) and np.all(np.isfinite(out[~bad]))
    good = sc.copy()
    good[bad] = 1.0
    o = R.filter_rect(img, good, 2, -1)
    assert rel_max(out[~bad], o[~bad]) < TOL
    lim = binding.filter_rect_max_scale(3, 3)
    assert 10.0 < lim < 1e4
    with pytest.raises(binding.BsfError) as ei:
        run(torch, img, np.ones_like(sc), 3, 3, a_max=lim * 2)
    assert ei.value.status == 4
    with pytest.raises(binding.BsfError):
        run(torch, img, np.ones_like(sc), 2, 4)  # model 4 is not provided


@pytest.mark.parametrize("n,n1", [(1, -1), (3, 3), (2, 0)])
def test_largest_windows(torch_dev, n, n1):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    lim = binding.filter_rect_max_scale(n, n1)
    rng = np.random.default_rng(4400 + n)
    H, W = 40, 36
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = scales2(rng, H, W, 0.5 * lim, lim)
    sc[0, :3] = np.float32(lim)
    s = run(torch, img, sc, n, n1, border="clamp", a_max=lim)
    pix = np.concatenate([[0, 1, 2, W * H - 1], np.random.default_rng(3).choice(H * W, 40, replace=False)])
    o = R.filter_rect(img, sc, n, n1, "clamp", pix)
    assert rel_max(s.reshape(-1)[pix], o) < TOL


def test_full_size_sampled(torch_dev):
    """The rect workload: 2048 x 2048 uint8 blurred noise, smooth scales in [1, 16] along each
    axis, order 2, impulse model, in the launch the bench times, on sampled pixels."""
    torch = torch_dev
    img, sc = synth.rect_workload()
    s = run(torch, img, sc, 2, -1, a_max=16.0)
    H, W = img.shape
    pr = np.random.default_rng(11)
    pix = np.concatenate([pr.choice(H * W, 400, replace=False), [0, W - 1, (H - 1) * W, H * W - 1, 31, 32]])
    o = R.filter_rect(img.astype(np.float64), sc, 2, -1, "clamp", pix)
    err = rel_max(s.reshape(-1)[pix], o)
    print(f"rect full size: rel_max {err:.2e} on {len(pix)} pixels")
    assert err < TOL
