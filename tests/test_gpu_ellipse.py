"""GPU parity of the scale field of elliptical windows (bsf_scales_from_ellipses) with the
brute-force oracle (oracle/ellipse.py), through the C ABI.

The kernel evaluates the closest-covariance scales in float64 and rounds them to float32
(the filter's scale format); the oracle's float64 scales, rounded to float32, must agree
to one float32 unit in the last place.
"""
import math

import numpy as np
import pytest

from oracle import ellipse as E
from paper_0908_3861_amd import synth

pytestmark = pytest.mark.gpu

ULP32 = 2.0 ** -23


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def check(got, ell, n):
    ref = E.scales_from_ellipses(ell, n).astype(np.float32).astype(np.float64)
    got = got.astype(np.float64)
    assert np.all(np.abs(got - ref) <= ULP32 * np.abs(ref) * 1.0001), np.abs(got - ref).max()


def mixed_ellipses(rng, h, w):
    """Random ellipses with the edge cases mixed in: isotropic, lattice-aligned, very
    elongated (unreachable), below the smallest kernel, angles outside [0, pi)."""
    ell = np.empty((h, w, 3), np.float32)
    s1 = np.exp(rng.uniform(np.log(0.1), np.log(30.0), size=(h, w)))
    ell[..., 0] = s1
    ell[..., 1] = s1 * rng.uniform(0.02, 1.0, size=(h, w))
    ell[..., 2] = rng.uniform(-4.0, 8.0, size=(h, w))
    flat = ell.reshape(-1, 3)
    k = flat.shape[0]
    idx = rng.choice(k, size=k // 4, replace=False)
    q = len(idx) // 4
    flat[idx[:q], 1] = flat[idx[:q], 0]                                          # isotropic
    flat[idx[q:2 * q], 2] = (rng.integers(0, 8, size=q) * (np.pi / 4)).astype(np.float32)  # lattice directions
    flat[idx[2 * q:3 * q], 1] = flat[idx[2 * q:3 * q], 0] * 0.01                  # needle-like
    flat[idx[3 * q:], :2] = rng.uniform(0.01, 0.3, size=(len(idx) - 3 * q, 2))   # below the smallest kernel
    return ell


@pytest.mark.parametrize("n", [1, 2, 3])
def test_parity_mixed_ellipses(torch_dev, n):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(700 + n)
    H, W = 23, 301  # two blocks per row, ragged tail
    ell = mixed_ellipses(rng, H, W)
    out = binding.scales_from_ellipses(torch.from_numpy(ell).cuda(), n)
    binding.default_context().check_device()
    check(out.cpu().numpy(), ell, n)


def test_padded_pitches_and_rows_left_alone(torch_dev):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(710)
    H, W = 9, 40
    big = torch.from_numpy(mixed_ellipses(rng, H, W + 7)).cuda()
    ell = big[:, :W]
    outbig = torch.zeros((H, W + 5, 4), dtype=torch.float32, device="cuda")
    out = outbig[:, :W]
    binding.scales_from_ellipses(ell, 2, out=out)
    check(out.cpu().numpy(), ell.cpu().numpy(), 2)
    assert float(outbig[:, W:].abs().max()) == 0.0


def test_invalid_ellipses_flag_and_nan(torch_dev):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    ell = np.ones((2, 5, 3), np.float32)
    ell[0, 1, 0] = np.nan
    ell[1, 3, 1] = -1.0
    ell[1, 4, 2] = np.inf
    ctx = binding.default_context()
    out = binding.scales_from_ellipses(torch.from_numpy(ell).cuda(), 2).cpu().numpy()
    assert ctx.device_error() == 5  # BSF_ERR_SCALE_RANGE
    bad = np.zeros((2, 5), bool)
    bad[0, 1] = bad[1, 3] = bad[1, 4] = True
    assert np.all(np.isnan(out[bad]))
    assert np.all(np.isfinite(out[~bad]))
    assert ctx.device_error() == 0  # the flag was read and cleared
    with pytest.raises(binding.BsfError):
        binding.scales_from_ellipses(torch.from_numpy(ell).cuda(), 4)


def test_full_size_field_sampled(torch_dev):
    """The benchmark's 2048x2048 field, in its launch configuration, on sampled pixels."""
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(synth.CONFIGS["ellipse"]["seed"])
    ell = synth.ellipse_field(rng, 2048, 2048)
    out = binding.scales_from_ellipses(torch.from_numpy(ell).cuda(), 2).cpu().numpy()
    binding.default_context().check_device()
    pix = np.random.default_rng(711).choice(2048 * 2048, size=600, replace=False)
    check(out.reshape(-1, 4)[pix], ell.reshape(-1, 3)[pix], 2)


def test_filter_with_scales_from_ellipses(torch_dev, oracle_mod):
    """The two steps composed on the GPU: an elliptical field drives the filter, and the
    result matches the oracle filter fed the same scales."""
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(712)
    H, W = 29, 37
    ell = synth.ellipse_field(rng, H, W, 1.0, 3.0, 3.0, sigma=6.0)
    img = synth.blurred_u8_image(rng, H, W, 2.0)
    sc = binding.scales_from_ellipses(torch.from_numpy(ell).cuda(), 2)
    s = binding.filter(torch.from_numpy(img).cuda(), sc, 2, path="f64", check=True).cpu().numpy()
    o = oracle_mod.filter(img.astype(np.float64), sc.cpu().numpy(), 2)
    assert float(np.abs(s - o).max() / np.abs(o).max()) < 1e-12
