"""GPU parity of the continuous image models with the four-direction box spline
(bsf_filter_model, Section 6 with phi = beta^m x beta^m, m = 0, 1, order 1) against the
oracle's direct projection (oracle.filter_model), through the C ABI.

Error measure as the other parity tests: rel_max over the compared pixels, 1e-12 on the
float64 path, 1e-5 on the float32-output path."""
import numpy as np
import pytest

from paper_0908_3861_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
F32_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_max(s, o):
    return float(np.abs(np.asarray(s, np.float64) - o).max() / np.abs(o).max())


def run(torch, img, sc, model, path="f64", border="clamp", a_max=None, order=1):
    from paper_0908_3861_amd import binding
    out = binding.filter(torch.from_numpy(np.ascontiguousarray(img)).cuda(),
                         torch.from_numpy(np.ascontiguousarray(sc)).cuda(), order, path=path, border=border,
                         a_max=a_max, check=True, model=model)
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("border", ["clamp", "zero"])
def test_parity_both_paths(torch_dev, oracle_mod, model, border):
    rng = np.random.default_rng(7100 + 10 * model + len(border))
    H, W = 37, 42  # several 16x16 tiles and ragged edges
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = synth.uniform_scales(rng, H, W, 0.5, 4.0)
    pix = np.concatenate([rng.choice(H * W, 160, replace=False), [0, W - 1, (H - 1) * W, H * W - 1, 16, 17 * W]])
    o = oracle_mod.filter_model(img, sc, 1, model, border, pixels=pix)
    s = run(torch_dev, img, sc, model, border=border).reshape(-1)[pix]
    s32 = run(torch_dev, img.astype(np.float32), sc, model, path="f32tiled", border=border).reshape(-1)[pix]
    err, err32 = rel_max(s, o), rel_max(s32, o)
    print(f"model {model} {border}: rel_max f64 {err:.2e}, f32 {err32:.2e}")
    assert err < TOL and err32 < F32_TOL


@pytest.mark.parametrize("model", [0, 1])
def test_dtypes_tiny_images_and_large_windows(torch_dev, oracle_mod, model):
    torch = torch_dev
    rng = np.random.default_rng(7200 + model)
    for dtype in (np.uint8, np.float32):
        img = rng.integers(0, 256, (20, 23)).astype(np.uint8) if dtype == np.uint8 else \
            synth.unit_grid_image(rng, 20, 23, np.float32)
        sc = synth.uniform_scales(rng, 20, 23, 1.0, 3.0)
        o = oracle_mod.filter_model(img.astype(np.float64), sc, 1, model, "clamp")
        assert rel_max(run(torch, img, sc, model), o) < TOL, dtype
    for (H, W) in [(1, 1), (1, 7), (6, 1)]:
        img = synth.unit_grid_image(rng, H, W, np.float64)
        sc = synth.uniform_scales(rng, H, W, 0.5, 2.0)
        for border in ("clamp", "zero"):
            o = oracle_mod.filter_model(img, sc, 1, model, border)
            assert rel_max(run(torch, img, sc, model, border=border), o) < TOL, (H, W, border)
    # windows beyond half and beyond all of the LDS (tiers 2 and 3): a block of large scales
    H, W = 36, 40
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = synth.uniform_scales(rng, H, W, 1.0, 3.0)
    sc[16:32, 16:32] = rng.uniform(30.0, 40.0, (16, 16, 4)).astype(np.float32)
    pix = np.concatenate([(np.arange(16, 32) * W + 24), rng.choice(H * W, 30, replace=False)])
    o = oracle_mod.filter_model(img, sc, 1, model, "clamp", pixels=pix)
    assert rel_max(run(torch, img, sc, model, a_max=40.0).reshape(-1)[pix], o) < TOL


def test_delta_model_is_bsf_filter_and_unsupported_pairs(torch_dev):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(7300)
    img = synth.unit_grid_image(rng, 30, 30, np.float64)
    sc = synth.uniform_scales(rng, 30, 30, 1.0, 3.0)
    a = run(torch, img, sc, -1, order=2)
    b = binding.filter(torch.from_numpy(img).cuda(), torch.from_numpy(sc).cuda(), 2, check=True).cpu().numpy()
    assert np.array_equal(a, b)
    for order, model in [(2, 0), (3, 1), (1, 2), (1, 4)]:
        with pytest.raises(binding.BsfError) as ei:
            run(torch, img, sc, model, order=order)
        assert ei.value.status == 4, (order, model)
