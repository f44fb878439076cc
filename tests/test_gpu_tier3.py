"""GPU parity of the third launch tier: restart windows larger than a workgroup's LDS, one
per 2x2 block of tiles, pre-integrated in a slice of global scratch and read by the mesh from an
LDS buffer in bands of rows, each pixel's taps taken up by the band that holds the first row of
their stencil.

The central 16x16 tile of each image has scales large enough for a window beyond the full LDS
(130 to 170 elements square plus the extension triangle, against 20k elements of LDS), so it
runs in tier 3 over two or three bands; its neighbours stay in tier 1.  Every pixel of that tile is
compared with the oracle (a sample at order 3 and for the bilinear model, whose oracle sums are
slow).  Windows so wide that a band would own fewer than 8 rows are read from the scratch slice
itself; that case is checked on constant images, which every box spline reproduces exactly
(partition of unity), at scales whose oracle sums would take minutes.
"""
import numpy as np
import pytest

from paper_0908_3861_amd import synth

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12
TOL_F32 = 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def bsf(torch_dev):
    from paper_0908_3861_amd import binding
    binding.load()
    return binding


def centre_tile_case(seed, lo, hi, dtype=np.float32):
    rng = np.random.default_rng(seed)
    H, W = 48, 48
    img = (rng.integers(0, 256, size=(H, W)).astype(np.uint8) if dtype == np.uint8
           else synth.unit_grid_image(rng, H, W, dtype))
    sc = synth.uniform_scales(rng, H, W, 1.0, 3.0)
    sc[16:32, 16:32] = rng.uniform(lo, hi, size=(16, 16, 4)).astype(np.float32)
    tile = (np.arange(16, 32)[:, None] * W + np.arange(16, 32)[None, :]).reshape(-1)
    return rng, img, sc, tile


def filt(bsf, torch, img, sc, n, path, border="clamp", model=-1, a_max=None):
    ti = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    ts = torch.from_numpy(np.ascontiguousarray(sc)).cuda()
    out = bsf.filter(ti, ts, n, path=path, border=border, a_max=a_max, model=model)
    st = bsf.default_context().device_error()
    return out.cpu().numpy().astype(np.float64), st


def rel_max(s, o):
    return float(np.abs(s - o).max() / np.abs(o).max())


@pytest.mark.parametrize("n,path,border,lo,hi,count,dtype", [
    (1, "f64", "clamp", 44.0, 48.0, 256, np.float32),
    (1, "f32tiled", "clamp", 44.0, 48.0, 256, np.float32),
    (2, "f64", "clamp", 16.0, 22.0, 256, np.float32),
    (2, "f32tiled", "clamp", 16.0, 22.0, 256, np.float32),
    (2, "f64", "zero", 16.0, 22.0, 128, np.float32),
    (2, "f32tiled", "zero", 24.0, 30.0, 96, np.float32),
    (2, "f64", "clamp", 24.0, 30.0, 96, np.uint8),
    (2, "f64", "zero", 16.0, 22.0, 96, np.float64),
    (3, "f64", "clamp", 14.0, 18.0, 16, np.float32),
    (3, "f32tiled", "clamp", 14.0, 18.0, 16, np.float32),
    (3, "f64", "zero", 14.0, 18.0, 16, np.uint8),
])
def test_banded_scratch_tile_against_oracle(bsf, torch_dev, oracle_mod, n, path, border, lo, hi, count, dtype):
    rng, img, sc, tile = centre_tile_case(300 + 10 * n + (path == "f32tiled") + 2 * (border == "zero") +
                                          4 * (dtype == np.uint8), lo, hi, dtype)
    s, st = filt(bsf, torch_dev, img, sc, n, path, border, a_max=hi)
    assert st == 0
    assert np.isfinite(s).all()
    pix = tile if count >= tile.size else rng.choice(tile, count, replace=False)
    pix = np.concatenate([pix, rng.choice(img.size, 8, replace=False)])  # and a few tier-1 pixels
    o = oracle_mod.filter(img.astype(np.float64), sc, n, border, pixels=pix)
    err = rel_max(s.reshape(-1)[pix], o)
    print(f"tier 3 banded, order {n} {path} {border} {np.dtype(dtype).name}: rel_max {err:.3g} over {pix.size} pixels")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err


@pytest.mark.parametrize("model,path,count", [(0, "f64", 32), (1, "f64", 8), (1, "f32tiled", 8)])
def test_banded_scratch_tile_continuous_models(bsf, torch_dev, oracle_mod, model, path, count):
    rng, img, sc, tile = centre_tile_case(330 + model, 44.0, 48.0, np.float64)
    s, st = filt(bsf, torch_dev, img, sc, 1, path, model=model, a_max=48.0)
    assert st == 0
    pix = rng.choice(tile, count, replace=False)
    o = oracle_mod.filter_model(img, sc, 1, model, "clamp", pixels=pix)
    err = rel_max(s.reshape(-1)[pix], o)
    print(f"tier 3 banded, model {model} {path}: rel_max {err:.3g}")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err


@pytest.mark.parametrize("n,lo,hi,path", [(1, 420, 440, "f64"), (1, 420, 440, "f32tiled"), (2, 210, 220, "f32tiled")])
def test_windows_too_wide_for_bands_read_scratch(bsf, torch_dev, n, lo, hi, path):
    """Windows about 1,080 elements wide leave a band fewer than 8 owned rows: the mesh reads
    the scratch slice itself.  With integer scales a1, a3 (a2, a4 anything) the integer
    translates of the box spline sum to one -- its Fourier transform vanishes at every nonzero
    lattice frequency, where one of the two axis factors sinc(pi a1 j1), sinc(pi a3 j2) is zero --
    so a constant image comes back unchanged.  (Order 2 on the float64 path is out of range
    there: the exact running sums of such a window exceed int64 for any digit split.)"""
    rng = np.random.default_rng(340 + n)
    H, W = 40, 36
    img = np.full((H, W), 0.625, np.float32)
    sc = synth.uniform_scales(rng, H, W, 1.0, 3.0)
    sc[16:32, 16:32] = rng.uniform(lo, hi, size=(16, 16, 4)).astype(np.float32)
    sc[..., 0] = np.round(sc[..., 0])
    sc[..., 2] = np.round(sc[..., 2])
    s, st = filt(bsf, torch_dev, img, sc, n, path, a_max=float(hi))
    assert st == 0
    err = float(np.abs(s - 0.625).max() / 0.625)
    big = float(np.abs(s[16:32, 16:32] - 0.625).max() / 0.625)
    print(f"wide scratch windows, order {n} {path}: rel_max {err:.3g} (the wide tile alone {big:.3g})")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err


@pytest.mark.parametrize("n,path", [(1, "f64"), (2, "f64"), (1, "f32tiled"), (2, "f32tiled")])
def test_full_and_ragged_blocks(bsf, torch_dev, oracle_mod, n, path):
    """Tier 3 filters 2x2 blocks of tiles from one window: full blocks (the four blocks of
    [0, 64)^2), a block holding only the image's ragged corner tile (8x8 pixels at
    [64, 72)^2), and the tier-1 tiles between."""
    rng = np.random.default_rng(350 + n + (path == "f32tiled"))
    H = W = 72
    img = synth.unit_grid_image(rng, H, W, np.float32)
    sc = synth.uniform_scales(rng, H, W, 1.0, 3.0)
    lo, hi = (44.0, 48.0) if n == 1 else (16.0, 22.0)
    sc[:64, :64] = rng.uniform(lo, hi, size=(64, 64, 4)).astype(np.float32)
    sc[64:, 64:] = rng.uniform(lo, hi, size=(8, 8, 4)).astype(np.float32)
    s, st = filt(bsf, torch_dev, img, sc, n, path, a_max=hi)
    assert st == 0
    assert np.isfinite(s).all()
    full = rng.choice(64 * 64, 64, replace=False)
    full = (full // 64) * W + full % 64
    corner = (np.arange(64, 72)[:, None] * W + np.arange(64, 72)[None, :]).reshape(-1)
    pix = np.concatenate([full, corner, rng.choice(H * W, 8, replace=False)])
    o = oracle_mod.filter(img.astype(np.float64), sc, n, pixels=pix)
    err = rel_max(s.reshape(-1)[pix], o)
    print(f"tier-3 blocks, order {n} {path}: rel_max {err:.3g} over {pix.size} pixels")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err


def test_batched_and_noalloc_blocks_equal_single_calls(bsf, torch_dev):
    """Batched calls, captured plans and the allocation-free entry point take tier-3 blocks
    exactly as single calls do (same tiers, same windows): bitwise equal outputs."""
    torch = torch_dev
    rng = np.random.default_rng(360)
    items, singles = [], []
    for (H, W, n, path) in [(40, 40, 2, "f64"), (48, 36, 1, "f32tiled"), (40, 56, 2, "f32tiled")]:
        img = torch.from_numpy(synth.unit_grid_image(rng, H, W, np.float32)).cuda()
        scn = synth.uniform_scales(rng, H, W, 1.0, 3.0)
        scn[8:40, 8:32] = rng.uniform(16.0, 22.0, size=(min(H, 40) - 8, 24, 4)).astype(np.float32)
        sc = torch.from_numpy(scn).cuda()
        items.append(dict(img=img, scales=sc, order=n, path=path, a_max=22.0))
        singles.append(bsf.filter(img, sc, n, path=path, a_max=22.0).cpu().numpy())
    outs = bsf.filter_batched(items)
    assert bsf.default_context().device_error() == 0
    for o, s1 in zip(outs, singles):
        o = o.cpu().numpy()
        assert np.array_equal(o.view(np.uint8), s1.view(np.uint8))
    for it, s1 in zip(items, singles):
        o = bsf.filter_noalloc(it["img"], it["scales"], it["order"], path=it["path"], a_max=22.0).cpu().numpy()
        assert np.array_equal(o.view(np.uint8), s1.view(np.uint8))
