"""bsf_filter_noalloc: the allocation-free variant of bsf_filter, called through the C ABI.

Its work area is a fixed array per GPU that keeps the previous call's contents, so two calls
in a row (the second on a smaller image, with fewer tiles and smaller windows) must each give
exactly what bsf_filter gives for the same job.
"""
import ctypes

import numpy as np
import pytest

from paper_0908_3861_amd import synth

pytestmark = pytest.mark.gpu


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


def _case(torch, rng, H, W, lo, hi, block_scale):
    img = torch.from_numpy(synth.unit_grid_image(rng, H, W, np.float64)).cuda()
    sc = synth.uniform_scales(rng, H, W, lo, hi)
    if block_scale:
        sc[16:32, 16:32] = rng.uniform(*block_scale, size=(16, 16, 4)).astype(np.float32)
    return img, torch.from_numpy(sc).cuda()


def test_noalloc_equals_filter_on_consecutive_calls(bsf, torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(701)
    ctx = bsf.Context()
    lib = bsf.load()
    cases = [
        # (H, W, scales, block of large scales, order, path, a_max): tiers 1+2+3, then 1+2, then 1
        (70, 83, (1.0, 4.0), (18.0, 24.0), 2, "f64", 24.0),
        (40, 36, (1.0, 3.0), (8.0, 9.0), 2, "f32tiled", 9.0),
        (20, 19, (1.0, 3.0), None, 1, "f64", 3.0),
    ]
    for (H, W, (lo, hi), blk, n, path, a_max) in cases:
        img, sc = _case(torch, rng, H, W, lo, hi, blk)
        ref = bsf.filter(img, sc, n, path=path, a_max=a_max, ctx=ctx, check=True)
        out = torch.full_like(ref, float("nan"))
        j, _ = bsf.make_job(img, sc, n, path=path, a_max=a_max, out=out)
        st = lib.bsf_filter_noalloc(ctx.handle, ctypes.byref(j), bsf._stream_ptr(None))
        assert st == 0, lib.bsf_last_error(ctx.handle)
        ctx.check_device()
        print(f"noalloc {H}x{W} n={n} {path}: equal = {torch.equal(out, ref)}")
        assert torch.equal(out, ref), (H, W, n, path)
    ctx.close()


def test_noalloc_rejects_work_area_beyond_its_array(bsf, torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(702)
    img, sc = _case(torch, rng, 24, 24, 1.0, 3.0, None)
    ctx = bsf.Context()
    # a_max = 3000 plans restart windows of tens of millions of elements: one window slice
    # alone exceeds the fixed array, so the call fails before launching anything
    with pytest.raises(bsf.BsfError) as ei:
        bsf.filter_noalloc(img, sc, 2, a_max=3000.0, ctx=ctx)
    assert ei.value.status == 2
    assert "fixed" in str(ei.value)
    # the context still works afterwards, through both entry points
    ref = bsf.filter(img, sc, 2, a_max=3.0, ctx=ctx, check=True)
    out = bsf.filter_noalloc(img, sc, 2, a_max=3.0, ctx=ctx, check=True)
    assert torch.equal(out, ref)
    ctx.close()
