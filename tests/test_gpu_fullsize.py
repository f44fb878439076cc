"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

The oracle evaluates sampled output pixels one by one (direct box-spline sums); the GPU
runs the whole image exactly as bench.py does (same a_max, path, dtype).  The float64
path must stay within 1e-12 (rel_max over the sample), the float32-output path within
its stated 1e-5.
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


def sampled_rel_max(out, img, sc, n, count, rng, oracle_mod):
    pix = np.sort(rng.choice(img.size, size=count, replace=False))
    o = oracle_mod.filter(img.astype(np.float64), sc, n, pixels=pix)
    s = out.reshape(-1)[pix].astype(np.float64)
    return float(np.abs(s - o).max() / np.abs(o).max())


def test_plain_workload_2048_order2_f64(torch_dev, oracle_mod):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    job = synth.config_job("plain")
    out = binding.filter(torch.from_numpy(job.image).cuda(), torch.from_numpy(job.scales).cuda(), 2, path="f64",
                         a_max=16.0, check=True).cpu().numpy()
    err = sampled_rel_max(out, job.image, job.scales, 2, 400, np.random.default_rng(601), oracle_mod)
    print(f"plain 2048^2 f64 rel_max {err:.3g}")
    assert err < TOL_F64


def test_plain_workload_2048_order2_f32tiled(torch_dev, oracle_mod):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    job = synth.config_job("plain")
    out = binding.filter(torch.from_numpy(job.image).cuda(), torch.from_numpy(job.scales).cuda(), 2,
                         path="f32tiled", a_max=16.0, check=True).cpu().numpy()
    err = sampled_rel_max(out, job.image, job.scales, 2, 400, np.random.default_rng(602), oracle_mod)
    assert err < TOL_F32


def test_precision_workload_4096_order2(torch_dev, oracle_mod):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    job = synth.config_job("precision")
    img = torch.from_numpy(job.image).cuda()
    sc = torch.from_numpy(job.scales).cuda()
    rng = np.random.default_rng(603)
    for path, tol in (("f32tiled", TOL_F32), ("f64", TOL_F64)):
        out = binding.filter(img, sc, 2, path=path, a_max=32.0, check=True).cpu().numpy()
        err = sampled_rel_max(out, job.image, job.scales, 2, 150, rng, oracle_mod)
        print(f"precision 4096^2 {path} rel_max {err:.3g}")
        assert err < tol, path


def test_batched_workload_64_images(torch_dev, oracle_mod):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    jobs = synth.batch_jobs(count=64)
    items = [dict(img=torch.from_numpy(j.image).cuda(), scales=torch.from_numpy(j.scales).cuda(), order=j.order,
                  path="f32tiled", a_max=8.0) for j in jobs]
    outs = binding.filter_batched(items, check=True)
    rng = np.random.default_rng(604)
    worst = 0.0
    for k, j in enumerate(jobs):  # 64 sampled pixels of every image
        err = sampled_rel_max(outs[k].cpu().numpy(), j.image, j.scales, j.order, 64, rng, oracle_mod)
        worst = max(worst, err)
        assert err < TOL_F32, (k, j.order, j.image.shape)
    print(f"batched 64 images: worst rel_max over 64 pixels each {worst:.3g}")


def test_padded_pitches(torch_dev, oracle_mod):
    """Rows of the input, the scales and the output longer than the image (views)."""
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(605)
    H, W, n = 37, 45, 2
    big = torch.from_numpy(rng.integers(0, 256, size=(H, W + 11)).astype(np.uint8)).cuda()
    bigsc = torch.from_numpy(synth.uniform_scales(rng, H, W + 5, 1.0, 6.0)).cuda()
    img, sc = big[:, :W], bigsc[:, :W]
    assert img.stride(0) == W + 11 and sc.stride(0) == 4 * (W + 5)
    outbig = torch.zeros((H, W + 7), dtype=torch.float64, device=img.device)
    out = outbig[:, :W]
    binding.filter(img, sc, n, path="f64", out=out, check=True)
    o = oracle_mod.filter(img.cpu().numpy().astype(np.float64), np.ascontiguousarray(sc.cpu().numpy()), n)
    s = out.cpu().numpy()
    assert float(np.abs(s - o).max() / np.abs(o).max()) < TOL_F64
    assert float(outbig[:, W:].abs().max()) == 0.0  # nothing written past the image
