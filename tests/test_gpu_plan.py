"""Captured batch plans (bsf_batch_plan_*), called through the C ABI.

One graph is captured per plan and replayed for batches of different sizes, orders and
paths; between the replays the program does its own eager work and synchronises.  Every
replay's outputs must equal, bitwise, what bsf_filter writes for each job alone, and a job
whose scales break the contract must report its error alone.
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


def _batch(torch, rng, specs):
    items = []
    for (H, W, n, path, hi, blk) in specs:
        img = synth.unit_grid_image(rng, H, W, np.float64 if path == "f64" else np.float32)
        sc = synth.uniform_scales(rng, H, W, 1.0, hi)
        if blk:
            sc[16:32, 16:32] = rng.uniform(*blk, size=(16, 16, 4)).astype(np.float32)
        items.append(dict(img=torch.from_numpy(img).cuda(), scales=torch.from_numpy(sc).cuda(), order=n, path=path))
    return items


def _alone(bsf, ctx, items, a_max):
    return [bsf.filter(it["img"], it["scales"], it["order"], path=it["path"], a_max=a_max, ctx=ctx) for it in items]


def test_plan_replays_equal_lone_calls(bsf, torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(801)
    ctx = bsf.Context()
    a_max = 24.0
    plan = bsf.BatchPlan(ctx, max_jobs=8, max_tiles=2048, a_max=a_max)
    # windows in every tier: large-scale blocks push order-2 tiles past the LDS (tier 3)
    b1 = _batch(torch, rng, [(70, 83, 2, "f64", 4.0, (18.0, 24.0)), (33, 20, 1, "f32tiled", 3.0, None),
                             (40, 36, 3, "f32tiled", 2.0, (6.0, 8.0)), (17, 64, 3, "f64", 2.0, None),
                             (48, 48, 2, "f32tiled", 3.0, (10.0, 12.0))])
    b2 = _batch(torch, rng, [(20, 19, 1, "f64", 3.0, None), (64, 40, 2, "f64", 5.0, None)])
    ref1 = _alone(bsf, ctx, b1, a_max)
    ref2 = _alone(bsf, ctx, b2, a_max)
    torch.cuda.synchronize()
    for rep, (batch, ref) in enumerate([(b1, ref1), (b2, ref2), (b1, ref1), (b1, ref1), (b2, ref2)]):
        outs = plan.run(batch)
        torch.cuda.synchronize()
        assert plan.job_status() == [0] * len(batch)
        for k, (o, r) in enumerate(zip(outs, ref)):
            assert torch.equal(o, r), (rep, k)
        # the program's own eager work between replays
        _alone(bsf, ctx, b2[:1], a_max)
        torch.cuda.synchronize()
        print(f"replay {rep}: {len(batch)} jobs equal to lone calls")
    ctx.check_device()
    plan.close()
    ctx.close()


def test_plan_reports_each_jobs_error(bsf, torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(802)
    ctx = bsf.Context()
    plan = bsf.BatchPlan(ctx, max_jobs=4, max_tiles=512, a_max=6.0)
    batch = _batch(torch, rng, [(30, 30, 2, "f64", 4.0, None), (25, 40, 1, "f32tiled", 4.0, None),
                                (18, 18, 3, "f64", 3.0, None)])
    batch[1]["scales"][5, 7, 2] = 0.25
    ref = _alone(bsf, ctx, [batch[0], batch[2]], 6.0)
    outs = plan.run(batch)
    assert plan.job_status() == [0, 5, 0]
    assert torch.equal(outs[0], ref[0]) and torch.equal(outs[2], ref[1])
    assert torch.isnan(outs[1][5, 7])
    # the next run starts clean
    good = [batch[0], batch[2]]
    outs = plan.run(good)
    assert plan.job_status() == [0, 0]
    assert torch.equal(outs[0], ref[0]) and torch.equal(outs[1], ref[1])
    ctx.check_device()
    plan.close()
    ctx.close()


def test_plan_rejects_batches_beyond_its_capacity(bsf, torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(803)
    ctx = bsf.Context()
    plan = bsf.BatchPlan(ctx, max_jobs=2, max_tiles=16, a_max=4.0)
    small = _batch(torch, rng, [(16, 16, 1, "f64", 3.0, None)] * 3)
    with pytest.raises(bsf.BsfError) as ei:
        plan.run(small)  # three jobs, two slots
    assert ei.value.status == 1
    big = _batch(torch, rng, [(80, 80, 1, "f64", 3.0, None)])
    with pytest.raises(bsf.BsfError):
        plan.run(big)  # 25 tiles, 16 held
    with pytest.raises(bsf.BsfError):
        plan.run([dict(small[0], a_max=8.0)])  # scales bounded above the plan's a_max
    outs = plan.run(small[:2])
    assert plan.job_status() == [0, 0]
    ref = _alone(bsf, ctx, small[:2], 4.0)
    assert all(torch.equal(o, r) for o, r in zip(outs, ref))
    plan.close()
    ctx.close()
