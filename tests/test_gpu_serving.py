"""Continuous batching: every request's result is the same in the mix as alone.

Requests of different sizes, orders, dtypes and paths are submitted together, so the
server admits them into concurrent groups on several streams; each result must be
bitwise equal to a lone bsf_filter call on the same inputs (the same kernel body runs
every tile, whatever the launch it lands in), and sampled pixels must match the
oracle within the float64 tolerance.  A request whose scales break the filter's contract
fails on its own: its future raises, the others are unaffected.
"""
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


def make_requests(rng, count):
    reqs = []
    for i in range(count):
        h, w = int(rng.integers(20, 160)), int(rng.integers(20, 160))
        n = int(rng.integers(1, 4))
        f64 = bool(i % 2)
        img = synth.unit_grid_image(rng, h, w, np.float64 if f64 else np.float32)
        sc = synth.integer_scales(rng, h, w, 1, 6)
        reqs.append((img, sc, n, "f64" if f64 else "f32tiled"))
    return reqs


@pytest.mark.parametrize("graphs", [True, False])
def test_results_in_the_mix_equal_results_alone(torch_dev, oracle_mod, graphs):
    torch = torch_dev
    from paper_0908_3861_amd import binding, serve
    rng = np.random.default_rng(501)
    reqs = make_requests(rng, 14)
    srv = serve.Server(budget_bytes=1 << 30, slots=6, streams=3, max_group=4, a_max=6.0, graphs=graphs,
                       max_tiles=4096)
    futs = [srv.submit(torch.from_numpy(img).pin_memory(), torch.from_numpy(sc).pin_memory(), n, path)
            for (img, sc, n, path) in reqs]
    outs = [f.result(timeout=120) for f in futs]
    srv.close()
    st = srv.stats()
    print(f"graphs={graphs}: {st}")
    assert st["completed"] == len(reqs) and st["failed"] == 0
    ctx = binding.Context()
    for (img, sc, n, path), got in zip(reqs, outs):
        alone = binding.filter(torch.from_numpy(img).cuda(), torch.from_numpy(sc).cuda(), n, path=path, a_max=6.0,
                               ctx=ctx).cpu()
        assert torch.equal(got, alone), (img.shape, n, path)
    ctx.check_device()
    ctx.close()
    # the mix against the oracle on sampled pixels of the float64 requests
    for (img, sc, n, path), got in zip(reqs, outs):
        if path != "f64":
            continue
        pix = rng.choice(img.size, size=24, replace=False)
        o = oracle_mod.filter(img.astype(np.float64), sc, n, pixels=pix)
        s = got.numpy().reshape(-1)[pix]
        assert np.abs(s - o).max() <= 1e-12 * np.abs(o).max(), (img.shape, n)


@pytest.mark.parametrize("bad", [0.25, float("nan")])
def test_a_failing_request_fails_alone(torch_dev, bad):
    """One request with a scale outside [0.5, 1e4] (or NaN) in a group of good ones: its
    future raises the scale-range error, every other request equals its lone result."""
    torch = torch_dev
    from paper_0908_3861_amd import binding, serve
    rng = np.random.default_rng(503)
    reqs = make_requests(rng, 6)
    img, sc, n, path = reqs[2]
    sc = sc.copy()
    sc[3, 5, 1] = bad
    reqs[2] = (img, sc, n, path)
    srv = serve.Server(budget_bytes=1 << 30, slots=8, streams=1, max_group=8, a_max=6.0, max_tiles=4096)
    # one stream: the requests queue behind each other and share groups (how they group
    # depends on timing; the plan test checks one bad job inside a single replay)
    futs = [srv.submit(torch.from_numpy(i).pin_memory(), torch.from_numpy(s).pin_memory(), k, p)
            for (i, s, k, p) in reqs]
    results = []
    for f in futs:
        try:
            results.append(f.result(timeout=120))
        except binding.BsfError as e:
            results.append(e)
    srv.close()
    assert isinstance(results[2], binding.BsfError) and results[2].status == 5, results[2]
    ctx = binding.Context()
    for k, ((i, s, o, p), got) in enumerate(zip(reqs, results)):
        if k == 2:
            continue
        alone = binding.filter(torch.from_numpy(i).cuda(), torch.from_numpy(s).cuda(), o, path=p, a_max=6.0,
                               ctx=ctx).cpu()
        assert torch.equal(got, alone), k
    ctx.check_device()
    ctx.close()
    assert srv.stats()["failed"] == 1


def test_admission_waits_for_memory(torch_dev):
    """A budget that holds one request at a time still serves every request, in order."""
    torch = torch_dev
    from paper_0908_3861_amd import serve
    rng = np.random.default_rng(502)
    reqs = make_requests(rng, 5)
    biggest = max(img.size * (img.itemsize + 16 + 8) + 4096 for img, _, _, _ in reqs)
    srv = serve.Server(budget_bytes=biggest, slots=4, streams=2, a_max=6.0, max_tiles=4096)
    futs = [srv.submit(torch.from_numpy(img), torch.from_numpy(sc), n, path) for (img, sc, n, path) in reqs]
    outs = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.stats()["failed"] == 0
    assert all(o.shape == tuple(img.shape) for o, (img, _, _, _) in zip(outs, reqs))
    assert np.all(np.isfinite(np.concatenate([o.numpy().reshape(-1) for o in outs])))
