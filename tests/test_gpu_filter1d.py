"""GPU parity of the one-dimensional scale-adaptive filter (bsf_filter1d, Section 3) with the
exact oracle (oracle/filter1d.py), through the C ABI.

Error measure: rel_max = max|s - O| / max|O| over the compared samples, bar 1e-12 (the
float64 bar of the two-dimensional path); the oracle is the correctly rounded exact
projection.  Sizes span several 256-output tiles with a ragged tail.
"""
import numpy as np
import pytest

import oracle.filter1d as F
from paper_0908_3861_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12
F32_TOL = 1e-5  # the float32-output path's stated bound
MODELS = [(n, n1) for n in (1, 2, 3) for n1 in (-1, 0, 1)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_max(s, o):
    s, o = np.asarray(s, np.float64), np.asarray(o, np.float64)
    return float(np.abs(s - o).max() / max(np.abs(o).max(), 1e-300))


def run(torch, sig, sc, n, n1, border="clamp", a_max=None, check=True, path="f64"):
    from paper_0908_3861_amd import binding
    dev = torch.device("cuda:0")
    out = binding.filter1d(torch.from_numpy(np.ascontiguousarray(sig)).to(dev),
                           torch.from_numpy(np.ascontiguousarray(sc)).to(dev), n, n1, border, a_max, check=check,
                           path=path)
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n,n1", MODELS)
def test_parity_every_order_and_model(torch_dev, n, n1):
    rng = np.random.default_rng(900 + 3 * n + n1)
    count, L = 2, 1100  # four full tiles and a ragged one per signal
    sig = synth.unit_grid_image(rng, count, L, np.float64)
    sc = rng.uniform(0.5, 12.0, size=(count, L)).astype(np.float32)
    s = run(torch_dev, sig, sc, n, n1)
    o = F.filter1d_batch(sig, sc, n, n1, "clamp")
    err = rel_max(s, o)
    print(f"order {n} model {n1}: rel_max {err:.2e}")
    assert err < TOL


@pytest.mark.parametrize("dtype", [np.uint8, np.float32, np.float64])
@pytest.mark.parametrize("border", ["clamp", "zero"])
def test_parity_dtypes_and_borders(torch_dev, dtype, border):
    rng = np.random.default_rng(950 + (0 if border == "clamp" else 7) + np.dtype(dtype).itemsize)
    count, L = 3, 700
    if dtype == np.uint8:
        sig = rng.integers(0, 256, size=(count, L)).astype(np.uint8)
    else:
        sig = synth.unit_grid_image(rng, count, L, dtype)
    sc = synth.smooth_scales_1d(rng, count, L, 0.5, 20.0, period=64)
    s = run(torch_dev, sig, sc, 2, -1, border)
    o = F.filter1d_batch(sig, sc, 2, -1, border)
    assert rel_max(s, o) < TOL


def test_edge_cases(torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(990)
    # a single sample: every tap is that sample (clamp) -> the kernel's mass at the sample
    for n, n1 in [(1, -1), (3, 1)]:
        sig = np.array([[3.25]])
        sc = np.array([[2.5]], np.float32)
        assert rel_max(run(torch, sig, sc, n, n1), F.filter1d_batch(sig, sc, n, n1)) < TOL
    # shorter than a tile, smallest scale everywhere, zero border
    sig = synth.unit_grid_image(rng, 4, 37, np.float64)
    sc = np.full((4, 37), 0.5, np.float32)
    for n, n1 in MODELS:
        assert rel_max(run(torch, sig, sc, n, n1, "zero"), F.filter1d_batch(sig, sc, n, n1, "zero")) < TOL
    # integer scales and scales equal to the bound a_max
    sig = synth.unit_grid_image(rng, 2, 600, np.float64)
    sc = rng.integers(1, 9, size=(2, 600)).astype(np.float32)
    sc[:, ::7] = 8.0
    assert rel_max(run(torch, sig, sc, 3, -1, a_max=8.0), F.filter1d_batch(sig, sc, 3, -1)) < TOL
    # exactly two tiles
    sig = synth.unit_grid_image(rng, 1, 512, np.float64)
    sc = rng.uniform(1, 6, size=(1, 512)).astype(np.float32)
    assert rel_max(run(torch, sig, sc, 2, 0), F.filter1d_batch(sig, sc, 2, 0)) < TOL


def test_padded_rows_and_large_scales(torch_dev):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(991)
    count, L, pitch = 3, 900, 1024
    sig = synth.unit_grid_image(rng, count, pitch, np.float32)
    sc = rng.uniform(40.0, 120.0, size=(count, pitch)).astype(np.float32)
    dev = torch.device("cuda:0")
    ts = torch.from_numpy(sig).to(dev)[:, :L]
    tc = torch.from_numpy(sc).to(dev)[:, :L]
    out = torch.full((count, pitch), 7.0, dtype=torch.float64, device=dev)
    binding.filter1d(ts, tc, 3, -1, "clamp", out=out[:, :L], check=True)
    got = out.cpu().numpy()
    assert np.all(got[:, L:] == 7.0)  # the row padding is not written
    o = F.filter1d_batch(sig[:, :L], sc[:, :L], 3, -1)
    assert rel_max(got[:, :L], o) < TOL


def test_scale_errors(torch_dev):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(992)
    sig = synth.unit_grid_image(rng, 2, 300, np.float64)
    sc = rng.uniform(1, 4, size=(2, 300)).astype(np.float32)
    sc[0, 10] = np.nan
    sc[1, 200] = 0.25
    sc[1, 201] = 5.0  # above the a_max given below
    ctx = binding.default_context(0)
    out = run(torch, sig, sc, 2, -1, a_max=4.0, check=False)
    assert ctx.device_error() == 5  # BSF_ERR_SCALE_RANGE, sticky until read
    assert ctx.device_error() == 0
    bad = np.zeros_like(out, bool)
    bad[0, 10] = bad[1, 200] = bad[1, 201] = True
    assert np.all(np.isnan(out[bad])) and np.all(np.isfinite(out[~bad]))
    good = sc.copy()
    good[bad] = 1.0
    o = F.filter1d_batch(sig, good, 2, -1)
    assert rel_max(out[~bad], o[~bad]) < TOL
    # a bound beyond what the on-chip window allows is refused before any launch
    lim = binding.filter1d_max_scale(3, 1)
    assert 100.0 < lim < 1e4
    with pytest.raises(binding.BsfError) as ei:
        run(torch, sig, np.ones_like(sc), 3, 1, a_max=lim * 2)
    assert ei.value.status == 4
    with pytest.raises(binding.BsfError):
        run(torch, sig, np.ones_like(sc), 4, -1)  # order 4 is not provided


@pytest.mark.parametrize("n,n1", [(1, -1), (3, 1), (2, 0)])
def test_largest_windows(torch_dev, n, n1):
    """Scales up to the largest bound the on-chip window allows (a 4096-sample window at
    order 1, the whole LDS at order 3 with the linear model), on sampled outputs."""
    torch = torch_dev
    from paper_0908_3861_amd import binding
    lim = binding.filter1d_max_scale(n, n1)
    rng = np.random.default_rng(994 + n)
    count, L = 2, 1300
    sig = synth.unit_grid_image(rng, count, L, np.float64)
    sc = rng.uniform(0.75 * lim, lim, size=(count, L)).astype(np.float32)
    sc[0, :3] = np.float32(lim)
    s = run(torch, sig, sc, n, n1, "zero", a_max=lim)
    pr = np.random.default_rng(6)
    pts = [(0, 0), (0, 1), (1, L - 1), (1, 255), (1, 256), (1, 511), (1, 512)]
    pts += [(int(b), int(m)) for b, m in zip(pr.integers(0, count, 40), pr.integers(0, L, 40))]
    o = F.filter1d_batch(sig, sc, n, n1, "zero", pts)
    assert rel_max(np.array([s[b, m] for b, m in pts]), o) < TOL


@pytest.mark.parametrize("n,n1", MODELS)
def test_f32_path_every_order_and_model(torch_dev, n, n1):
    """The float32-output path (compensated running sums, plain float64 mask) against the
    same exact oracle, at its stated bound; smallest scales (the mask's largest gain) and
    scales up to 12 on ragged signals."""
    rng = np.random.default_rng(1900 + 3 * n + n1)
    count, L = 2, 1100
    sig = synth.unit_grid_image(rng, count, L, np.float32)
    sc = rng.uniform(0.5, 12.0, size=(count, L)).astype(np.float32)
    sc[0, :300] = 0.5
    s = run(torch_dev, sig, sc, n, n1, path="f32tiled")
    o = F.filter1d_batch(sig, sc, n, n1, "clamp")
    err = rel_max(s, o)
    print(f"f32 path, order {n} model {n1}: rel_max {err:.2e}")
    assert err < F32_TOL


@pytest.mark.parametrize("n,n1", [(1, -1), (3, 1), (3, -1)])
def test_f32_path_largest_windows(torch_dev, n, n1):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    lim = binding.filter1d_max_scale(n, n1)
    rng = np.random.default_rng(1994 + n + n1)
    count, L = 2, 1300
    sig = rng.integers(0, 256, size=(count, L)).astype(np.uint8)
    sc = rng.uniform(0.5, lim, size=(count, L)).astype(np.float32)
    sc[1, :5] = np.float32(lim)
    s = run(torch, sig, sc, n, n1, "zero", a_max=lim, path="f32tiled")
    pr = np.random.default_rng(7)
    pts = [(1, 0), (1, 4), (0, L - 1), (0, 255), (0, 256)]
    pts += [(int(b), int(m)) for b, m in zip(pr.integers(0, count, 40), pr.integers(0, L, 40))]
    o = F.filter1d_batch(sig, sc, n, n1, "zero", pts)
    err = rel_max(np.array([s[b, m] for b, m in pts]), o)
    print(f"f32 path, largest windows, order {n} model {n1}: rel_max {err:.2e}")
    assert err < F32_TOL


def test_f32_path_scale_errors_and_padding(torch_dev):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(1995)
    count, L, pitch = 2, 700, 768
    sig = synth.unit_grid_image(rng, count, pitch, np.float64)
    sc = rng.uniform(1.0, 6.0, size=(count, pitch)).astype(np.float32)
    sc[1, 77] = np.inf
    dev = torch.device("cuda:0")
    out = torch.full((count, pitch), 3.0, dtype=torch.float32, device=dev)
    ctx = binding.default_context(0)
    binding.filter1d(torch.from_numpy(sig).to(dev)[:, :L], torch.from_numpy(sc).to(dev)[:, :L], 2, 0, "clamp",
                     a_max=6.0, out=out[:, :L], path="f32tiled")
    assert ctx.device_error() == 5
    got = out.cpu().numpy().astype(np.float64)
    assert np.all(got[:, L:] == 3.0) and np.isnan(got[1, 77])
    good = sc[:, :L].copy()
    good[1, 77] = 1.0
    o = F.filter1d_batch(sig[:, :L], good, 2, 0, "clamp")
    mask = np.ones((count, L), bool)
    mask[1, 77] = False
    assert rel_max(got[:, :L][mask], o[mask]) < F32_TOL


def test_full_size_sampled(torch_dev):
    """The full throughput workload (1024 signals x 65536 samples, f32, smooth scales [1,16],
    order 3, impulse model), in the launch the bench times, on sampled outputs."""
    torch = torch_dev
    rng = np.random.default_rng(synth.CONFIGS["signal1d"]["seed"])
    count, L = 1024, 65536
    sig = synth.unit_grid_image(rng, count, L, np.float32)
    sc = synth.smooth_scales_1d(rng, count, L, 1.0, 16.0)
    s = run(torch, sig, sc, 3, -1, a_max=16.0)
    pr = np.random.default_rng(5)
    pts = [(int(b), int(m)) for b, m in zip(pr.integers(0, count, 1500), pr.integers(0, L, 1500))]
    pts += [(0, 0), (count - 1, L - 1), (5, 255), (5, 256), (7, L - 257)]  # ends and tile seams
    o = F.filter1d_batch(sig, sc, 3, -1, "clamp", pts)
    got = np.array([s[b, m] for b, m in pts])
    err = rel_max(got, o)
    print(f"full size: rel_max {err:.2e} on {len(pts)} samples")
    assert err < TOL


def test_full_size_reproduces_linear_signals(torch_dev):
    """A property at any size: with integer scales the kernel sums to one and has zero mean,
    so a ramp is reproduced away from the ends (every output checked)."""
    torch = torch_dev
    rng = np.random.default_rng(993)
    count, L = 64, 65536
    ramp = np.tile(np.arange(L, dtype=np.float64) * 2.0 ** -10 - 17.0, (count, 1))
    sc = rng.integers(1, 17, size=(count, L)).astype(np.float32)
    for n, n1 in [(2, -1), (3, -1), (3, 1)]:
        s = run(torch, ramp, sc, n, n1)
        inner = slice(64, L - 64)
        err = np.abs(s[:, inner] - ramp[:, inner]).max() / np.abs(ramp).max()
        assert err < TOL, (n, n1, err)


def test_distinct_pitches_and_many_short_signals(torch_dev):
    """Signals, scales and output with three different row pitches; then 3000 signals of 7
    samples (one tile each, the signal index taken from the workgroup index)."""
    torch = torch_dev
    from paper_0908_3861_amd import binding
    rng = np.random.default_rng(996)
    dev = torch.device("cuda:0")
    count, L = 3, 600
    sig = synth.unit_grid_image(rng, count, 1000, np.float32)
    sc = rng.uniform(0.5, 9.0, size=(count, 1024)).astype(np.float32)
    out = torch.full((count, 960), -1.0, dtype=torch.float64, device=dev)
    binding.filter1d(torch.from_numpy(sig).to(dev)[:, :L], torch.from_numpy(sc).to(dev)[:, :L], 2, 1, "zero",
                     a_max=9.0, out=out[:, :L], check=True)
    got = out.cpu().numpy()
    assert np.all(got[:, L:] == -1.0)
    assert rel_max(got[:, :L], F.filter1d_batch(sig[:, :L], sc[:, :L], 2, 1, "zero")) < TOL
    count, L = 3000, 7
    sig = synth.unit_grid_image(rng, count, L, np.float64)
    sc = rng.uniform(0.5, 4.0, size=(count, L)).astype(np.float32)
    s = run(torch, sig, sc, 3, -1, a_max=4.0)
    rows = [0, 1, 1234, 2999]
    o = F.filter1d_batch(sig[rows], sc[rows], 3, -1, "clamp")
    assert rel_max(s[rows], o) < TOL
    s32 = run(torch, sig, sc, 3, -1, a_max=4.0, path="f32tiled")
    assert rel_max(s32[rows], o) < F32_TOL


# --- prefiltered models (degree 2 and 3): the IIR inverse of the interpolation filter --------

PF_MODELS = [(n, n1) for n in (1, 2, 3) for n1 in (2, 3)]


@pytest.mark.parametrize("n,n1", PF_MODELS)
@pytest.mark.parametrize("border", ["clamp", "zero"])
def test_prefiltered_models_parity(torch_dev, n, n1, border):
    """Both paths against the exact oracle (prefilter solved in rationals), ragged signals over
    several tiles, smallest scales included (the mask's largest gain)."""
    rng = np.random.default_rng(2100 + 10 * n + n1 + (0 if border == "clamp" else 5))
    count, L = 2, 1100
    sig = synth.unit_grid_image(rng, count, L, np.float64)
    sc = rng.uniform(0.5, 12.0, size=(count, L)).astype(np.float32)
    sc[1, 600:700] = 0.5
    o = F.filter1d_batch(sig, sc, n, n1, border)
    s = run(torch_dev, sig, sc, n, n1, border)
    err = rel_max(s, o)
    s32 = run(torch_dev, sig.astype(np.float32), sc, n, n1, border, path="f32tiled")
    err32 = rel_max(s32, o)
    print(f"prefiltered model {n1}, order {n}, {border}: rel_max f64 {err:.2e}, f32 {err32:.2e}")
    assert err < TOL and err32 < F32_TOL


def test_prefiltered_models_edge_cases(torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(2190)
    for n, n1 in PF_MODELS:
        # one sample (clamp: a constant signal, reproduced exactly by the model)
        sig = np.array([[3.25]])
        sc = np.array([[2.5]], np.float32)
        assert rel_max(run(torch, sig, sc, n, n1), F.filter1d_batch(sig, sc, n, n1)) < TOL
        # shorter than the prefilter's reach, zero border, smallest scale
        sig = synth.unit_grid_image(rng, 3, 20, np.float64)
        sc = np.full((3, 20), 0.5, np.float32)
        assert rel_max(run(torch, sig, sc, n, n1, "zero"), F.filter1d_batch(sig, sc, n, n1, "zero")) < TOL
    # u8 input, exactly two tiles, a bound equal to the largest scale
    sig = rng.integers(0, 256, size=(2, 512)).astype(np.uint8)
    sc = rng.uniform(1, 6, size=(2, 512)).astype(np.float32)
    sc[:, ::9] = 6.0
    assert rel_max(run(torch, sig, sc, 2, 3, a_max=6.0), F.filter1d_batch(sig, sc, 2, 3)) < TOL


@pytest.mark.parametrize("n,n1", [(1, 2), (3, 3)])
def test_prefiltered_largest_windows(torch_dev, n, n1):
    torch = torch_dev
    from paper_0908_3861_amd import binding
    lim = binding.filter1d_max_scale(n, n1)
    assert lim > 50.0
    rng = np.random.default_rng(2195 + n)
    count, L = 2, 1300
    sig = synth.unit_grid_image(rng, count, L, np.float64)
    sc = rng.uniform(0.75 * lim, lim, size=(count, L)).astype(np.float32)
    sc[0, :3] = np.float32(lim)
    s = run(torch, sig, sc, n, n1, "clamp", a_max=lim)
    pr = np.random.default_rng(8)
    pts = [(0, 0), (0, 1), (1, L - 1), (1, 255), (1, 256)]
    pts += [(int(b), int(m)) for b, m in zip(pr.integers(0, count, 30), pr.integers(0, L, 30))]
    o = F.filter1d_batch(sig, sc, n, n1, "clamp", pts)
    assert rel_max(np.array([s[b, m] for b, m in pts]), o) < TOL


def test_prefiltered_full_size_sampled(torch_dev):
    """The 1024 x 65536 workload shape with the cubic model, on sampled outputs."""
    torch = torch_dev
    rng = np.random.default_rng(synth.CONFIGS["signal1d"]["seed"])
    count, L = 1024, 65536
    sig = synth.unit_grid_image(rng, count, L, np.float32)
    sc = synth.smooth_scales_1d(rng, count, L, 1.0, 16.0)
    s = run(torch, sig, sc, 3, 3, a_max=16.0)
    pr = np.random.default_rng(9)
    pts = [(int(b), int(m)) for b, m in zip(pr.integers(0, count, 300), pr.integers(0, L, 300))]
    pts += [(0, 0), (count - 1, L - 1), (5, 255), (5, 256), (7, L - 257)]
    o = F.filter1d_batch(sig, sc, 3, 3, "clamp", pts)
    err = rel_max(np.array([s[b, m] for b, m in pts]), o)
    print(f"cubic model, full size: rel_max {err:.2e} on {len(pts)} samples")
    assert err < TOL
