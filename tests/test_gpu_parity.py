"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Error measure (the paper fixes none): rel_max = max|s - O| / max|O| over the compared
pixels.  The float64 path must stay within 1e-12 of the oracle; the oracle itself sums
only non-negative terms in float64, so its own error is a few ulps.
"""
import math

import numpy as np
import pytest

from paper_0908_3861_amd import synth

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12


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


def rel_max(s, o):
    return float(np.abs(s - o).max() / np.abs(o).max())


def run(bsf, torch, img, sc, n, path="f64", border="clamp", a_max=None):
    ti = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    ts = torch.from_numpy(np.ascontiguousarray(sc)).cuda()
    out = bsf.filter(ti, ts, n, path=path, border=border, a_max=a_max)
    ctx = bsf.default_context()
    st = ctx.device_error()
    return out.cpu().numpy(), st


def test_stage1_tile_window_bit_exact(bsf, torch_dev, oracle_mod):
    """The on-chip pre-integrator equals the paper's recursions on the same window."""
    torch = torch_dev
    rng = np.random.default_rng(101)
    H, W = 45, 38
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    for n in (1, 2):
        sc = synth.uniform_scales(rng, H, W, 1.0, 4.0)
        ti = torch.from_numpy(img).cuda()
        ts = torch.from_numpy(sc).cuda()
        ntiles = math.ceil(W / 16) * math.ceil(H / 16)
        for tile in (0, ntiles - 1, 4):
            win, (x0, y0, wq, hq), ovf = bsf.debug_tile_window(ti, ts, n, tile, centred=False)
            assert not ovf
            ys = np.clip(np.arange(y0, y0 + hq), 0, H - 1)
            xs = np.clip(np.arange(x0, x0 + wq), 0, W - 1)
            fwin = img[np.ix_(ys, xs)].astype(np.int64)
            ref = oracle_mod.preintegrate(fwin, n)
            assert np.array_equal(win, ref), (n, tile)


def test_global_preintegrate_bit_exact(bsf, torch_dev, oracle_mod):
    torch = torch_dev
    rng = np.random.default_rng(102)
    H, W = 30, 41
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    ti = torch.from_numpy(img).cuda()
    for n, (x0, y0, wq, hq) in [(1, (-5, -3, 50, 37)), (2, (3, 2, 20, 25)), (3, (-2, -4, 17, 15))]:
        g = bsf.preintegrate(ti, n, x0, y0, wq, hq).cpu().numpy()
        ys = np.clip(np.arange(y0, y0 + hq), 0, H - 1)
        xs = np.clip(np.arange(x0, x0 + wq), 0, W - 1)
        ref = oracle_mod.preintegrate(img[np.ix_(ys, xs)].astype(np.int64), n)
        assert np.array_equal(g, ref), n


@pytest.mark.parametrize("n,x0,y0,wq,hq,dtype", [
    (1, -7, -3, 1300, 20, np.uint8),     # rows longer than one 1024-element chunk
    (2, -3, -9, 37, 260, np.float32),    # tall window, float samples on the 2^-24 grid
    (3, 5, 1, 150, 140, np.uint8),       # values beyond int64: compared modulo 2^64
    (2, -42, -42, 700, 700, np.uint8),
    (1, 0, 0, 1, 1, np.uint8),
])
def test_global_preintegrate_large_windows(bsf, torch_dev, oracle_mod, n, x0, y0, wq, hq, dtype):
    torch = torch_dev
    rng = np.random.default_rng(103 + n)
    H, W = 600, 610
    if dtype == np.uint8:
        img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
        scale = 1
    else:
        img = (rng.integers(0, 1 << 24, size=(H, W)) / float(1 << 24)).astype(np.float32)
        scale = 1 << 24
    g = bsf.preintegrate(torch.from_numpy(img).cuda(), n, x0, y0, wq, hq).cpu().numpy()
    ys = np.clip(np.arange(y0, y0 + hq), 0, H - 1)
    xs = np.clip(np.arange(x0, x0 + wq), 0, W - 1)
    win = np.rint(img[np.ix_(ys, xs)].astype(np.float64) * scale).astype(np.int64)
    ref = oracle_mod.preintegrate(win, n, wrap=True)
    assert np.array_equal(g, ref), (n, x0, y0, wq, hq)


def test_global_preintegrate_on_two_streams(bsf, torch_dev, oracle_mod):
    """Calls in flight on different streams each get their own workspace."""
    torch = torch_dev
    rng = np.random.default_rng(106)
    H, W = 300, 280
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    ti = torch.from_numpy(img).cuda()
    ctx = bsf.default_context()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    wins = [(2, -20, -10, 320, 310, s1), (3, 5, 7, 150, 260, s2), (1, 0, 0, 280, 300, s1), (2, -3, -3, 90, 40, s2)]
    outs = []
    for n, x0, y0, wq, hq, st in wins:
        outs.append(bsf.preintegrate(ti, n, x0, y0, wq, hq, ctx=ctx, stream=st))
    torch.cuda.synchronize()
    for (n, x0, y0, wq, hq, _), g in zip(wins, outs):
        ys = np.clip(np.arange(y0, y0 + hq), 0, H - 1)
        xs = np.clip(np.arange(x0, x0 + wq), 0, W - 1)
        ref = oracle_mod.preintegrate(img[np.ix_(ys, xs)].astype(np.int64), n, wrap=True)
        assert np.array_equal(g.cpu().numpy(), ref), (n, wq, hq)


def test_global_preintegrate_plain_workload_full_size(bsf, torch_dev, oracle_mod):
    """The paper's global stage 1 over the whole padded box of the 2048x2048 order-2 workload."""
    torch = torch_dev
    job = synth.config_job("plain")
    x0 = y0 = -42
    wq = hq = job.image.shape[0] + 84
    g = bsf.preintegrate(torch.from_numpy(job.image).cuda(), 2, x0, y0, wq, hq).cpu().numpy()
    H, W = job.image.shape
    ys = np.clip(np.arange(y0, y0 + hq), 0, H - 1)
    xs = np.clip(np.arange(x0, x0 + wq), 0, W - 1)
    ref = oracle_mod.preintegrate(job.image[np.ix_(ys, xs)].astype(np.int64), 2, wrap=True)
    assert np.array_equal(g, ref)


def test_parity_order1_integer_scales_f64(bsf, torch_dev, oracle_mod):
    rng = np.random.default_rng(103)
    H, W = 50, 67  # several tiles and ragged edges
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = synth.integer_scales(rng, H, W, 1, 8)
    s, st = run(bsf, torch_dev, img, sc, 1)
    assert st == 0
    o = oracle_mod.filter(img, sc, 1)
    assert rel_max(s, o) < TOL_F64


def test_parity_order2_smooth_real_scales_f64(bsf, torch_dev, oracle_mod):
    rng = np.random.default_rng(104)
    H, W = 40, 53
    img = synth.blurred_u8_image(rng, H, W, 3.0)
    sc = synth.smooth_scales(rng, H, W, 1.0, 8.0, 8.0)
    s, st = run(bsf, torch_dev, img, sc, 2)
    assert st == 0
    o = oracle_mod.filter(img.astype(np.float64), sc, 2)
    assert rel_max(s, o) < TOL_F64


def test_parity_order2_iid_real_scales_f64(bsf, torch_dev, oracle_mod):
    rng = np.random.default_rng(105)
    H, W = 33, 35
    img = synth.unit_grid_image(rng, H, W, np.float32)
    sc = synth.uniform_scales(rng, H, W, 1.0, 6.0)
    s, st = run(bsf, torch_dev, img, sc, 2)
    assert st == 0
    o = oracle_mod.filter(img.astype(np.float64), sc, 2)
    assert rel_max(s, o) < TOL_F64


def test_parity_small_config_full(bsf, torch_dev, oracle_mod):
    job = synth.config_job("small")
    s, st = run(bsf, torch_dev, job.image, job.scales, job.order, a_max=8.0)
    assert st == 0
    o = oracle_mod.filter(job.image, job.scales, job.order)
    assert rel_max(s, o) < TOL_F64


def test_zero_border_and_tiny_images(bsf, torch_dev, oracle_mod):
    rng = np.random.default_rng(106)
    for (H, W) in [(1, 1), (1, 9), (7, 1), (17, 16), (16, 17)]:
        img = synth.unit_grid_image(rng, H, W, np.float64)
        sc = synth.uniform_scales(rng, H, W, 1.0, 3.0)
        for n in (1, 2):
            for border in ("clamp", "zero"):
                s, st = run(bsf, torch_dev, img, sc, n, border=border)
                assert st == 0
                o = oracle_mod.filter(img, sc, n, border)
                assert np.abs(s - o).max() <= TOL_F64 * max(np.abs(o).max(), 1e-300), (H, W, n, border)


def test_constant_image_is_reproduced(bsf, torch_dev):
    rng = np.random.default_rng(107)
    H, W = 37, 29
    sc = synth.integer_scales(rng, H, W, 1, 6)
    sc[..., 1] = rng.uniform(1, 6, size=(H, W))  # real diagonal scales keep the DC gain exact
    img = np.full((H, W), 200, np.uint8)
    for n in (1, 2):
        s, st = run(bsf, torch_dev, img, sc, n)
        assert st == 0
        assert np.abs(s - 200.0).max() < 200.0 * TOL_F64


def test_invalid_scales_flag_and_nan(bsf, torch_dev):
    rng = np.random.default_rng(108)
    H, W = 20, 20
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = synth.uniform_scales(rng, H, W, 1.0, 2.0)
    sc[3, 4, 2] = 0.1
    sc[10, 11, 0] = np.nan
    s, st = run(bsf, torch_dev, img, sc, 1, a_max=2.0)
    assert st == 5  # BSF_ERR_SCALE_RANGE
    assert np.isnan(s[3, 4]) and np.isnan(s[10, 11])
    assert np.isfinite(s).sum() == H * W - 2


def test_invalid_arguments(bsf, torch_dev):
    import ctypes
    torch = torch_dev
    ctx = bsf.default_context()
    img = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    sc = torch.ones((8, 8, 4), dtype=torch.float32, device="cuda")
    j, out = bsf.make_job(img, sc, 1)
    j.order = 4
    assert ctx.lib.bsf_filter(ctx.handle, ctypes.byref(j), None) == 4
    j.order = 1
    j.width = 0
    assert ctx.lib.bsf_filter(ctx.handle, ctypes.byref(j), None) == 1
    j.width = 8
    j.out_pitch = 3
    assert ctx.lib.bsf_filter(ctx.handle, ctypes.byref(j), None) == 1
    j.out_pitch = 8
    j.a_max = 1e9
    assert ctx.lib.bsf_filter(ctx.handle, ctypes.byref(j), None) == 1
    j.a_max = 0.3  # neither 0 (chip-sized windows) nor an admissible bound
    assert ctx.lib.bsf_filter(ctx.handle, ctypes.byref(j), None) == 1
    j.a_max = float("nan")
    assert ctx.lib.bsf_filter(ctx.handle, ctypes.byref(j), None) == 1


F32_TOL = 1e-5  # the float32-output path's stated bound (rel_max against the oracle)


@pytest.mark.parametrize("n,lo,hi,seed", [(1, 1, 8, 109), (2, 1, 8, 110), (3, 1, 8, 111), (2, 1, 32, 112),
                                          (1, 0.5, 1.5, 113), (2, 0.5, 1.5, 114), (3, 0.5, 1.5, 115)])
def test_f32_path_error_is_stated(bsf, torch_dev, oracle_mod, n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    H, W = 40, 37
    img = synth.unit_grid_image(rng, H, W, np.float32)
    sc = synth.uniform_scales(rng, H, W, lo, hi)
    s, st = run(bsf, torch_dev, img, sc, n, path="f32tiled")
    assert st == 0 and s.dtype == np.float32
    o = oracle_mod.filter(img.astype(np.float64), sc, n)
    err = rel_max(s.astype(np.float64), o)
    print(f"f32tiled n={n} scales [{lo},{hi}] rel_max {err:.3g}")
    assert err < F32_TOL, err


@pytest.mark.parametrize("n,lo,hi", [(1, 0.5, 1.5), (2, 0.5, 1.5), (3, 0.5, 1.2)])
def test_parity_smallest_scales(bsf, torch_dev, oracle_mod, n, lo, hi):
    """Scales near the admissible minimum: the mesh cancels the most here (the output is
    a small difference of large interpolated running sums)."""
    rng = np.random.default_rng(120 + n)
    H, W = 23, 26
    sc = synth.uniform_scales(rng, H, W, lo, hi)
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    s, st = run(bsf, torch_dev, img, sc, n)
    assert st == 0
    o = oracle_mod.filter(img.astype(np.float64), sc, n)
    assert rel_max(s, o) < TOL_F64, (n, rel_max(s, o))


@pytest.mark.parametrize("n", [2, 3])
def test_split_evaluation_and_its_fallback(bsf, torch_dev, oracle_mod, n):
    """Tiles whose samples need one digit evaluate each tap's terms of total degree above 2
    (order 2) or 3 (order 3) in plain float64 under a rigorous bound on their rounding error; a pixel whose bound
    exceeds 2^-44 of its value is evaluated again, compensated.  The scales are large
    everywhere (every wave tries the split); the left part of the image is a blurred
    positive image (the bound holds), the right part a +-100 checkerboard, which the
    filter all but cancels while its high differences are the largest possible (the
    relative bound fails there).  Both branches run, and every pixel stays within the
    float64 tolerance."""
    torch = torch_dev
    rng = np.random.default_rng(130 + n)
    H, W, cut = 37, 75, 40
    img = synth.blurred_u8_image(rng, H, W, 3.0).astype(np.float64)
    yy, xx = np.mgrid[0:H, cut:W]
    img[:, cut:] = 100.0 * (1 - 2 * ((xx + yy) & 1))
    sc = synth.smooth_scales(rng, H, W, 5.5, 8.0, 8.0) if n == 2 else synth.smooth_scales(rng, H, W, 5.0, 6.5, 8.0)
    ctx = bsf.default_context()
    ctx.counters(reset=True)
    s, st = run(bsf, torch, img, sc, n)
    assert st == 0
    tried, redo = ctx.counters(reset=True)
    print(f"n={n}: {tried} of {H * W} pixels split, {redo} evaluated again")
    assert tried > 0 and 0 < redo < tried
    o = oracle_mod.filter(img, sc, n)
    assert rel_max(s, o) < TOL_F64, rel_max(s, o)
    assert rel_max(s[:, :cut], o[:, :cut]) < TOL_F64


def test_parity_order3_u8_and_float(bsf, torch_dev, oracle_mod):
    rng = np.random.default_rng(110)
    H, W = 19, 21
    sc = synth.uniform_scales(rng, H, W, 1.0, 2.5)
    img8 = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    s, st = run(bsf, torch_dev, img8, sc, 3)
    assert st == 0
    o = oracle_mod.filter(img8.astype(np.float64), sc, 3)
    assert rel_max(s, o) < TOL_F64
    # float input on the 2^-24 grid: the running sums need two digits at order 3
    imgf = synth.unit_grid_image(rng, H, W, np.float64)
    s, st = run(bsf, torch_dev, imgf, sc, 3)
    assert st == 0
    o = oracle_mod.filter(imgf, sc, 3)
    assert rel_max(s, o) < TOL_F64


def test_arbitrary_float_inputs(bsf, torch_dev, oracle_mod):
    """Inputs off any short grid (full 53-bit mantissas), negative and large values."""
    rng = np.random.default_rng(111)
    H, W = 26, 31
    sc = synth.uniform_scales(rng, H, W, 1.0, 5.0)
    for img in (rng.standard_normal((H, W)) * 1e3 + 17.0,
                rng.random((H, W)) - 0.5,
                np.exp(rng.uniform(-20, 20, size=(H, W)))):
        for n in (1, 2):
            s, st = run(bsf, torch_dev, img, sc, n)
            assert st == 0
            o = oracle_mod.filter(img, sc, n)
            assert rel_max(s, o) < TOL_F64, n
    s, st = run(bsf, torch_dev, img.astype(np.float32), sc, 2)
    assert st == 0
    o = oracle_mod.filter(img.astype(np.float32).astype(np.float64), sc, 2)
    assert rel_max(s, o) < TOL_F64


def test_large_windows_need_digits(bsf, torch_dev, oracle_mod):
    """Scales up to 14 at order 2 with float input: windows past 100 px, two digits."""
    rng = np.random.default_rng(112)
    H, W = 24, 24
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = synth.uniform_scales(rng, H, W, 1.0, 14.0)
    s, st = run(bsf, torch_dev, img, sc, 2, a_max=14.0)
    assert st == 0
    pix = rng.choice(H * W, size=40, replace=False)
    o = oracle_mod.filter(img, sc, 2, pixels=pix)
    assert rel_max(s.reshape(-1)[pix], o) < TOL_F64


def test_batched_bitwise_equals_single(bsf, torch_dev):
    """One persistent launch over a mixed batch writes exactly what single calls write."""
    torch = torch_dev
    rng = np.random.default_rng(113)
    specs = [(37, 50, 1, "f64", np.float64), (64, 48, 2, "f32tiled", np.float32), (23, 17, 3, "f64", np.uint8),
             (80, 96, 2, "f64", np.uint8), (16, 16, 1, "f32tiled", np.float64), (45, 31, 3, "f32tiled", np.float32)]
    items, singles = [], []
    for (H, W, n, path, dt) in specs:
        img = (rng.integers(0, 256, size=(H, W)).astype(np.uint8) if dt == np.uint8
               else synth.unit_grid_image(rng, H, W, dt))
        sc = synth.uniform_scales(rng, H, W, 1.0, 3.0 if n == 3 else 7.0)
        ti, ts = torch.from_numpy(img).cuda(), torch.from_numpy(sc).cuda()
        items.append(dict(img=ti, scales=ts, order=n, path=path, a_max=0.0))
        singles.append(bsf.filter(ti, ts, n, path=path, a_max=0.0).cpu().numpy())
    outs = bsf.filter_batched(items)
    assert bsf.default_context().device_error() == 0
    for o, s1 in zip(outs, singles):
        o = o.cpu().numpy()
        assert o.dtype == s1.dtype and np.array_equal(o.view(np.uint8), s1.view(np.uint8))


def test_tier2_tiles_match_oracle(bsf, torch_dev, oracle_mod):
    """Large reach: windows exceed the first launch's LDS share and go to the second."""
    rng = np.random.default_rng(114)
    H, W = 40, 44
    img = synth.blurred_u8_image(rng, H, W, 2.0)
    sc = synth.uniform_scales(rng, H, W, 1.0, 3.0)
    sc[:16, :16] = rng.uniform(10.0, 16.0, size=(16, 16, 4)).astype(np.float32)  # one tile with a big window
    s, st = run(bsf, torch_dev, img, sc, 2, a_max=0.0)
    assert st == 0
    pix = np.concatenate([rng.choice(H * W, 40, replace=False), np.arange(0, 16 * W, W + 1)[:10]])
    o = oracle_mod.filter(img.astype(np.float64), sc, 2, pixels=pix)
    assert rel_max(s.reshape(-1)[pix], o) < TOL_F64


def test_scratch_tier_for_windows_beyond_lds(bsf, torch_dev, oracle_mod):
    """Reach ~60 px: windows past the chip's LDS run in global scratch (third tier)."""
    rng = np.random.default_rng(115)
    H, W = 36, 40
    img = synth.unit_grid_image(rng, H, W, np.float32)
    sc = synth.uniform_scales(rng, H, W, 1.0, 4.0)
    sc[16:32, 16:32] = rng.uniform(18.0, 24.0, size=(16, 16, 4)).astype(np.float32)
    for path, tol in (("f64", TOL_F64), ("f32tiled", F32_TOL)):
        s, st = run(bsf, torch_dev, img, sc, 2, path=path, a_max=24.0)
        assert st == 0
        pix = np.concatenate([rng.choice(H * W, 20, replace=False), (np.arange(16, 32) * W + 20)])
        o = oracle_mod.filter(img.astype(np.float64), sc, 2, pixels=pix)
        err = rel_max(s.reshape(-1)[pix].astype(np.float64), o)
        print(f"tier 3, {path}: rel_max {err:.3g}")
        assert np.isfinite(s).all()
        assert err < tol, (path, err)


@pytest.mark.parametrize("n,path", [(1, "f32tiled"), (2, "f32tiled"), (3, "f32tiled"), (3, "f64")])
def test_zero_border_other_paths(bsf, torch_dev, oracle_mod, n, path):
    """The zero border rule on the float32-output path at every order, and at order 3 on the
    float64 path, on tiny, one-tile and ragged images (every pixel against the oracle)."""
    rng = np.random.default_rng(140 + 10 * n + len(path))
    tol = TOL_F64 if path == "f64" else F32_TOL
    for (H, W) in [(1, 1), (1, 9), (7, 1), (17, 16), (16, 17), (33, 20)]:
        img = synth.unit_grid_image(rng, H, W, np.float64)
        sc = synth.uniform_scales(rng, H, W, 1.0, 3.0 if n < 3 else 2.0)
        for border in ("zero", "clamp"):
            s, st = run(bsf, torch_dev, img, sc, n, path=path, border=border)
            assert st == 0
            o = oracle_mod.filter(img, sc, n, border)
            err = np.abs(s.astype(np.float64) - o).max() / max(np.abs(o).max(), 1e-300)
            assert err <= tol, (H, W, n, path, border, err)


def invert_stage1(g, n):
    """The n-fold lattice differences along l4, l3, l2, l1 -- the recursions of eq. RS undone
    in reverse order -- on a box [hq][wq] (row r = k2, column c = k1), and the mask of the
    points whose every difference found its predecessor inside the box.  int64 arithmetic
    wraps modulo 2^64, which the recursions commute with, so the samples come back exactly
    whenever they fit int64."""
    x = g.copy()
    ok = np.ones(g.shape, bool)
    for dr, dc in [(-1, 1), (-1, 0), (-1, -1), (0, -1)]:  # predecessor of l4, l3, l2, l1
        for _ in range(n):
            y = np.zeros_like(x)
            v = np.zeros_like(ok)
            H, W = x.shape
            r0, c0 = max(0, -dr), max(0, -dc)
            r1, c1 = H - max(0, dr), W - max(0, dc)
            with np.errstate(over="ignore"):
                y[r0:r1, c0:c1] = x[r0:r1, c0:c1] - x[r0 + dr:r1 + dr, c0 + dc:c1 + dc]
            v[r0:r1, c0:c1] = ok[r0:r1, c0:c1] & ok[r0 + dr:r1 + dr, c0 + dc:c1 + dc]
            x, ok = y, v
    return x, ok


@pytest.mark.parametrize("n,path", [(1, "f64"), (2, "f64"), (3, "f64"), (1, "f32tiled"), (2, "f32tiled")])
def test_stage1_anchored_window_inverts(bsf, torch_dev, n, path):
    """The window stage 1 leaves on chip for the filter itself: every running sum anchored at
    the tile centre.  Anchoring changes a line's sums by a polynomial of degree < n along
    that line, which the mesh's n-fold differences along the same direction annihilate; so
    the n-fold lattice differences of the anchored window, taken along l4, l3, l2, l1, must
    give the samples back exactly, wherever the differences stay inside the window.  (The
    float32-output path keeps float64 running sums, exact here: u8 samples and sums below
    2^53.)"""
    torch = torch_dev
    rng = np.random.default_rng(150 + n + 10 * len(path))
    H, W = 45, 38
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    sc = synth.uniform_scales(rng, H, W, 1.0, 4.0 if n < 3 else 2.5)
    ti, ts = torch.from_numpy(img).cuda(), torch.from_numpy(sc).cuda()
    ntiles = math.ceil(W / 16) * math.ceil(H / 16)
    for tile in (0, 4, ntiles - 1):
        win, (x0, y0, wq, hq), _ = bsf.debug_tile_window(ti, ts, n, tile, centred=True, path=path)
        if path == "f32tiled":
            wd = win.view(np.float64)
            assert np.all(np.abs(wd) < 2.0 ** 53) and np.all(wd == np.round(wd))
            win = wd.astype(np.int64)
        ys = np.clip(np.arange(y0, y0 + hq), 0, H - 1)
        xs = np.clip(np.arange(x0, x0 + wq), 0, W - 1)
        fwin = img[np.ix_(ys, xs)].astype(np.int64)
        back, ok = invert_stage1(win, n)
        assert ok.sum() >= (hq - 4 * n) * (wq - 4 * n) // 2, ok.sum()
        assert np.array_equal(back[ok], fwin[ok]), (n, path, tile)
        # and the anchoring is really there: the window differs from the zero-start sums
        plain, _, _ = bsf.debug_tile_window(ti, ts, n, tile, centred=False, path=path)
        if path == "f32tiled":
            plain = plain.view(np.float64).astype(np.int64)
        assert not np.array_equal(plain, win)


@pytest.mark.parametrize("n", [2, 3])
def test_f32_path_worst_case_small_scales_beside_large(bsf, torch_dev, oracle_mod, n):
    """The float32-output path's hardest case for its stated 1e-5: one tile whose left half
    has every scale in [0.5, 1] (the largest mask gain, (2/a)^(4n)) and whose right half has
    scales 24-32, so the restart window -- and with it the float64 running sums the small
    kernels cancel -- is sized for the large ones (tier-3 windows).  Every small-scale pixel
    is compared (all pixels at order 2; 16 large ones at order 3, whose oracle sums are slow)."""
    rng = np.random.default_rng(160 + n)
    H, W = 16, 16
    img = synth.unit_grid_image(rng, H, W, np.float32)
    sc = np.empty((H, W, 4), np.float32)
    sc[:, :8] = rng.uniform(0.5, 1.0, size=(H, 8, 4))
    sc[:, 8:] = rng.uniform(24.0, 32.0, size=(H, 8, 4))
    s, st = run(bsf, torch_dev, img, sc, n, path="f32tiled", a_max=32.0)
    assert st == 0
    small = (np.arange(H)[:, None] * W + np.arange(8)[None, :]).reshape(-1)
    big = (np.arange(H)[:, None] * W + np.arange(8, 16)[None, :]).reshape(-1)
    pix = np.concatenate([small, big if n == 2 else rng.choice(big, 16, replace=False)])
    o = oracle_mod.filter(img.astype(np.float64), sc, n, pixels=pix)
    got = s.reshape(-1)[pix].astype(np.float64)
    err = rel_max(got, o)
    err_small = float(np.abs(got[:len(small)] - o[:len(small)]).max() / np.abs(o[:len(small)]).max())
    print(f"f32tiled worst case n={n}: rel_max {err:.3g}, small-scale pixels alone {err_small:.3g}")
    assert err < F32_TOL and err_small < F32_TOL


def test_workspace_limit(bsf, torch_dev):
    """A context's workspace limit: a call whose work area exceeds it fails with
    BSF_ERR_OUT_OF_MEMORY (tier-3 scratch), one whose area fits runs (tier-2 lists), and a
    limit equal to bsf_workspace_size lets the call run and gives the same output."""
    import ctypes
    torch = torch_dev
    rng = np.random.default_rng(170)
    H, W = 40, 44
    img = torch.from_numpy(synth.unit_grid_image(rng, H, W, np.float64)).cuda()
    scn = synth.uniform_scales(rng, H, W, 1.0, 3.0)
    scn[:16, :16] = rng.uniform(12.0, 13.0, size=(16, 16, 4)).astype(np.float32)
    sc = torch.from_numpy(scn).cuda()
    small = bsf.Context(workspace_limit=4096)
    ref = bsf.filter(img, sc, 2, a_max=13.0)  # tier 2 on the default context
    got = bsf.filter(img, sc, 2, a_max=13.0, ctx=small, check=True)
    assert torch.equal(got, ref)
    with pytest.raises(bsf.BsfError) as ei:
        bsf.filter(img, sc, 2, a_max=40.0, ctx=small)  # tier-3 slices of ~180 KB each
    assert ei.value.status == 2
    lib = bsf.load()
    # a_max bounds every scale of the image (the tile at [0,16)^2 reaches 13)
    for a_max in (13.0, 14.5, 16.0, 17.5, 19.0, 24.0):
        j, _ = bsf.make_job(img, sc, 2, a_max=a_max)
        need = ctypes.c_size_t()
        assert lib.bsf_workspace_size(ctypes.byref(j), ctypes.byref(need)) == 0
        ctx = bsf.Context(workspace_limit=max(need.value, 1))
        out = bsf.filter(img, sc, 2, a_max=a_max, ctx=ctx, check=True)
        assert torch.equal(out, bsf.filter(img, sc, 2, a_max=a_max)), a_max
        ctx.close()
    small.close()
