"""GPU parity of the mesh's integer-scale form.  When a1 and a3 are integers the (n+1)^2
taps (k1, k3) of each pair (k2, k4) share their cell -- their anchors differ by (k1 a1, k3 a3),
their offset and quarter turn agree -- and a tile whose pixels all qualify interpolates the
window combined with the finite-difference weights along r1 and r3 once per pair.  The sum is
the same (eq. final_eqn regrouped), so the bars are the float64 path's 1e-12 and the float32
path's 1e-5 against the oracle; the diagonal scales a2, a4 stay real.  Also checked: tiles that
mix integer and real a1 (they take the per-tap form), float64 windows of integer running sums
(the combined values in wrapping int64), the split evaluation and its fallback, tier 2, and
batched calls equal to single calls bitwise.
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


def rel_max(s, o):
    return float(np.abs(s - o).max() / np.abs(o).max())


def run(bsf, torch, img, sc, n, path="f64", border="clamp", a_max=None):
    ti = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    ts = torch.from_numpy(np.ascontiguousarray(sc)).cuda()
    out = bsf.filter(ti, ts, n, path=path, border=border, a_max=a_max)
    st = bsf.default_context().device_error()
    return out.cpu().numpy().astype(np.float64), st


def lattice_scales(rng, H, W, lo, hi):
    """a1, a3 integers in lo..hi, a2, a4 real in [lo, hi]."""
    sc = synth.uniform_scales(rng, H, W, float(lo), float(hi))
    sc[..., 0] = rng.integers(lo, hi + 1, size=(H, W))
    sc[..., 2] = rng.integers(lo, hi + 1, size=(H, W))
    return sc


@pytest.mark.parametrize("n,path,border,dtype,H,W,hi", [
    (1, "f64", "clamp", np.float64, 37, 41, 8),
    (1, "f32tiled", "zero", np.float32, 37, 41, 8),
    (2, "f64", "clamp", np.uint8, 37, 41, 6),
    (2, "f64", "zero", np.float64, 35, 33, 6),
    (2, "f32tiled", "clamp", np.float32, 37, 41, 6),
    (2, "f32tiled", "zero", np.float32, 35, 33, 6),
    (3, "f64", "clamp", np.float64, 19, 21, 3),
    (3, "f64", "zero", np.uint8, 19, 21, 3),
    (3, "f32tiled", "clamp", np.float32, 19, 21, 3),
])
def test_integer_a1_a3_every_pixel(bsf, torch_dev, oracle_mod, n, path, border, dtype, H, W, hi):
    rng = np.random.default_rng(400 + 10 * n + (path == "f32tiled") + 2 * (border == "zero"))
    img = (rng.integers(0, 256, size=(H, W)).astype(np.uint8) if dtype == np.uint8
           else synth.unit_grid_image(rng, H, W, dtype))
    sc = lattice_scales(rng, H, W, 1, hi)
    s, st = run(bsf, torch_dev, img, sc, n, path, border)
    assert st == 0
    o = oracle_mod.filter(img.astype(np.float64), sc, n, border)
    err = rel_max(s, o)
    print(f"integer a1, a3: order {n} {path} {border} {np.dtype(dtype).name}: rel_max {err:.3g}")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err


@pytest.mark.parametrize("n,path", [(2, "f64"), (2, "f32tiled"), (1, "f64")])
def test_tiles_mixing_integer_and_real_a1(bsf, torch_dev, oracle_mod, n, path):
    """Integer a1 on the left, real from column 22 on: the first column of tiles qualifies,
    the second (where both meet) and the third do not."""
    rng = np.random.default_rng(420 + n + (path == "f32tiled"))
    H, W = 34, 45
    img = synth.unit_grid_image(rng, H, W, np.float64)
    sc = lattice_scales(rng, H, W, 1, 5)
    sc[:, 22:, 0] += rng.uniform(0.05, 0.95, size=(H, W - 22)).astype(np.float32)
    s, st = run(bsf, torch_dev, img, sc, n, path)
    assert st == 0
    o = oracle_mod.filter(img, sc, n)
    err = rel_max(s, o)
    print(f"mixed tiles: order {n} {path}: rel_max {err:.3g}")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err


def test_integer_running_sums_combined_in_int64(bsf, torch_dev, oracle_mod):
    """Float inputs of wide range: the windows hold integer running sums above the exact
    float64 range, so the combined values are formed in wrapping int64 (or, past 2^(62-2n),
    the per-tap form takes over); every pixel within the float64 tolerance."""
    rng = np.random.default_rng(430)
    H, W = 26, 31
    sc = lattice_scales(rng, H, W, 1, 5)
    for img in (rng.standard_normal((H, W)) * 1e3 + 17.0,
                rng.random((H, W)) - 0.5,
                np.exp(rng.uniform(-20, 20, size=(H, W)))):
        for n in (1, 2):
            s, st = run(bsf, torch_dev, img, sc, n)
            assert st == 0
            o = oracle_mod.filter(img, sc, n)
            assert rel_max(s, o) < TOL_F64, (n, rel_max(s, o))


@pytest.mark.parametrize("n", [2, 3])
def test_split_evaluation_of_combined_taps(bsf, torch_dev, oracle_mod, n):
    """Integer scales large enough that every wave tries the split evaluation of the combined
    polynomials: a blurred image (the bound holds) beside a +-100 checkerboard (it fails and
    the pixels are evaluated again, compensated)."""
    rng = np.random.default_rng(440 + n)
    H, W, cut = 37, 75, 40
    img = synth.blurred_u8_image(rng, H, W, 3.0).astype(np.float64)
    yy, xx = np.mgrid[0:H, cut:W]
    img[:, cut:] = 100.0 * (1 - 2 * ((xx + yy) & 1))
    lo, hi = (6, 8) if n == 2 else (5, 6)
    sc = rng.integers(lo, hi + 1, size=(H, W, 4)).astype(np.float32)
    ctx = bsf.default_context()
    ctx.counters(reset=True)
    s, st = run(bsf, torch_dev, img, sc, n, a_max=float(hi))
    assert st == 0
    tried, redo = ctx.counters(reset=True)
    print(f"n={n}: {tried} of {H * W} pixels split, {redo} evaluated again")
    assert tried > 0 and 0 < redo < tried
    pix = np.arange(H * W) if n == 2 else rng.choice(H * W, 120, replace=False)
    o = oracle_mod.filter(img, sc, n, pixels=pix)
    assert rel_max(s.reshape(-1)[pix], o) < TOL_F64, rel_max(s.reshape(-1)[pix], o)


@pytest.mark.parametrize("path", ["f64", "f32tiled"])
def test_order3_tier2_windows(bsf, torch_dev, oracle_mod, path):
    """Order 3 at integer scales up to 8: windows beyond half the LDS (tier 2)."""
    rng = np.random.default_rng(450 + (path == "f32tiled"))
    H, W = 40, 36
    img = synth.unit_grid_image(rng, H, W, np.float32)
    sc = synth.integer_scales(rng, H, W, 1, 8)
    s, st = run(bsf, torch_dev, img, sc, 3, path, a_max=8.0)
    assert st == 0
    pix = rng.choice(H * W, 60, replace=False)
    o = oracle_mod.filter(img.astype(np.float64), sc, 3, pixels=pix)
    err = rel_max(s.reshape(-1)[pix], o)
    print(f"order 3 tier 2, integer scales, {path}: rel_max {err:.3g}")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err


def test_batched_equals_single_with_integer_scales(bsf, torch_dev):
    """Batched calls take the combined-tap form for exactly the tiles single calls do."""
    torch = torch_dev
    rng = np.random.default_rng(460)
    items, singles = [], []
    for (H, W, n, path) in [(40, 33, 1, "f64"), (37, 50, 2, "f64"), (30, 30, 3, "f32tiled"), (45, 29, 2, "f32tiled")]:
        img = torch.from_numpy(synth.unit_grid_image(rng, H, W, np.float32)).cuda()
        scn = synth.integer_scales(rng, H, W, 1, 6)
        scn[20:, 20:, 0] += 0.5  # tiles of real a1 beside integer ones
        sc = torch.from_numpy(scn).cuda()
        items.append(dict(img=img, scales=sc, order=n, path=path, a_max=6.0))
        singles.append(bsf.filter(img, sc, n, path=path, a_max=6.0).cpu().numpy())
    outs = bsf.filter_batched(items)
    assert bsf.default_context().device_error() == 0
    for o, s1 in zip(outs, singles):
        assert np.array_equal(o.cpu().numpy().view(np.uint8), s1.view(np.uint8))


@pytest.mark.parametrize("path", ["f64", "f32tiled"])
def test_scattered_integer_tiles_in_a_large_image(bsf, torch_dev, oracle_mod, path):
    """4,096 tiles, of which a random fifth have integer a1, a3 throughout and another fifth only
    in their first pixel: the per-tap tier-1 kernel leaves exactly the former to the integer-scale
    kernel, whose persistent workgroups take several tiles each and check every candidate in full.
    Every pixel is written once: the output equals the batched form's bitwise (one kernel there
    decides per tile), and sampled pixels of both kinds of tile match the oracle."""
    torch = torch_dev
    rng = np.random.default_rng(470 + (path == "f32tiled"))
    H = W = 1024
    img = synth.unit_grid_image(rng, H, W, np.float32)
    sc = synth.uniform_scales(rng, H, W, 1.0, 4.0)
    kind = rng.integers(0, 5, size=(H // 16, W // 16))  # 0: integer tile, 1: integer first pixel
    for ty, tx in zip(*np.nonzero(kind == 0)):
        blk = sc[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16]
        blk[..., 0] = np.round(blk[..., 0])
        blk[..., 2] = np.round(blk[..., 2])
    for ty, tx in zip(*np.nonzero(kind == 1)):
        sc[ty * 16, tx * 16, 0] = np.round(sc[ty * 16, tx * 16, 0])
        sc[ty * 16, tx * 16, 2] = np.round(sc[ty * 16, tx * 16, 2])
    ti, ts = torch.from_numpy(img).cuda(), torch.from_numpy(sc).cuda()
    s = bsf.filter(ti, ts, 2, path=path, a_max=4.0)
    assert bsf.default_context().device_error() == 0
    b = bsf.filter_batched([dict(img=ti, scales=ts, order=2, path=path, a_max=4.0)])[0]
    s, b = s.cpu().numpy(), b.cpu().numpy()
    assert np.isfinite(s).all()
    assert np.array_equal(s.view(np.uint8), b.view(np.uint8))
    tiles = np.concatenate([rng.choice(np.flatnonzero(kind.reshape(-1) == k), 6, replace=False) for k in (0, 1, 2)])
    pix = np.array([(t // (W // 16)) * 16 * W + (t % (W // 16)) * 16 + int(rng.integers(0, 16)) * W + int(rng.integers(0, 16))
                    for t in tiles])
    o = oracle_mod.filter(img.astype(np.float64), sc, 2, pixels=pix)
    err = rel_max(s.reshape(-1)[pix], o)
    print(f"scattered integer tiles, {path}: rel_max {err:.3g} over {pix.size} pixels")
    assert err < (TOL_F64 if path == "f64" else TOL_F32), err
