#!/usr/bin/env python3
"""Throughput of the adaptive box-spline filter on one MI355X.

Default workload ("plain"): one step = one bsf_filter call (the whole hot path: restart
windows, exact pre-integration, localisation mesh) over a 2048x2048 uint8 image
(Gaussian-blurred noise) with smooth real scale fields in [1, 16], order 2, float64
path.  Inputs are resident in HBM before timing starts.  Prints one JSON line with
Mpixel/s, the roofline of the filter call (HIP events on its launch stream) and the CPU
oracle timed on a bounded pixel sample.

The default run also times the float32-output path on the same inputs (its speedup and its
error against the oracle at the same pixels, in extra.f32tiled), reports the cancellation
factor kappa of the sampled pixels (extra.kappa) and runs a short serving stream
(extra.serving: p50/p99 latency, Mpixel/s; the full 60 s form is --workload serving).

Other forms (not run by default): --workload small | precision | batched | serving | stage1 |
ellipse (the scale field of elliptical windows, the step before the filter) | signal1d (the
one-dimensional scale-adaptive filter of Section 3 on a batch of signals) | rect (the
two-direction box spline, Section 4 with N = 2).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_0908_3861_amd import synth  # noqa: E402

METRIC = "Mpixel/s + HBM roofline %, FP64 vs FP32-tiled at stated err; serve p50/p99"
PEAK_FP64_VALU = 78.6e12   # MI355X vector FP64, FLOP/s
PEAK_FP32_VALU = 157.3e12
PEAK_HBM = 8.0e12          # B/s

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (scaled by a 1 GiB device copy), keyed by the kernel source they were taken on: once
# the source changes, the figure no longer applies and the bench reports null.
MEASURED_TRAFFIC = {"1e1dbb754bcea6df": {("plain", "f64"): 148.6e6, ("ellipse", "f32"): 117.5e6,
                                        ("signal1d", "f64"): 1140.7e6, ("signal1d", "f32tiled"): 872.2e6}}
# Fraction of the chip's VALU issue slots the dominant kernel used (rocprofv3 SQ_INSTS_VALU x 4
# cycles over 1024 SIMDs x 2.4 GHz x kernel time), keyed the same way.
MEASURED_VALU_ISSUE = {"1e1dbb754bcea6df": {("plain", "f64"): 0.86, ("signal1d", "f64"): 0.76,
                                           ("signal1d", "f32tiled"): 0.71}}


def kernel_source_key() -> str:
    """sha256 prefix over every source the kernels are compiled from."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0908_3861_amd", "csrc")
    for f in [os.path.join(csrc, "bsf.hip")] + sorted(glob.glob(os.path.join(csrc, "*.h"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def mesh_flops_per_pixel(order: int) -> float:
    """Interpolation-weighted tap MACs: (n+1)^4 taps x 7n^2 lattice weights x 2."""
    return 2.0 * (order + 1) ** 4 * 7 * order ** 2


def algorithmic_flops(pixels: int, order: int, pbox: int) -> float:
    """Tap MACs per pixel plus 4n running-sum adds per element of the padded stage-1 box."""
    return pixels * mesh_flops_per_pixel(order) + pbox * 4.0 * order


def padded_box(h: int, w: int, order: int, a_max: float) -> int:
    R = 0.5 * order * (a_max + 2 * a_max / math.sqrt(2))
    return int((w + 2 * math.ceil(R) + 3 * order) * (h + 2 * math.ceil(R) + 3 * order))


def time_steps(step, steps: int, warmup: int, stream):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))


def oracle_sample(img64, scales, order, pixels_total, cpu_seconds, rng, border="clamp"):
    """Time the CPU oracle on a bounded random pixel sample (about cpu_seconds of work)."""
    import oracle
    probe = rng.choice(pixels_total, size=16, replace=False)
    t0 = time.perf_counter()
    oracle.filter(img64, scales, order, border, pixels=probe)
    tp = max(time.perf_counter() - t0, 1e-3)
    count = int(min(pixels_total, max(32, 16 * cpu_seconds / tp)))
    sample = np.sort(rng.choice(pixels_total, size=count, replace=False))
    t0 = time.perf_counter()
    o = oracle.filter(img64, scales, order, border, pixels=sample)
    return sample, o, time.perf_counter() - t0


def kappa_summary(img, scales, order, sample, o, seconds) -> dict:
    """Percentiles of the cancellation factor kappa(m) = sum|terms| / |s| of the two-stage
    method on per-pixel restart windows, over the first pixels of the oracle's sample that fit
    in about `seconds` (the errors above are of order kappa eps; tile windows see more)."""
    from oracle import kappa as OK
    ks, worst, t0 = [], 0.0, time.perf_counter()
    for p, v in zip(sample, o):
        k, w = OK.kappa(img, scales, order, [p], [v])
        ks.append(float(k[0]))
        worst = max(worst, w)
        if time.perf_counter() - t0 > seconds:
            break
    ks = np.array(ks)
    return {"p50": float(np.percentile(ks, 50)), "p99": float(np.percentile(ks, 99)), "max": float(ks.max()),
            "pixels": int(len(ks)), "window": "per-pixel restart window",
            "two_stage_check": worst}


def threads_used() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


def errors(s, o) -> dict:
    s = np.asarray(s, np.float64)
    return {"rel_max": float(np.abs(s - o).max() / np.abs(o).max()),
            "rel_rms": float(np.sqrt(np.mean((s - o) ** 2)) / np.sqrt(np.mean(o ** 2))),
            "frac_within_1e-5": float(np.mean(np.abs(s - o) <= 1e-5 * np.abs(o).max())),
            "compared": int(len(o))}


def record(value, wall, steps, warmup, dtype, config, roofline, cpu, extra, unit="Mpixel/s"):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": wall / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline, "cpu_baseline": cpu,
            "extra": extra}


# ---------------------------------------------------------------------------------------
def run_single(args, name, job, a_max, path):
    import torch
    from paper_0908_3861_amd import binding
    H, W = job.image.shape
    n = job.order
    dev = torch.device("cuda:0")
    img = torch.from_numpy(job.image).to(dev)
    sc = torch.from_numpy(job.scales).to(dev)
    out = torch.empty((H, W), dtype=torch.float64 if path == "f64" else torch.float32, device=dev)
    ctx = binding.default_context(0)
    stream = torch.cuda.current_stream()

    def step():
        binding.filter(img, sc, n, path=path, a_max=a_max, out=out, ctx=ctx)

    ctx.counters(reset=True)
    wall, ms = time_steps(step, args.steps, args.warmup, stream)
    ctx.check_device()
    tried, redo = ctx.counters(reset=True)
    if args.copy_probe_mib:
        # a plain device copy of known size, for scaling the profiler's byte counters
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    P = H * W
    flops = algorithmic_flops(P, n, padded_box(H, W, n, a_max))
    peak = PEAK_FP64_VALU  # the mesh runs in float64 on both paths
    roof = {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": flops / (ms * 1e-3) / peak, "traffic": None}
    in_bytes = job.image.dtype.itemsize
    alg_bytes = P * (in_bytes + 16 + (8 if path == "f64" else 4))
    extra = {"filter_ms": ms, "hbm_algorithmic_GBps": alg_bytes / (ms * 1e-3) / 1e9,
             "hbm_frac_of_8TBps": alg_bytes / (ms * 1e-3) / PEAK_HBM, "a_max": a_max}
    if path == "f64" and n > 1:
        # pixels whose taps were evaluated split (high-degree terms in plain float64 under
        # an error bound), and the fraction of them evaluated again compensated
        extra["split_eval"] = {"pixels_per_call": tried / max(1, args.steps + args.warmup),
                               "reevaluated_frac": redo / tried if tried else None}
    return out, ms, wall, roof, extra


def stage1_alone(job, halo: int, steps: int, warmup: int) -> dict:
    """The paper's global pre-integrator (bsf_preintegrate) over the image's whole padded box.

    Four passes (rows fused with the sample load; diagonals; columns; anti-diagonals
    writing g), each reading and writing every element of its domain once: the
    algorithmic bytes are Pbox*(in + 8) for the end points plus 48 B per element of the
    extended domain D1 (box + extension triangle) for the three int64 hand-overs."""
    import torch
    from paper_0908_3861_amd import binding
    H, W = job.image.shape
    n = job.order
    wq, hq = W + 2 * halo, H + 2 * halo
    dev = torch.device("cuda:0")
    img = torch.from_numpy(job.image).to(dev)
    g = torch.empty((hq, wq), dtype=torch.int64, device=dev)
    ctx = binding.default_context(0)
    lib = ctx.lib
    j = binding.Job()
    j.width, j.height = W, H
    j.in_dtype = binding._dtype_code(img)
    j.in_ = img.data_ptr()
    j.in_pitch = img.stride(0)
    j.order = n
    stream = torch.cuda.current_stream()

    def step():
        ctx._check(lib.bsf_preintegrate(ctx.handle, binding.ctypes.byref(j), -halo, -halo, wq, hq, g.data_ptr(),
                                        g.stride(0), binding._stream_ptr(stream)))

    wall, ms = time_steps(step, steps, warmup, stream)
    box = wq * hq
    d1 = box + hq * (hq - 1) // 2
    alg = box * (job.image.dtype.itemsize + 8) + 48 * d1
    return {"window": [wq, hq], "order": n, "ms": ms, "algorithmic_bytes": alg,
            "GBps": alg / (ms * 1e-3) / 1e9, "hbm_frac": alg / (ms * 1e-3) / PEAK_HBM,
            "Mpixel_per_s": H * W / (ms * 1e-3) / 1e6}


def workload_plain(args):
    job = synth.config_job("plain", size=(args.size, args.size))
    a_max = 16.0  # the workload's scale fields lie in [1, 16]
    out, ms, wall, roof, extra = run_single(args, "plain", job, a_max, args.path)
    H, W = job.image.shape
    P = H * W
    cpu = None
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(12345)
        sample, o, tc = oracle_sample(job.image.astype(np.float64), job.scales, job.order, P, args.cpu_seconds, rng)
        cpu = {"value": len(sample) / tc / 1e6, "unit": "Mpixel/s", "cores": threads_used(), "kind": "oracle",
               "sample": f"{len(sample)} random pixels of the same {W}x{H} order-{job.order} workload "
                         f"(direct box-spline sum, float64, OpenMP), {tc:.1f} s"}
        extra["err_vs_oracle"] = errors(out.cpu().numpy().reshape(-1)[sample], o)
        extra["kappa"] = kappa_summary(job.image, job.scales, job.order, sample, o, args.kappa_seconds)
    if args.path == "f64" and not args.no_f32_leg:
        # the float32-output path on the same inputs: its speedup and its error at the same pixels
        out32, ms32, wall32, _, _ = run_single(args, "plain", job, a_max, "f32tiled")
        leg = {"filter_ms": ms32, "Mpixel_per_s": P * args.steps / wall32 / 1e6,
               "speedup_over_f64": ms / ms32}
        if cpu is not None:
            leg["err_vs_oracle"] = errors(out32.cpu().numpy().reshape(-1)[sample].astype(np.float64), o)
        extra["f32tiled"] = leg
    # the global (paper's literal) stage 1 alone over the same image, padded by the
    # halo of the largest scale: R = (n/2)(a + 2a/sqrt2) + 3n, about 42 at n = 2, a = 16
    extra["stage1_global_alone"] = stage1_alone(job, 42, max(3, args.steps // 2), 2)
    if args.serving_seconds > 0:
        # a short run of the serving stream (the full form: --workload serving, 60 s)
        sv = serving_stream(args, args.serving_seconds, False)
        for k in ("_pixels", "_wall", "budget_gib", "streams", "pool"):
            sv.pop(k, None)
        extra["serving"] = sv
    if W == 2048 and H == 2048:
        key = kernel_source_key()
        roof["traffic"] = MEASURED_TRAFFIC.get(key, {}).get(("plain", args.path))
        extra["executed_valu_issue_frac"] = MEASURED_VALU_ISSUE.get(key, {}).get(("plain", args.path))
    config = {"workload": f"plain: {W}x{H} uint8 blurred-noise image, smooth real scales in [1,16], "
                          f"order {job.order}, {args.path} path", "pixels": P, "order": job.order, "path": args.path}
    dtype = "f64" if args.path == "f64" else "f64-mesh/f32-out"
    return record(P * args.steps / wall / 1e6, wall, args.steps, args.warmup, dtype, config, roof, cpu, extra)


def workload_small(args):
    job = synth.config_job("small")
    out, ms, wall, roof, extra = run_single(args, "small", job, 8.0, "f64")
    import oracle
    t0 = time.perf_counter()
    o = oracle.filter(job.image, job.scales, job.order)
    tc = time.perf_counter() - t0
    P = job.pixels
    extra["err_vs_oracle"] = errors(out.cpu().numpy().reshape(-1), o.reshape(-1))
    cpu = {"value": P / tc / 1e6, "unit": "Mpixel/s", "cores": threads_used(), "kind": "oracle",
           "sample": f"the full 256x256 image, {tc:.2f} s"}
    config = {"workload": "small: 256x256 f64 unit-grid pixels, integer scales U{1..8}, order 1, f64 path",
              "pixels": P, "order": 1, "path": "f64"}
    return record(P * args.steps / wall / 1e6, wall, args.steps, args.warmup, "f64", config, roof, cpu, extra)


def workload_precision(args):
    side = args.size if args.size != 2048 else 4096
    job = synth.config_job("precision", size=(side, side))
    P = job.pixels
    out32, ms32, wall32, roof, extra = run_single(args, "precision", job, 32.0, "f32tiled")
    out64, ms64, wall64, _, extra64 = run_single(args, "precision", job, 32.0, "f64")
    rng = np.random.default_rng(777)
    sample, o, tc = oracle_sample(job.image.astype(np.float64), job.scales, job.order, P, args.cpu_seconds, rng)
    extra["f64_path_ms"] = ms64
    extra["f32tiled_speedup_over_f64"] = ms64 / ms32
    extra["err_f32tiled_vs_oracle"] = errors(out32.cpu().numpy().reshape(-1)[sample], o)
    extra["err_f64_vs_oracle"] = errors(out64.cpu().numpy().reshape(-1)[sample], o)
    cpu = {"value": len(sample) / tc / 1e6, "unit": "Mpixel/s", "cores": threads_used(), "kind": "oracle",
           "sample": f"{len(sample)} random pixels of the {side}x{side} workload, {tc:.1f} s"}
    config = {"workload": f"precision: {side}x{side} f32 unit-grid pixels, i.i.d. real scales U[1,32], order 2, "
                          "f32tiled path (f64 path timed beside it)", "pixels": P, "order": 2, "path": "f32tiled"}
    return record(P * args.steps / wall32 / 1e6, wall32, args.steps, args.warmup, "f64-mesh/f32-out", config, roof,
                  cpu, extra)


def workload_batched(args):
    import torch
    from paper_0908_3861_amd import binding
    jobs = synth.batch_jobs(count=args.batch_count)
    dev = torch.device("cuda:0")
    items = []
    for j in jobs:
        items.append(dict(img=torch.from_numpy(j.image).to(dev), scales=torch.from_numpy(j.scales).to(dev),
                          order=j.order, path="f32tiled", a_max=8.0))
    for it in items:
        it["out"] = torch.empty(it["img"].shape, dtype=torch.float32, device=dev)
    ctx = binding.default_context(0)
    stream = torch.cuda.current_stream()

    def step():
        binding.filter_batched(items, ctx=ctx)

    wall, ms = time_steps(step, args.steps, args.warmup, stream)
    ctx.check_device()
    P = sum(j.pixels for j in jobs)
    flops = sum(algorithmic_flops(j.pixels, j.order, padded_box(*j.image.shape, j.order, 8.0)) for j in jobs)
    roof = {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / PEAK_FP64_VALU, "traffic": None}
    # each image alone, and the oracle on sampled pixels of a few images
    rng = np.random.default_rng(99)
    equal = True
    for k in rng.choice(len(jobs), size=3, replace=False):
        it = items[k]
        alone = binding.filter(it["img"], it["scales"], it["order"], path="f32tiled", a_max=8.0, ctx=ctx)
        equal &= bool(torch.equal(alone, it["out"]))
    errs = []
    import oracle
    t_or = 0.0
    n_or = 0
    for k in rng.choice(len(jobs), size=4, replace=False):
        j = jobs[k]
        pix = rng.choice(j.pixels, size=16, replace=False)
        t0 = time.perf_counter()
        o = oracle.filter(j.image.astype(np.float64), j.scales, j.order, pixels=pix)
        t_or += time.perf_counter() - t0
        n_or += len(pix)
        errs.append(errors(items[k]["out"].cpu().numpy().reshape(-1)[pix], o)["rel_max"])
    orders = [j.order for j in jobs]
    extra = {"batch_ms": ms, "images": len(jobs), "orders": {str(n): orders.count(n) for n in (1, 2, 3)},
             "batched_equals_alone": equal, "err_rel_max_sampled": max(errs)}
    cpu = {"value": n_or / t_or / 1e6, "unit": "Mpixel/s", "cores": threads_used(), "kind": "oracle",
           "sample": f"{n_or} random pixels of 4 of the images (orders mixed), {t_or:.1f} s"}
    config = {"workload": f"batched: {len(jobs)} images, sides U{{256..2048 step 64}}, f32 unit-grid pixels, "
                          "integer scales U{1..8}, orders U{1,2,3}, one persistent launch", "pixels": P,
              "path": "f32tiled"}
    return record(P * args.steps / wall / 1e6, wall, args.steps, args.warmup, "f64-mesh/f32-out", config, roof, cpu,
                  extra)


def serving_stream(args, duration: float, compare: bool) -> dict:
    """A Poisson stream of requests through the continuous-batching server: square sides
    log-uniform in [128, max_side], f32/f64 50/50, integer scales U{1..8}, orders U{1,2,3};
    the rate is 0.7 x the capacity of a closed-loop probe on the same pool (or --rate)."""
    import torch
    from paper_0908_3861_amd import serve
    rng = np.random.default_rng(5)
    # a pool of requests with the stream's shape/order/dtype mix, in pinned host memory
    pool = []
    for i in range(args.pool):
        s = int(round(math.exp(rng.uniform(math.log(128), math.log(args.max_side)))))
        f64 = bool(rng.integers(0, 2))
        n = int(rng.integers(1, 4))
        img = synth.unit_grid_image(rng, s, s, np.float64 if f64 else np.float32)
        sc = synth.integer_scales(rng, s, s, 1, 8)
        pool.append((torch.from_numpy(img).pin_memory(), torch.from_numpy(sc).pin_memory(), n,
                     "f64" if f64 else "f32tiled"))

    def server(graphs):
        return serve.Server(budget_bytes=args.budget_gib << 30, slots=args.slots, streams=4, a_max=8.0,
                            graphs=graphs, max_group=args.slots)

    # closed-loop capacity probe: every pool request at once
    srv = server(True)
    t0 = time.perf_counter()
    futs = [srv.submit(im, sc, n, path) for (im, sc, n, path) in pool]
    for f in futs:
        f.result()
    probe_s = time.perf_counter() - t0
    capacity = len(pool) / probe_s
    srv.close()
    rate = args.rate if args.rate > 0 else 0.7 * capacity
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * duration * 2) + 10))
    arrivals = arrivals[arrivals < duration]
    picks = rng.integers(0, len(pool), size=len(arrivals))

    def stream_run(graphs):
        srv = server(graphs)
        t_start = time.perf_counter()
        futs = []  # outstanding requests; finished ones are dropped with their pinned results
        for t_a, k in zip(arrivals, picks):
            now = time.perf_counter() - t_start
            if t_a > now:
                time.sleep(t_a - now)
            im, sc, n, path = pool[k]
            futs.append(srv.submit(im, sc, n, path))
            still = []
            for f in futs:
                if f.done():
                    f.result()
                else:
                    still.append(f)
            futs = still
        for f in futs:
            f.result()
        wall = time.perf_counter() - t_start
        srv.close()
        st = srv.stats()
        print(f"serving ({'graph replays' if graphs else 'eager launches'}): {st}", file=sys.stderr, flush=True)
        return st, wall

    st, wall = stream_run(True)
    out = {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"], "requests": st["completed"],
           "failed": st["failed"], "launches": st["launches"], "Mpixel_per_s": st["pixels"] / wall / 1e6,
           "launch_form": "captured batch plans (graph replay)", "arrival_rate_hz": rate,
           "capacity_probe_hz": capacity, "duration_s": duration, "budget_gib": args.budget_gib,
           "slots": args.slots, "streams": 4, "pool": len(pool), "max_side": args.max_side,
           "_pixels": st["pixels"], "_wall": wall}
    if compare:
        st_e, wall_e = stream_run(False)
        out["eager"] = {"p50_ms": st_e["p50_ms"], "p99_ms": st_e["p99_ms"], "mean_ms": st_e["mean_ms"],
                        "Mpixel_per_s": st_e["pixels"] / wall_e / 1e6, "launches": st_e["launches"]}
    return out


def workload_serving(args):
    extra = serving_stream(args, args.duration, args.serving_compare)
    pixels, wall = extra.pop("_pixels"), extra.pop("_wall")
    config = {"workload": "serving: Poisson stream, square sides log-uniform [128, %d], f32/f64 50/50, "
                          "integer scales U{1..8}, orders U{1,2,3}" % args.max_side}
    return record(pixels / wall / 1e6, wall, 1, 0, "f64 / f64-mesh+f32-out (mixed)", config, None, None, extra)


def workload_stage1(args):
    """Stage 1 alone, as the paper's global pre-integrator, on the plain workload's image."""
    job = synth.config_job("plain", size=(args.size, args.size))
    r = stage1_alone(job, 42, args.steps, args.warmup)
    H, W = job.image.shape
    roof = {"bound": "hbm", "achieved": r["GBps"], "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": r["hbm_frac"],
            "traffic": None}
    config = {"workload": f"stage1: global n-fold running sums (4 directions, order {job.order}) over the "
                          f"{r['window'][0]}x{r['window'][1]} padded box of the {W}x{H} uint8 plain image",
              "pixels": H * W, "order": job.order}
    wall = r["ms"] * 1e-3 * args.steps
    return record(r["Mpixel_per_s"], wall, args.steps, args.warmup, "int64", config, roof, None, r)


def time_queued(launch, reps: int, stream) -> float:
    """Device milliseconds per launch of a short kernel: the launches are queued behind a
    spin kernel, so the GPU runs them back to back between the two events (events around
    each launch would time the host's launch overhead too)."""
    import torch
    torch.cuda.synchronize()
    torch.cuda._sleep(50_000_000)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def workload_ellipse(args):
    """The scale field of elliptical windows (bsf_scales_from_ellipses), the step before
    the filter: 12 B read and 16 B written per pixel, bound by HBM."""
    import torch
    from paper_0908_3861_amd import binding
    import oracle.ellipse as OE
    H = W = args.size
    rng = np.random.default_rng(synth.CONFIGS["ellipse"]["seed"])
    ell_np = synth.ellipse_field(rng, H, W)
    dev = torch.device("cuda:0")
    ell = torch.from_numpy(ell_np).to(dev)
    out = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
    ctx = binding.default_context(0)
    stream = torch.cuda.current_stream()

    def step():
        binding.scales_from_ellipses(ell, 2, out=out, ctx=ctx, stream=stream)

    for _ in range(args.warmup):
        step()
    reps = max(args.steps, 1)
    t0 = time.perf_counter()
    ms = time_queued(step, reps, stream)
    wall = time.perf_counter() - t0
    ctx.check_device()
    if args.copy_probe_mib:  # a plain device copy of known size, for scaling the byte counters
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    P = H * W
    alg = P * (12 + 16)
    key = kernel_source_key()
    roof = {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": alg / (ms * 1e-3) / PEAK_HBM, "traffic": MEASURED_TRAFFIC.get(key, {}).get(("ellipse", "f32"))}
    extra = {"kernel_ms": ms, "algorithmic_bytes": alg}
    cpu = None
    if not args.no_cpu_baseline:
        g = out.cpu().numpy().reshape(-1, 4).astype(np.float64)
        pr = np.random.default_rng(12346)
        probe = pr.choice(P, size=16, replace=False)
        t0 = time.perf_counter()
        OE.scales_from_ellipses(ell_np.reshape(-1, 3)[probe], 2)
        tp = max(time.perf_counter() - t0, 1e-3)
        count = int(min(P, max(32, 16 * args.cpu_seconds / tp)))
        pix = np.sort(pr.choice(P, size=count, replace=False))
        t0 = time.perf_counter()
        ref = OE.scales_from_ellipses(ell_np.reshape(-1, 3)[pix], 2)
        tc = time.perf_counter() - t0
        ref32 = ref.astype(np.float32).astype(np.float64)
        extra["err_vs_oracle"] = {"max_ulp32": float(np.max(np.abs(g[pix] - ref32) / (np.abs(ref32) * 2.0 ** -23))),
                                  "compared": int(count)}
        cpu = {"value": count / tc / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
               "sample": f"{count} random pixels of the same {W}x{H} field (brute-force active sets, numpy, "
                         f"one thread), {tc:.1f} s"}
    config = {"workload": f"ellipse: {W}x{H} field of (s_major in [1,8], elongation in [1,4], orientation in "
                          f"[0,pi)), smooth sigma=32 fields -> order-2 scales", "pixels": P, "order": 2}
    extra["wall_s"] = wall
    return record(P / (ms * 1e-3) / 1e6, ms * 1e-3 * reps, reps, args.warmup, "f64-compute/f32-io", config, roof,
                  cpu, extra)


def workload_signal1d(args):
    """The one-dimensional scale-adaptive filter (bsf_filter1d, Section 3): 1024 signals of
    65536 float32 samples, smooth scales in [1, 16], order 3, impulse model.  One step = one
    bsf_filter1d call (running sums on restart windows, interpolant tables, the mask);
    algorithmic HBM bytes per sample: 4 in + 4 scale + 8 out."""
    import torch
    from paper_0908_3861_amd import binding
    import oracle.filter1d as OF
    count, L, order, model = args.signals, args.length, 3, -1
    path = args.path
    ob = 8 if path == "f64" else 4
    rng = np.random.default_rng(synth.CONFIGS["signal1d"]["seed"])
    sig_np = synth.unit_grid_image(rng, count, L, np.float32)
    sc_np = synth.smooth_scales_1d(rng, count, L, 1.0, 16.0)
    dev = torch.device("cuda:0")
    sig = torch.from_numpy(sig_np).to(dev)
    sc = torch.from_numpy(sc_np).to(dev)
    out = torch.empty((count, L), dtype=torch.float64 if path == "f64" else torch.float32, device=dev)
    ctx = binding.default_context(0)
    stream = torch.cuda.current_stream()

    def step():
        binding.filter1d(sig, sc, order, model, "clamp", a_max=16.0, out=out, ctx=ctx, stream=stream, path=path)

    for _ in range(args.warmup):
        step()
    reps = max(args.steps, 1)
    t0 = time.perf_counter()
    ms = time_queued(step, reps, stream)
    wall = time.perf_counter() - t0
    ctx.check_device()
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    N = count * L
    alg = N * (4 + 4 + ob)
    key = kernel_source_key()
    roof = {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": alg / (ms * 1e-3) / PEAK_HBM,
            "traffic": MEASURED_TRAFFIC.get(key, {}).get(("signal1d", path))}
    extra = {"kernel_ms": ms, "algorithmic_bytes": alg,
             "executed_valu_issue_frac": MEASURED_VALU_ISSUE.get(key, {}).get(("signal1d", path))}
    cpu = None
    if not args.no_cpu_baseline:
        s = out.cpu().numpy().astype(np.float64)
        pr = np.random.default_rng(12347)
        probe = [(int(b), int(m)) for b, m in zip(pr.integers(0, count, 64), pr.integers(0, L, 64))]
        t0 = time.perf_counter()
        OF.filter1d_batch(sig_np, sc_np, order, model, "clamp", probe)
        tp = max(time.perf_counter() - t0, 1e-3)
        k = int(min(N, max(64, 64 * args.cpu_seconds / tp)))
        pts = [(int(b), int(m)) for b, m in zip(pr.integers(0, count, k), pr.integers(0, L, k))]
        t0 = time.perf_counter()
        ref = OF.filter1d_batch(sig_np, sc_np, order, model, "clamp", pts)
        tc = time.perf_counter() - t0
        extra["err_vs_oracle"] = errors(np.array([s[b, m] for b, m in pts]), ref)
        cpu = {"value": k / tc / 1e6, "unit": "Msample/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} random samples of the same {count}x{L} batch (exact rational sums, Python, "
                         f"one thread), {tc:.1f} s"}
    config = {"workload": f"signal1d: {count} signals x {L} f32 unit-grid samples, smooth scales [1,16] "
                          f"(knots every 256 samples), order {order}, impulse model, clamp, {path} path",
              "samples": N, "order": order, "model": model, "path": path}
    extra["wall_s"] = wall
    return record(N / (ms * 1e-3) / 1e6, ms * 1e-3 * reps, reps, args.warmup,
                  "f64" if path == "f64" else "f64-compute/f32-out", config, roof, cpu, extra, unit="Msample/s")


def rect_flops_per_pixel(order: int, model: int) -> float:
    """Interpolation-weighted tap MACs of the two-direction mask: (n+1)^2 taps x (D+1)^2
    tensor B-spline weights x 2, D = model + n."""
    D = model + order
    return 2.0 * (order + 1) ** 2 * (D + 1) ** 2


def workload_rect(args):
    """The two-direction (rect, N = 2) filter (bsf_filter_rect): 2048 x 2048 uint8 blurred
    noise, two smooth scale fields in [1, 16], order 2, impulse model.  One step = one call
    (restart windows, running sums along rows and columns, the separable mask)."""
    import torch
    from paper_0908_3861_amd import binding
    import oracle.rect as OR
    order, model, path = 2, -1, args.path
    img_np, sc_np = synth.rect_workload((args.size, args.size))
    H, W = img_np.shape
    dev = torch.device("cuda:0")
    img = torch.from_numpy(img_np).to(dev)
    sc = torch.from_numpy(sc_np).to(dev)
    out = torch.empty((H, W), dtype=torch.float64 if path == "f64" else torch.float32, device=dev)
    ctx = binding.default_context(0)
    stream = torch.cuda.current_stream()

    def step():
        binding.filter_rect(img, sc, order, model, path, "clamp", a_max=16.0, out=out, ctx=ctx, stream=stream)

    wall, ms = time_steps(step, args.steps, args.warmup, stream)
    ctx.check_device()
    P = H * W
    T, halo = 32, 2 * math.ceil(17 * order / 2 + (model + order + 1) / 2) + 2
    box = math.ceil(W / T) * math.ceil(H / T) * (T + halo) ** 2
    flops = P * rect_flops_per_pixel(order, model) + box * 2.0 * order
    roof = {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
            "frac": flops / (ms * 1e-3) / PEAK_FP64_VALU, "traffic": None}
    alg_bytes = P * (1 + 8 + (8 if path == "f64" else 4))
    extra = {"filter_ms": ms, "hbm_algorithmic_GBps": alg_bytes / (ms * 1e-3) / 1e9,
             "flops_per_pixel": rect_flops_per_pixel(order, model)}
    cpu = None
    if not args.no_cpu_baseline:
        s = out.cpu().numpy().reshape(-1).astype(np.float64)
        pr = np.random.default_rng(12348)
        probe = pr.choice(P, size=64, replace=False)
        t0 = time.perf_counter()
        OR.filter_rect(img_np, sc_np, order, model, "clamp", probe)
        tp = max(time.perf_counter() - t0, 1e-3)
        k = int(min(P, max(64, 64 * args.cpu_seconds / tp)))
        pix = np.sort(pr.choice(P, size=k, replace=False))
        t0 = time.perf_counter()
        ref = OR.filter_rect(img_np, sc_np, order, model, "clamp", pix)
        tc = time.perf_counter() - t0
        extra["err_vs_oracle"] = errors(s[pix], ref)
        cpu = {"value": k / tc / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} random pixels of the same {W}x{H} image (separable direct sum, numpy, one thread), "
                         f"{tc:.1f} s"}
    config = {"workload": f"rect: {W}x{H} uint8 blurred-noise image, two smooth real scale fields in [1,16], "
                          f"two-direction box spline, order {order}, impulse model, {path} path",
              "pixels": P, "order": order, "model": model, "path": path}
    return record(P * args.steps / wall / 1e6, wall, args.steps, args.warmup,
                  "f64" if path == "f64" else "f64-compute/f32-out", config, roof, cpu, extra)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--path", default="f64", choices=["f64", "f32tiled"])
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--workload", default="plain",
                    choices=["plain", "small", "precision", "batched", "serving", "stage1", "ellipse", "signal1d",
                             "rect"])
    ap.add_argument("--no-f32-leg", action="store_true", help="plain workload: skip the float32-output leg")
    ap.add_argument("--kappa-seconds", type=float, default=6.0, help="CPU time for the kappa percentiles")
    ap.add_argument("--serving-seconds", type=float, default=15.0,
                    help="plain workload: length of the short serving stream (0: skip)")
    ap.add_argument("--serving-compare", action="store_true", help="serving: also run the stream with eager launches")
    ap.add_argument("--signals", type=int, default=1024)
    ap.add_argument("--length", type=int, default=65536)
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--rate", type=float, default=0.0)
    ap.add_argument("--pool", type=int, default=24)
    ap.add_argument("--max-side", type=int, default=4096)
    ap.add_argument("--budget-gib", type=int, default=32)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--copy-probe-mib", type=int, default=0, help="also run a device copy of this size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "every workload here fits one MI355X.", file=sys.stderr)
        sys.exit(2)
    fn = {"plain": workload_plain, "small": workload_small, "precision": workload_precision,
          "batched": workload_batched, "serving": workload_serving, "stage1": workload_stage1,
          "ellipse": workload_ellipse, "signal1d": workload_signal1d, "rect": workload_rect}[args.workload]
    print(json.dumps(fn(args)), flush=True)


if __name__ == "__main__":
    main()
