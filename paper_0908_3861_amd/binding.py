"""Thin ctypes binding of libbsf (include/bsf.h): argument marshalling only.

Tensors come from PyTorch (device memory and the current HIP stream); every step of
the filter runs in the library's kernels.  There is no fallback: if ``libbsf.so`` is
missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libbsf.so")

U8, F32, F64 = 0, 1, 2
PATHS = {"f64": 0, "f32tiled": 1}
BORDERS = {"clamp": 0, "zero": 1}
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP error", 4: "unsupported",
          5: "scale out of range", 6: "integer range exceeded"}


class BsfError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__(f"bsf: {STATUS.get(status, status)}" + (f" ({detail})" if detail else ""))


class Job(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int), ("height", ctypes.c_int),
        ("in_dtype", ctypes.c_int), ("in_", ctypes.c_void_p), ("in_pitch", ctypes.c_ssize_t),
        ("scales", ctypes.c_void_p), ("scale_pitch", ctypes.c_ssize_t),
        ("order", ctypes.c_int), ("path", ctypes.c_int), ("border", ctypes.c_int),
        ("a_max", ctypes.c_float),
        ("out", ctypes.c_void_p), ("out_pitch", ctypes.c_ssize_t),
    ]


class Job1d(ctypes.Structure):
    _fields_ = [
        ("length", ctypes.c_int), ("count", ctypes.c_int),
        ("in_dtype", ctypes.c_int), ("in_", ctypes.c_void_p), ("in_pitch", ctypes.c_ssize_t),
        ("scales", ctypes.c_void_p), ("scale_pitch", ctypes.c_ssize_t),
        ("order", ctypes.c_int), ("model", ctypes.c_int), ("path", ctypes.c_int), ("border", ctypes.c_int),
        ("a_max", ctypes.c_float),
        ("out", ctypes.c_void_p), ("out_pitch", ctypes.c_ssize_t),
    ]


class JobRect(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int), ("height", ctypes.c_int),
        ("in_dtype", ctypes.c_int), ("in_", ctypes.c_void_p), ("in_pitch", ctypes.c_ssize_t),
        ("scales", ctypes.c_void_p), ("scale_pitch", ctypes.c_ssize_t),
        ("order", ctypes.c_int), ("model", ctypes.c_int), ("path", ctypes.c_int), ("border", ctypes.c_int),
        ("a_max", ctypes.c_float),
        ("out", ctypes.c_void_p), ("out_pitch", ctypes.c_ssize_t),
    ]


_lib = None
_lock = threading.Lock()


def load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(lib_path):
                raise RuntimeError(f"{lib_path} is missing: build it with `python -m paper_0908_3861_amd.build`")
            lib = ctypes.CDLL(lib_path)
            vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
            jp = ctypes.POINTER(Job)
            lib.bsf_create.argtypes = [ctypes.POINTER(vp), i, sz]
            lib.bsf_destroy.argtypes = [vp]
            lib.bsf_workspace_size.argtypes = [jp, ctypes.POINTER(sz)]
            lib.bsf_filter.argtypes = [vp, jp, vp]
            lib.bsf_filter_batched.argtypes = [vp, jp, i, vp]
            lib.bsf_filter_noalloc.argtypes = [vp, jp, vp]
            lib.bsf_filter_model.argtypes = [vp, jp, i, vp]
            lib.bsf_batch_plan_create.argtypes = [vp, i, ctypes.c_longlong, ctypes.c_float, ctypes.POINTER(vp)]
            lib.bsf_batch_plan_run.argtypes = [vp, jp, i, vp]
            lib.bsf_batch_plan_job_status.argtypes = [vp, ctypes.POINTER(i), i]
            lib.bsf_batch_plan_destroy.argtypes = [vp]
            lib.bsf_preintegrate.argtypes = [vp, jp, i, i, i, i, vp, ctypes.c_ssize_t, vp]
            lib.bsf_get_device_error.argtypes = [vp, vp]
            lib.bsf_get_counters.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_ulonglong), i]
            lib.bsf_scales_from_ellipses.argtypes = [vp, vp, ctypes.c_ssize_t, i, i, i, vp, ctypes.c_ssize_t, vp]
            lib.bsf_filter1d.argtypes = [vp, ctypes.POINTER(Job1d), vp]
            lib.bsf_filter1d_max_scale.argtypes = [vp, i, i, ctypes.POINTER(ctypes.c_float)]
            lib.bsf_filter_rect.argtypes = [vp, ctypes.POINTER(JobRect), vp]
            lib.bsf_filter_rect_max_scale.argtypes = [vp, i, i, ctypes.POINTER(ctypes.c_float)]
            lib.bsf_status_string.argtypes = [i]
            lib.bsf_status_string.restype = ctypes.c_char_p
            lib.bsf_last_error.argtypes = [vp]
            lib.bsf_last_error.restype = ctypes.c_char_p
            lib.bsf_debug_tile_window.argtypes = [vp, jp, i, vp, ctypes.c_longlong, vp, vp]
            for fn in ("bsf_create", "bsf_destroy", "bsf_workspace_size", "bsf_filter", "bsf_filter_batched",
                       "bsf_filter_noalloc", "bsf_filter_model", "bsf_batch_plan_create", "bsf_batch_plan_run", "bsf_batch_plan_job_status",
                       "bsf_batch_plan_destroy", "bsf_filter_rect", "bsf_filter_rect_max_scale",
                       "bsf_preintegrate", "bsf_get_device_error", "bsf_get_counters", "bsf_scales_from_ellipses",
                       "bsf_debug_tile_window", "bsf_filter1d", "bsf_filter1d_max_scale"):
                getattr(lib, fn).restype = i
            _lib = lib
    return _lib


class Context:
    """Owns a bsf_ctx on one HIP device."""

    def __init__(self, device: int | None = None, workspace_limit: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("bsf needs a HIP device; none is visible")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.lib = load()
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._check(self.lib.bsf_create(ctypes.byref(self._h), self.device, workspace_limit))

    def _check(self, st: int):
        if st != 0:
            detail = self.lib.bsf_last_error(self._h).decode() if self._h else ""
            raise BsfError(st, detail)

    @property
    def handle(self):
        return self._h

    def device_error(self, stream=None) -> int:
        return self.lib.bsf_get_device_error(self._h, _stream_ptr(stream))

    def check_device(self, stream=None):
        self._check(self.device_error(stream))

    def counters(self, stream=None, reset: bool = False) -> tuple[int, int]:
        """(pixels of the float64 path evaluated split, pixels evaluated again compensated)."""
        out = (ctypes.c_ulonglong * 2)()
        self._check(self.lib.bsf_get_counters(self._h, _stream_ptr(stream), out, int(reset)))
        return int(out[0]), int(out[1])

    def close(self):
        if self._h:
            self.lib.bsf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: dict[int, Context] = {}


def default_context(device: int | None = None) -> Context:
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.uint8:
        return U8
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"image dtype {t.dtype} is not uint8/float32/float64")


def make_job(img, scales, order: int, path: str = "f64", border: str = "clamp", a_max: float | None = None,
             out=None):
    """Build the C job (and the output tensor) for device tensors img [H,W], scales [H,W,4] f32."""
    import torch
    if img.dim() != 2 or scales.dim() != 3 or scales.shape[2] != 4:
        raise ValueError("expected img [H, W] and scales [H, W, 4]")
    H, W = img.shape
    if tuple(scales.shape[:2]) != (H, W):
        raise ValueError("scales must match the image size")
    if not (img.is_cuda and scales.is_cuda):
        raise ValueError("img and scales must be device tensors")
    if scales.dtype != torch.float32 or scales.stride(2) != 1 or scales.stride(1) != 4:
        raise ValueError("scales must be float32 with contiguous (a1..a4) per pixel")
    if img.stride(1) != 1:
        raise ValueError("image rows must be contiguous")
    odt = torch.float64 if path == "f64" else torch.float32
    if out is None:
        out = torch.empty((H, W), dtype=odt, device=img.device)
    elif out.dtype != odt or tuple(out.shape) != (H, W) or out.stride(1) != 1:
        raise ValueError("bad output tensor")
    if a_max is None:
        a_max = float(scales.max().item())
    j = Job()
    j.width, j.height = W, H
    j.in_dtype = _dtype_code(img)
    j.in_ = img.data_ptr()
    j.in_pitch = img.stride(0)
    j.scales = scales.data_ptr()
    j.scale_pitch = scales.stride(0) // 4
    j.order = int(order)
    j.path = PATHS[path]
    j.border = BORDERS[border]
    j.a_max = float(a_max)
    j.out = out.data_ptr()
    j.out_pitch = out.stride(0)
    return j, out


def _on(stream):
    """Allocate on the stream the library writes on (the caching allocator ties memory to it)."""
    import contextlib
    import torch
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def filter(img, scales, order: int, path: str = "f64", border: str = "clamp", a_max: float | None = None,
           out=None, ctx: Context | None = None, stream=None, check: bool = False, model: int = -1):
    """Adaptive box-spline filter of ``img`` with per-pixel scale vectors ``scales``.
    ``model`` >= 0 selects the continuous image model of that degree (bsf_filter_model)."""
    ctx = ctx or default_context(img.device.index)
    with _on(stream):
        j, out = make_job(img, scales, order, path, border, a_max, out)
    if model == -1:
        ctx._check(ctx.lib.bsf_filter(ctx.handle, ctypes.byref(j), _stream_ptr(stream)))
    else:
        ctx._check(ctx.lib.bsf_filter_model(ctx.handle, ctypes.byref(j), int(model), _stream_ptr(stream)))
    if check:
        ctx.check_device(stream)
    return out


def filter_noalloc(img, scales, order: int, path: str = "f64", border: str = "clamp", a_max: float | None = None,
                   out=None, ctx: Context | None = None, stream=None, check: bool = False):
    """``filter`` through bsf_filter_noalloc: the library allocates nothing (its work area is a
    fixed array per GPU; ``out`` and ``a_max`` should be given to keep the call free of torch
    allocations and host syncs too)."""
    ctx = ctx or default_context(img.device.index)
    with _on(stream):
        j, out = make_job(img, scales, order, path, border, a_max, out)
    ctx._check(ctx.lib.bsf_filter_noalloc(ctx.handle, ctypes.byref(j), _stream_ptr(stream)))
    if check:
        ctx.check_device(stream)
    return out


def filter_batched(items, ctx: Context | None = None, stream=None, check: bool = False):
    """items: list of dicts with keys img, scales, order[, path, border, a_max, out]."""
    if not items:
        return []
    ctx = ctx or default_context(items[0]["img"].device.index)
    jobs = (Job * len(items))()
    outs = []
    with _on(stream):
        for i, it in enumerate(items):
            j, o = make_job(it["img"], it["scales"], it["order"], it.get("path", "f64"), it.get("border", "clamp"),
                            it.get("a_max"), it.get("out"))
            jobs[i] = j
            outs.append(o)
    ctx._check(ctx.lib.bsf_filter_batched(ctx.handle, jobs, len(items), _stream_ptr(stream)))
    if check:
        ctx.check_device(stream)
    return outs


class BatchPlan:
    """A captured batched launch (bsf_batch_plan_*): create once, then ``run`` any batch of up
    to ``max_jobs`` jobs and ``max_tiles`` tiles whose scales are bounded by ``a_max``."""

    def __init__(self, ctx: Context, max_jobs: int, max_tiles: int, a_max: float):
        self.ctx = ctx
        self.lib = ctx.lib
        self.max_jobs = int(max_jobs)
        self.a_max = float(a_max)
        self._h = ctypes.c_void_p()
        ctx._check(self.lib.bsf_batch_plan_create(ctx.handle, self.max_jobs, int(max_tiles), self.a_max,
                                                  ctypes.byref(self._h)))
        self._last = 0

    def run(self, items, stream=None):
        """items: dicts as for ``filter_batched`` (each job's a_max defaults to the plan's).
        Returns the output tensors; the call is asynchronous on ``stream``."""
        jobs = (Job * max(len(items), 1))()
        outs = []
        with _on(stream):
            for i, it in enumerate(items):
                j, o = make_job(it["img"], it["scales"], it["order"], it.get("path", "f64"),
                                it.get("border", "clamp"), it.get("a_max") or self.a_max, it.get("out"))
                jobs[i] = j
                outs.append(o)
        self.ctx._check(self.lib.bsf_batch_plan_run(self._h, jobs, len(items), _stream_ptr(stream)))
        self._last = len(items)
        return outs

    def job_status(self) -> list[int]:
        """Per-job status of the last run (waits for it)."""
        st = (ctypes.c_int * max(self._last, 1))()
        self.ctx._check(self.lib.bsf_batch_plan_job_status(self._h, st, self._last))
        return [int(st[i]) for i in range(self._last)]

    def close(self):
        if self._h:
            self.lib.bsf_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scales_from_ellipses(ell, order: int, out=None, ctx: Context | None = None, stream=None):
    """[H, W, 3] float32 device tensor of (s_major, s_minor, phi) -> [H, W, 4] float32 scales
    for an order-`order` filter (bsf_scales_from_ellipses).  Rows may be padded (views)."""
    import torch
    ctx = ctx or default_context(ell.device.index)
    if ell.dtype != torch.float32 or ell.dim() != 3 or ell.shape[2] != 3 or ell.stride(2) != 1 or ell.stride(1) != 3:
        raise ValueError("ellipses must be a float32 [H, W, 3] tensor with contiguous pixels")
    if ell.stride(0) % 3:
        raise ValueError("the row pitch of the ellipses must be a whole number of pixels")
    H, W, _ = ell.shape
    if out is None:
        with _on(stream):
            out = torch.empty((H, W, 4), dtype=torch.float32, device=ell.device)
    if out.shape != (H, W, 4) or out.dtype != torch.float32 or out.stride(2) != 1 or out.stride(1) != 4 \
            or out.stride(0) % 4:
        raise ValueError("out must be a float32 [H, W, 4] tensor with contiguous pixels")
    ctx._check(ctx.lib.bsf_scales_from_ellipses(ctx.handle, ell.data_ptr(), ell.stride(0) // 3, W, H, int(order),
                                                out.data_ptr(), out.stride(0) // 4, _stream_ptr(stream)))
    return out


def filter1d_max_scale(order: int, model: int = -1, ctx: Context | None = None) -> float:
    """The largest scale bound bsf_filter1d accepts for this order and model (either path)."""
    ctx = ctx or default_context()
    v = ctypes.c_float()
    ctx._check(ctx.lib.bsf_filter1d_max_scale(ctx.handle, int(order), int(model), ctypes.byref(v)))
    return float(v.value)


def filter1d(signals, scales, order: int, model: int = -1, border: str = "clamp", a_max: float | None = None,
             out=None, ctx: Context | None = None, stream=None, check: bool = False, path: str = "f64"):
    """One-dimensional scale-adaptive filter (bsf_filter1d) of device tensors ``signals``
    [count, length] (uint8/float32/float64) with per-sample float32 ``scales`` [count, length];
    returns [count, length], float64 (path "f64") or float32 (path "f32tiled").  Rows may be padded (contiguous samples within a row).
    ``a_max`` defaults to the largest scale (one device reduction and a host sync)."""
    import torch
    ctx = ctx or default_context(signals.device.index)
    if signals.dim() != 2 or scales.dim() != 2 or tuple(scales.shape) != tuple(signals.shape):
        raise ValueError("expected signals and scales of the same shape [count, length]")
    if not (signals.is_cuda and scales.is_cuda):
        raise ValueError("signals and scales must be device tensors")
    if scales.dtype != torch.float32 or scales.stride(1) != 1 or signals.stride(1) != 1:
        raise ValueError("scales must be float32; samples within a row must be contiguous")
    count, length = signals.shape
    odt = torch.float64 if path == "f64" else torch.float32
    if out is None:
        with _on(stream):
            out = torch.empty((count, length), dtype=odt, device=signals.device)
    elif out.dtype != odt or tuple(out.shape) != (count, length) or out.stride(1) != 1:
        raise ValueError("bad output tensor")
    if a_max is None:
        with _on(stream):
            a_max = float(scales.max().item())
    j = Job1d()
    j.length, j.count = length, count
    j.in_dtype = _dtype_code(signals)
    j.in_ = signals.data_ptr()
    j.in_pitch = signals.stride(0)
    j.scales = scales.data_ptr()
    j.scale_pitch = scales.stride(0)
    j.order = int(order)
    j.model = int(model)
    j.path = PATHS[path]
    j.border = BORDERS[border]
    j.a_max = float(a_max)
    j.out = out.data_ptr()
    j.out_pitch = out.stride(0)
    ctx._check(ctx.lib.bsf_filter1d(ctx.handle, ctypes.byref(j), _stream_ptr(stream)))
    if check:
        ctx.check_device(stream)
    return out


def preintegrate(img, order: int, x0: int, y0: int, wq: int, hq: int, border: str = "clamp",
                 ctx: Context | None = None, stream=None):
    """Stage 1 alone on the window [y0, y0+hq) x [x0, x0+wq): int64 [hq, wq] (unit weights)."""
    import torch
    ctx = ctx or default_context(img.device.index)
    H, W = img.shape
    j = Job()
    j.width, j.height = W, H
    j.in_dtype = _dtype_code(img)
    j.in_ = img.data_ptr()
    j.in_pitch = img.stride(0)
    j.order = int(order)
    j.border = BORDERS[border]
    with _on(stream):
        g = torch.empty((hq, wq), dtype=torch.int64, device=img.device)
    ctx._check(ctx.lib.bsf_preintegrate(ctx.handle, ctypes.byref(j), x0, y0, wq, hq, g.data_ptr(), g.stride(0),
                                        _stream_ptr(stream)))
    return g


def debug_tile_window(img, scales, order: int, tile: int, centred: bool, path: str = "f64",
                      border: str = "clamp", cap: int = 1 << 20, ctx: Context | None = None):
    """Stage-1 window of one tile as computed on chip: (int64 [hq, wq], (x0, y0, wq, hq), overflow)."""
    import torch
    ctx = ctx or default_context(img.device.index)
    j, _ = make_job(img, scales, order, path, border, None, None)
    win = torch.zeros(cap, dtype=torch.int64, device=img.device)
    geom = torch.zeros(8, dtype=torch.int32, device=img.device)
    geom[4] = 1 if centred else 0
    ctx._check(ctx.lib.bsf_debug_tile_window(ctx.handle, ctypes.byref(j), int(tile), win.data_ptr(), cap,
                                             geom.data_ptr(), _stream_ptr()))
    torch.cuda.synchronize()
    x0, y0, wq, hq, _, ovf, sh, _ = [int(v) for v in geom.cpu()]
    return win[: wq * hq].view(hq, wq).cpu().numpy(), (x0, y0, wq, hq), bool(ovf)


def filter_rect_max_scale(order: int, model: int = -1, ctx: Context | None = None) -> float:
    """The largest scale bound bsf_filter_rect accepts for this order and model."""
    ctx = ctx or default_context()
    v = ctypes.c_float()
    ctx._check(ctx.lib.bsf_filter_rect_max_scale(ctx.handle, int(order), int(model), ctypes.byref(v)))
    return float(v.value)


def filter_rect(img, scales, order: int, model: int = -1, path: str = "f64", border: str = "clamp",
                a_max: float | None = None, out=None, ctx: Context | None = None, stream=None, check: bool = False):
    """Two-direction (rect) adaptive filter (bsf_filter_rect) of a device image [H, W]
    (uint8/float32/float64) with float32 scales [H, W, 2] = (a1 along x, a2 along y).
    ``a_max`` defaults to the largest scale (one device reduction and a host sync)."""
    import torch
    ctx = ctx or default_context(img.device.index)
    if img.dim() != 2 or scales.dim() != 3 or scales.shape[2] != 2 or tuple(scales.shape[:2]) != tuple(img.shape):
        raise ValueError("expected img [H, W] and scales [H, W, 2]")
    if not (img.is_cuda and scales.is_cuda):
        raise ValueError("img and scales must be device tensors")
    if scales.dtype != torch.float32 or scales.stride(2) != 1 or scales.stride(1) != 2 or img.stride(1) != 1:
        raise ValueError("scales must be float32 with contiguous (a1, a2) per pixel; image rows contiguous")
    H, W = img.shape
    odt = torch.float64 if path == "f64" else torch.float32
    if out is None:
        with _on(stream):
            out = torch.empty((H, W), dtype=odt, device=img.device)
    elif out.dtype != odt or tuple(out.shape) != (H, W) or out.stride(1) != 1:
        raise ValueError("bad output tensor")
    if a_max is None:
        with _on(stream):
            a_max = float(scales.max().item())
    j = JobRect()
    j.width, j.height = W, H
    j.in_dtype = _dtype_code(img)
    j.in_ = img.data_ptr()
    j.in_pitch = img.stride(0)
    j.scales = scales.data_ptr()
    j.scale_pitch = scales.stride(0) // 2
    j.order = int(order)
    j.model = int(model)
    j.path = PATHS[path]
    j.border = BORDERS[border]
    j.a_max = float(a_max)
    j.out = out.data_ptr()
    j.out_pitch = out.stride(0)
    ctx._check(ctx.lib.bsf_filter_rect(ctx.handle, ctypes.byref(j), _stream_ptr(stream)))
    if check:
        ctx.check_device(stream)
    return out
