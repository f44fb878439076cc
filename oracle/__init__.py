"""CPU oracle for the space-variant four-direction box-spline filter.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP path (``paper_0908_3861_amd``) and never imports it.

* ``box_spline(x, a, n)``   -- the order-n four-direction box spline B_a(x)
  (Section 4, eq. def with N = 4; order n = n-fold self-convolution), evaluated
  exactly (up to rounding) by cell-wise integration of its segment-convolution
  definition; see ``bsf_oracle.c``.
* ``filter(img, scales, n)`` -- s[m] = sum_k f_ext[k] B_{a(m)}(m - k), the
  projection of Section 6 with phi = delta (Section 7).  Every term is
  non-negative, so plain float64 is accurate to a few ulps.
* ``box_spline_model(x, a, n, n1)``, ``filter_model(img, scales, n, n1)`` -- the same for
  the continuous image models f(x) = sum_k c[k] phi(x - k), phi = beta^{n1} (x) beta^{n1}
  (Section 6): the box spline convolved with phi, and the projections with the
  interpolating coefficients c.
* ``preintegrate(window, n)`` -- stage 1 alone: the recursion of Section 7
  (eq. RS, steps (1)-(4)), n times per direction, unit weights, exact integers.

Sibling modules: ``oracle.ellipse`` (the scale field of elliptical windows),
``oracle.filter1d`` (the one-dimensional scale-adaptive filter of Section 3, exact rationals,
with the prefiltered B-spline models) and ``oracle.rect`` (the two-direction box spline,
eq. def with N = 2, with any of those models).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

BORDERS = {"clamp": 0, "zero": 1}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (never hipcc)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.bsf_oracle_box_spline.restype = ctypes.c_double
        lib.bsf_oracle_box_spline.argtypes = [ctypes.c_double, ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.bsf_oracle_filter.restype = ctypes.c_int
        lib.bsf_oracle_filter.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_ssize_t,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p]
        lib.bsf_oracle_box_spline_model.restype = ctypes.c_double
        lib.bsf_oracle_box_spline_model.argtypes = [ctypes.c_double, ctypes.c_double,
                                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int]
        lib.bsf_oracle_filter_model.restype = ctypes.c_int
        lib.bsf_oracle_filter_model.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_ssize_t,
                                                ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.bsf_oracle_preintegrate.restype = ctypes.c_int
        lib.bsf_oracle_preintegrate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_void_p]
        _lib = lib
    return _lib


def box_spline(x1: float, x2: float, a, n: int) -> float:
    arr = (ctypes.c_double * 4)(*[float(v) for v in a])
    return float(_load().bsf_oracle_box_spline(float(x1), float(x2), arr, int(n)))


def filter(img: np.ndarray, scales: np.ndarray, n: int, border: str = "clamp",
           pixels: np.ndarray | None = None, threads: int | None = None) -> np.ndarray:
    """s[m] for every pixel ([H, W] float64), or for the flat indices ``pixels``."""
    lib = _load()
    f = np.ascontiguousarray(img, dtype=np.float64)
    sc = np.ascontiguousarray(scales, dtype=np.float32)
    H, W = f.shape
    assert sc.shape == (H, W, 4)
    if threads is not None:
        os.environ["OMP_NUM_THREADS"] = str(threads)
    if pixels is None:
        out = np.empty((H, W), np.float64)
        rc = lib.bsf_oracle_filter(f.ctypes.data, H, W, W, sc.ctypes.data, int(n), BORDERS[border],
                                   None, 0, out.ctypes.data)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        out = np.empty(pix.shape[0], np.float64)
        rc = lib.bsf_oracle_filter(f.ctypes.data, H, W, W, sc.ctypes.data, int(n), BORDERS[border],
                                   pix.ctypes.data, pix.shape[0], out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle filter rejected its arguments (rc={rc})")
    return out


def box_spline_model(x1: float, x2: float, a, n: int, n1: int) -> float:
    """(phi * B_a)(x) with phi = beta^{n1} (x) beta^{n1} (n1 = -1: B_a itself)."""
    arr = (ctypes.c_double * 4)(*[float(v) for v in a])
    return float(_load().bsf_oracle_box_spline_model(float(x1), float(x2), arr, int(n), int(n1)))


def filter_model(img: np.ndarray, scales: np.ndarray, n: int, n1: int, border: str = "clamp",
                 pixels: np.ndarray | None = None) -> np.ndarray:
    """s[m] = sum_k c[k] (phi * B_a(m))(m - k) (Section 6) for the continuous model of degree
    n1 in {-1, 0, 1, 2, 3}: c = f_ext for n1 <= 1, the exact interpolating coefficients of
    f_ext (oracle.rect.coefficients_2d, rounded to float64) for n1 = 2, 3."""
    from . import rect as _rect
    lib = _load()
    f = np.ascontiguousarray(img, dtype=np.float64)
    sc = np.ascontiguousarray(scales, dtype=np.float32)
    H, W = f.shape
    assert sc.shape == (H, W, 4)
    amax = float(sc.max())
    org = int(np.ceil(0.5 * n * amax * (1.0 + np.sqrt(2.0)) + 0.5 * (max(n1, -1) + 1))) + 2
    if n1 <= 1:
        ys = np.arange(-org, H + org)
        xs = np.arange(-org, W + org)
        c = f[np.ix_(np.clip(ys, 0, H - 1), np.clip(xs, 0, W - 1))].copy()
        if border == "zero":
            c[(ys < 0) | (ys >= H), :] = 0.0
            c[:, (xs < 0) | (xs >= W)] = 0.0
    else:
        rows = _rect.coefficients_2d(f, n1, border, -org, H + org, -org, W + org)
        c = np.array([[float(v) for v in r] for r in rows])
    c = np.ascontiguousarray(c)
    pitch = c.shape[1]
    if pixels is None:
        out = np.empty((H, W), np.float64)
        rc = lib.bsf_oracle_filter_model(c.ctypes.data, H, W, pitch, org, sc.ctypes.data, int(n), int(n1),
                                         None, 0, out.ctypes.data)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        out = np.empty(pix.shape[0], np.float64)
        rc = lib.bsf_oracle_filter_model(c.ctypes.data, H, W, pitch, org, sc.ctypes.data, int(n), int(n1),
                                         pix.ctypes.data, pix.shape[0], out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle filter_model rejected its arguments (rc={rc})")
    return out


def preintegrate(window: np.ndarray, n: int, wrap: bool = False) -> np.ndarray:
    """Unit-weight n-fold pre-integration of an integer window ([Hq, Wq], row 0 = smallest k2).

    The recursions run in 128-bit integers.  With ``wrap=False`` a value outside int64 raises
    OverflowError; with ``wrap=True`` the low 64 bits of every exact value are returned (the
    result modulo 2^64, as two's-complement int64)."""
    lib = _load()
    w = np.ascontiguousarray(window, dtype=np.int64)
    Hq, Wq = w.shape
    g = np.empty_like(w)
    rc = lib.bsf_oracle_preintegrate(w.ctypes.data, Hq, Wq, int(n), g.ctypes.data)
    if rc == -2 and not wrap:
        raise OverflowError("pre-integrated value exceeds int64")
    if rc not in (0, -2):
        raise ValueError("bad arguments")
    return g
