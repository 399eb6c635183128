"""ctypes front end of the plain-C FP64 oracle (test infrastructure only)."""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIBRARY

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise RuntimeError(f"{LIBRARY} is not built; run oracle/build.py or __graft_entry__.build()")
        lib = ctypes.CDLL(LIBRARY)
        i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.oracle_resize_rows.argtypes = [vp, i64, i64, i64, i64, vp, i64, i64, ctypes.c_int, dbl,
                                           vp, i64, ctypes.c_int]
        lib.oracle_resize_rows.restype = ctypes.c_int
        lib.oracle_adjoint.argtypes = [vp, i64, i64, i64, i64, vp, i64, i64, ctypes.c_int, dbl,
                                       ctypes.c_int]
        lib.oracle_adjoint.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _planes_f32(img) -> np.ndarray:
    img = np.asarray(img)
    if img.ndim == 2:
        img = img[None, :, :, None]
    elif img.ndim == 3:
        img = img[None]
    if img.ndim != 4:
        raise ValueError("image must have shape (H, W), (H, W, C) or (P, H, W, C)")
    if img.dtype not in (np.uint8, np.float16, np.float32):
        raise TypeError("the C oracle reads uint8, float16 or float32 pixels")
    return np.ascontiguousarray(img.astype(np.float32, copy=False))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def resize_rows(img, out_h: int, out_w: int, rows, filt: int, a: float = -0.5,
                threads: int = 0) -> np.ndarray:
    """float64 (P, len(rows), out_w, C) output rows, computed pixel by pixel in C."""
    src = _planes_f32(img)
    planes, in_h, in_w, ch = src.shape
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.empty((planes, rows.size, out_w, ch), dtype=np.float64)
    rc = _load().oracle_resize_rows(src.ctypes.data, planes, in_h, in_w, ch, out.ctypes.data,
                                    int(out_h), int(out_w), int(filt), float(a),
                                    rows.ctypes.data, rows.size, int(threads))
    if rc != 0:
        raise ValueError("oracle_resize_rows rejected its arguments")
    return out


def resize(img, out_h: int, out_w: int, filt: int, a: float = -0.5, threads: int = 0) -> np.ndarray:
    return resize_rows(img, out_h, out_w, np.arange(out_h), filt, a, threads)


def adjoint(grad_out, in_h: int, in_w: int, filt: int, a: float = -0.5, threads: int = 0) -> np.ndarray:
    g = _planes_f32(grad_out)
    planes, out_h, out_w, ch = g.shape
    out = np.empty((planes, in_h, in_w, ch), dtype=np.float64)
    rc = _load().oracle_adjoint(g.ctypes.data, planes, out_h, out_w, ch, out.ctypes.data,
                                int(in_h), int(in_w), int(filt), float(a), int(threads))
    if rc != 0:
        raise ValueError("oracle_adjoint rejected its arguments")
    return out
