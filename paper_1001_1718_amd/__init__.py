"""MI355X (gfx950) bilinear / Keys-bicubic image resize behind a C ABI.

PyTorch supplies device memory and streams; every pixel is computed by the HIP
kernels in libxresize.so. Functions here only translate tensors into the
library's image descriptors.

Layouts: ``"hwc"`` tensors are (H, W), (H, W, C) or (P, H, W, C) with C in
{1, 4} interleaved channels; ``"nchw"`` tensors are (N, C, H, W) planes.
"""

from __future__ import annotations

import ctypes
import os

import torch

from . import _lib
from ._lib import (  # noqa: F401
    XR_BICUBIC,
    XR_BILINEAR,
    XR_F16,
    XR_F32,
    XR_KERNEL_AUTO,
    XR_KERNEL_GATHER,
    XR_KERNEL_STRIP,
    XR_KERNEL_STRIP_ANY,
    XR_KERNEL_STRIP_LDS,
    XR_MAP_HALF_PIXEL,
    XR_MAP_PAPER,
    XR_NEAREST,
    XR_BILINEAR_AA,
    XR_BICUBIC_AA,
    XR_U8,
    XResizeError,
    XrImage,
    XrJob,
    XrTile,
    check,
    lib,
    tile,
)

_DTYPES = {torch.uint8: XR_U8, torch.float16: XR_F16, torch.float32: XR_F32}
_FILTERS = {"bilinear": XR_BILINEAR, "bicubic": XR_BICUBIC, "nearest": XR_NEAREST,
            "bilinear_aa": XR_BILINEAR_AA, "bicubic_aa": XR_BICUBIC_AA}
_MAPPINGS = {"half_pixel": XR_MAP_HALF_PIXEL, "paper": XR_MAP_PAPER}


def filter_code(mode) -> int:
    if isinstance(mode, int):
        return mode
    try:
        return _FILTERS[mode]
    except KeyError:
        raise ValueError(f"mode must be one of {sorted(_FILTERS)}, not {mode!r}") from None


def mapping_code(mapping) -> int:
    if isinstance(mapping, int):
        return mapping
    try:
        return _MAPPINGS[mapping]
    except KeyError:
        raise ValueError(f"mapping must be 'half_pixel' or 'paper', not {mapping!r}") from None


def _stream_handle(t: torch.Tensor, stream=None):
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(stream.cuda_stream)


def image(t: torch.Tensor, layout: str = "hwc", row0: int = 0, height: int | None = None) -> XrImage:
    """Descriptor of tensor ``t``. For a row band pass the band's first logical
    row ``row0`` and the full logical ``height``."""
    if t.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {t.dtype}")
    es = t.element_size()
    if layout == "hwc":
        if t.dim() == 2:
            planes, rows, width, ch = 1, t.shape[0], t.shape[1], 1
            s_plane, s_row, s_col, s_ch = 0, t.stride(0), t.stride(1), 1
        elif t.dim() == 3:
            planes, (rows, width, ch) = 1, t.shape
            s_plane, (s_row, s_col, s_ch) = 0, t.stride()
        elif t.dim() == 4:
            planes, rows, width, ch = t.shape
            s_plane, s_row, s_col, s_ch = t.stride()
        else:
            raise ValueError("hwc tensors are (H, W), (H, W, C) or (P, H, W, C)")
        if (ch > 1 and s_ch != 1) or s_col != ch:
            raise ValueError("pixels must be contiguous within a row (channels interleaved)")
    elif layout == "nchw":
        if t.dim() != 4:
            raise ValueError("nchw tensors are (N, C, H, W)")
        n, c, rows, width = t.shape
        sn, sc, s_row, s_col = t.stride()
        if s_col != 1:
            raise ValueError("rows must be contiguous")
        planes, ch = n * c, 1
        if n > 1 and c > 1 and sn != sc * c:
            raise ValueError("planes must be equally spaced (contiguous N, C)")
        s_plane = sc if c > 1 else sn
    else:
        raise ValueError(f"unknown layout {layout!r}")
    im = XrImage()
    im.data = t.data_ptr()
    im.width = width
    im.height = rows if height is None else int(height)
    im.channels = ch
    im.dtype = _DTYPES[t.dtype]
    im.row_pitch = s_row * es
    im.planes = planes
    im.plane_pitch = s_plane * es if planes > 1 else 0
    im.row0 = int(row0)
    im.rows = rows
    return im


def _tile_ptr(t):
    return ctypes.byref(t) if t is not None else None


def resize_into(src: torch.Tensor, dst: torch.Tensor, mode="bilinear", layout="hwc", tile=None,
                src_row0: int = 0, src_height: int | None = None, dst_row0: int = 0,
                dst_height: int | None = None, stream=None, mapping="half_pixel") -> torch.Tensor:
    """Resize ``src`` into the preallocated ``dst`` (both on the same GPU).
    ``mode``: 'bilinear', 'bicubic', 'nearest', 'bilinear_aa' or 'bicubic_aa'
    (antialiased: the filter stretched when shrinking); ``mapping``:
    'half_pixel' (pixel centres) or 'paper' (eq. 1 as printed, s = x * in / out)."""
    s = image(src, layout, src_row0, src_height)
    d = image(dst, layout, dst_row0, dst_height)
    f, m = filter_code(mode), mapping_code(mapping)
    if m == XR_MAP_HALF_PIXEL and f in (XR_BILINEAR, XR_BICUBIC):
        fn = lib.xr_resize_bicubic if f == XR_BICUBIC else lib.xr_resize_bilinear
        rc = fn(ctypes.byref(s), ctypes.byref(d), _tile_ptr(tile), _stream_handle(src, stream))
    else:
        rc = lib.xr_resize(ctypes.byref(s), ctypes.byref(d), f, m, _tile_ptr(tile),
                           _stream_handle(src, stream))
    check(rc, "resize")
    return dst


def resize(x: torch.Tensor, size, mode="bilinear", layout="hwc", tile=None, stream=None,
           mapping="half_pixel") -> torch.Tensor:
    """Resize to ``size = (out_h, out_w)``; returns a new tensor of x's dtype."""
    out_h, out_w = int(size[0]), int(size[1])
    if layout == "hwc":
        if x.dim() == 2:
            shape = (out_h, out_w)
        elif x.dim() == 3:
            shape = (out_h, out_w, x.shape[2])
        else:
            shape = (x.shape[0], out_h, out_w, x.shape[3])
    else:
        shape = (x.shape[0], x.shape[1], out_h, out_w)
    out = torch.empty(shape, dtype=x.dtype, device=x.device)
    return resize_into(x, out, mode, layout, tile, stream=stream, mapping=mapping)


def resize_backward(grad_out: torch.Tensor, in_size, mode="bilinear", layout="nchw",
                    out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Adjoint of ``resize`` w.r.t. its input (float32 or float16 gradients,
    summed in float32): returns A^T grad_out in grad_out's dtype."""
    in_h, in_w = int(in_size[0]), int(in_size[1])
    g = grad_out.contiguous()
    if out is None:
        if layout == "nchw":
            shape = (g.shape[0], g.shape[1], in_h, in_w)
        elif g.dim() == 2:
            shape = (in_h, in_w)
        elif g.dim() == 3:
            shape = (in_h, in_w, g.shape[2])
        else:
            shape = (g.shape[0], in_h, in_w, g.shape[3])
        out = torch.empty(shape, dtype=g.dtype, device=g.device)
    gd = image(g, layout)
    gs = image(out, layout)
    check(lib.xr_resize_backward(ctypes.byref(gd), ctypes.byref(gs), filter_code(mode),
                                 _stream_handle(g, stream)), "resize_backward")
    return out


class ResizeFn(torch.autograd.Function):
    """Differentiable resize of float32 or float16 NCHW tensors w.r.t. the input."""

    @staticmethod
    def forward(ctx, x, size, mode="bilinear"):
        ctx.in_size = (x.shape[2], x.shape[3])
        ctx.mode = mode
        return resize(x.contiguous(), size, mode, layout="nchw")

    @staticmethod
    def backward(ctx, grad_out):
        return resize_backward(grad_out, ctx.in_size, ctx.mode, layout="nchw"), None, None


class Batch:
    """A prepared batched launch over (src, dst, mode) triples of one dtype."""

    def __init__(self, pairs, tile=None, layout="hwc", stream=None):
        if not pairs:
            raise ValueError("empty batch")
        self.n = len(pairs)
        jobs = (XrJob * self.n)()
        for k, (s, d, mode) in enumerate(pairs):
            jobs[k].src = image(s, layout)
            jobs[k].dst = image(d, layout)
            jobs[k].filter = filter_code(mode)
        device = pairs[0][0].device
        nbytes = int(lib.xr_batch_workspace_bytes(self.n))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        self._jobs = jobs
        self._keep = pairs
        check(lib.xr_batch_prepare(jobs, self.n, _tile_ptr(tile), ctypes.c_void_p(self.ws_ptr),
                                   nbytes, _stream_handle(pairs[0][0], stream)), "batch_prepare")

    def run(self, stream=None):
        check(lib.xr_resize_batched(ctypes.c_void_p(self.ws_ptr), self.n,
                                    _stream_handle(self.workspace, stream)), "resize_batched")

    def autotune(self, candidates=None, reps: int = 3, groups: int = 3, stream=None):
        """Time batched launch shapes (xr_batch_autotune); re-prepares this
        batch with the fastest and returns (XrTile, ms per launch)."""
        best, ms = XrTile(), ctypes.c_float()
        if candidates is None:
            cand_ptr, nc = None, 0
        else:
            cand_ptr = (XrTile * len(candidates))(*candidates)
            nc = len(candidates)
        check(lib.xr_batch_autotune(self._jobs, self.n, cand_ptr, nc, reps, groups,
                                    ctypes.c_void_p(self.ws_ptr), self.ws_bytes, ctypes.byref(best),
                                    ctypes.byref(ms), _stream_handle(self.workspace, stream)),
              "batch_autotune")
        return best, float(ms.value)


def autotune(src, dst, mode="bicubic", layout="hwc", candidates=None, reps: int = 20,
             groups: int = 5, stream=None):
    """Time launch shapes; returns (best XrTile, ms per launch).

    ``src`` / ``dst`` are tensors or equally long lists of tensors; with lists
    the launches cycle through the pairs (use enough pairs to exceed the
    caches). The winner is remembered for later launches with the same key.
    """
    srcs = list(src) if isinstance(src, (list, tuple)) else [src]
    dsts = list(dst) if isinstance(dst, (list, tuple)) else [dst]
    if len(srcs) != len(dsts):
        raise ValueError("src and dst lists differ in length")
    n = len(srcs)
    s_arr = (XrImage * n)(*[image(t, layout) for t in srcs])
    d_arr = (XrImage * n)(*[image(t, layout) for t in dsts])
    best, ms = XrTile(), ctypes.c_float()
    if candidates is None:
        cand_ptr, nc = None, 0
    else:
        cand_ptr = (XrTile * len(candidates))(*candidates)
        nc = len(candidates)
    check(lib.xr_autotune(s_arr, d_arr, n, filter_code(mode), cand_ptr, nc, reps, groups,
                          ctypes.byref(best), ctypes.byref(ms), _stream_handle(srcs[0], stream)),
          "autotune")
    return best, float(ms.value)


def tune_save(path: str) -> None:
    """Write the tuned launch shapes to `path` (xr_tune_save)."""
    check(lib.xr_tune_save(os.fsencode(path)), "tune_save")


def tune_load(path: str) -> int:
    """Merge the launch shapes of `path` if it was written for this GPU and
    build (xr_tune_load); returns how many were loaded."""
    n = ctypes.c_int32()
    check(lib.xr_tune_load(os.fsencode(path), ctypes.byref(n)), "tune_load")
    return int(n.value)


def tune_candidates(mode, dtype_code, channels, in_w, in_h, out_w, out_h):
    n = lib.xr_tune_candidates(filter_code(mode), dtype_code, channels, in_w, in_h, out_w, out_h,
                               None, 0)
    arr = (XrTile * n)()
    lib.xr_tune_candidates(filter_code(mode), dtype_code, channels, in_w, in_h, out_w, out_h, arr, n)
    return list(arr)


def get_tile(mode, dtype_code, channels, in_w, in_h, out_w, out_h) -> XrTile:
    t = XrTile()
    check(lib.xr_get_tile(filter_code(mode), dtype_code, channels, in_w, in_h, out_w, out_h,
                          ctypes.byref(t)), "get_tile")
    return t


def set_tile(mode, dtype_code, channels, in_w, in_h, out_w, out_h, t: XrTile) -> None:
    check(lib.xr_set_tile(filter_code(mode), dtype_code, channels, in_w, in_h, out_w, out_h,
                          ctypes.byref(t)), "set_tile")


def source_taps(n_in: int, n_out: int, x: int):
    """(x0, t_num, t_den): base tap and exact offset t = t_num / t_den of output x."""
    x0, num, den = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    check(lib.xr_source_taps(n_in, n_out, x, ctypes.byref(x0), ctypes.byref(num), ctypes.byref(den)),
          "source_taps")
    return x0.value, num.value, den.value


def needed_rows(in_h: int, out_h: int, row0: int, rows: int, mode, mapping="half_pixel") -> tuple:
    first, last = ctypes.c_int32(), ctypes.c_int32()
    check(lib.xr_needed_rows_map(in_h, out_h, row0, rows, filter_code(mode), mapping_code(mapping),
                                 ctypes.byref(first), ctypes.byref(last)), "needed_rows")
    return first.value, last.value


def thread_of_pixel(t: XrTile, px: int, py: int) -> tuple:
    vals = [ctypes.c_int32() for _ in range(6)]
    check(lib.xr_thread_of_pixel(ctypes.byref(t), px, py, *[ctypes.byref(v) for v in vals]),
          "thread_of_pixel")
    return tuple(v.value for v in vals)
