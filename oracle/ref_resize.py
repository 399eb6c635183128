"""FP64 reference resampler.

TEST INFRASTRUCTURE ONLY. This module is the oracle that the HIP library is
checked against. Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the library itself never does, and it shares no
code, header, table or constant with the HIP path.

What it computes (paper section II.B, eqs. 1-5, generalised to 4x4 taps):

For an image of size N_in along one axis resized to N_out, the source
coordinate of output index x is taken at pixel centres,

    s(x) = ((2x + 1) N_in - N_out) / (2 N_out)        (eq. 1, half-pixel reading)

the base tap is x0 = floor(s) and the fractional offset t = s - x0
(eqs. 2-4, with int() read as floor). Bilinear uses taps x0, x0+1 with weights
(1 - t, t); Keys bicubic uses taps x0-1 .. x0+2 with weights K(t - j) for
j = -1..2 (Keys 1981, parameter a, -0.5 by default). Every tap index is clamped
to [0, N_in - 1] (replicate edge). An output value is

    v = sum_j sum_i wy_j wx_i src[clamp(y0 + j)][clamp(x0 + i)]

(eq. 5, with the second bracket's weight read as (1 - offsetX) so that the four
weights sum to one). Everything is evaluated in float64. The adjoint scatters
wy_j wx_i g[y][x] onto the same clamped taps.

Images are arrays of shape (planes, height, width, channels).

Parity status: every function below is pinned in tests/test_oracle.py against
brute force in exact rational arithmetic, closed forms, invariants and
independent library routines (torch, PIL).
"""

from __future__ import annotations

import numpy as np

BILINEAR = 0
BICUBIC = 1
KEYS_A = -0.5


def source_coordinate(x, n_in: int, n_out: int):
    """Half-pixel form of eq. 1: s = ((2x+1) n_in - n_out) / (2 n_out), in float64.

    The numerator and denominator are exact integers, so s carries a single
    rounding.
    """
    x = np.asarray(x, dtype=np.int64)
    num = (2 * x + 1) * int(n_in) - int(n_out)
    return num.astype(np.float64) / float(2 * int(n_out))


def keys_kernel(d, a: float = KEYS_A):
    """Keys cubic convolution kernel K(d) with parameter a (Keys 1981).

    K(d) = (a+2)|d|^3 - (a+3)|d|^2 + 1        for |d| <= 1
         = a|d|^3 - 5a|d|^2 + 8a|d| - 4a       for 1 < |d| < 2
         = 0                                    otherwise
    """
    d = np.abs(np.asarray(d, dtype=np.float64))
    near = (a + 2.0) * d ** 3 - (a + 3.0) * d ** 2 + 1.0
    far = a * d ** 3 - 5.0 * a * d ** 2 + 8.0 * a * d - 4.0 * a
    return np.where(d <= 1.0, near, np.where(d < 2.0, far, 0.0))


def axis_taps(n_in: int, n_out: int, filt: int, a: float = KEYS_A):
    """Per output index: clamped tap indices and float64 weights.

    Returns (idx, w, x0, t) with idx, w of shape (n_out, k), k = 2 (bilinear)
    or 4 (bicubic); idx[x, j] is the clamped source index of tap j and w[x, j]
    its weight; x0 = floor(s) and t = s - x0 (eqs. 2-4).
    """
    s = source_coordinate(np.arange(n_out), n_in, n_out)
    x0 = np.floor(s)
    t = s - x0
    x0 = x0.astype(np.int64)
    if filt == BILINEAR:
        offs = np.array([0, 1], dtype=np.int64)
        w = np.stack([1.0 - t, t], axis=1)
    elif filt == BICUBIC:
        offs = np.array([-1, 0, 1, 2], dtype=np.int64)
        w = keys_kernel(t[:, None] - offs[None, :].astype(np.float64), a)
    else:
        raise ValueError(f"unknown filter {filt}")
    idx = np.clip(x0[:, None] + offs[None, :], 0, n_in - 1)
    return idx, w, x0, t


def _as_planes(img) -> np.ndarray:
    img = np.asarray(img)
    if img.ndim == 2:
        img = img[None, :, :, None]
    elif img.ndim == 3:
        img = img[None]
    if img.ndim != 4:
        raise ValueError("image must have shape (H, W), (H, W, C) or (P, H, W, C)")
    return img.astype(np.float64)


def resize_rows(img, out_h: int, out_w: int, rows, filt: int, a: float = KEYS_A,
                absolute: bool = False) -> np.ndarray:
    """Output rows ``rows`` of the resize of ``img`` (P, H, W, C) to (out_h, out_w).

    Returns float64 of shape (P, len(rows), out_w, C). Direct double sum over
    the taps of each output pixel (eq. 5 generalised). With ``absolute`` the
    sum is taken over |w_y w_x src| instead: the scale of the rounding error of
    any evaluation of the same sum.
    """
    src = _as_planes(img)
    if absolute:
        src = np.abs(src)
    _, in_h, in_w, _ = src.shape
    rows = np.asarray(rows, dtype=np.int64)
    iy, wy, _, _ = axis_taps(in_h, out_h, filt, a)
    ix, wx, _, _ = axis_taps(in_w, out_w, filt, a)
    iy, wy = iy[rows], wy[rows]
    if absolute:
        wy, wx = np.abs(wy), np.abs(wx)
    out = np.zeros((src.shape[0], rows.size, out_w, src.shape[3]), dtype=np.float64)
    k = iy.shape[1]
    for j in range(k):
        src_rows = src[:, iy[:, j]]                      # (P, R, W, C)
        for i in range(k):
            wgt = wy[:, j][:, None] * wx[:, i][None, :]  # (R, out_w)
            out += wgt[None, :, :, None] * src_rows[:, :, ix[:, i]]
    return out


def resize(img, out_h: int, out_w: int, filt: int, a: float = KEYS_A) -> np.ndarray:
    """Whole-image resize, float64, shape (P, out_h, out_w, C)."""
    return resize_rows(img, out_h, out_w, np.arange(out_h), filt, a)


def adjoint(grad_out, in_h: int, in_w: int, filt: int, a: float = KEYS_A,
            absolute: bool = False) -> np.ndarray:
    """Adjoint of ``resize`` with respect to its input.

    grad_out has shape (P, out_h, out_w, C); returns float64 (P, in_h, in_w, C)
    with grad_src[p, clamp(y0+j), clamp(x0+i), c] += wy_j wx_i grad_out[p, y, x, c].
    With ``absolute`` it accumulates |wy_j wx_i g| (the rounding-error scale).
    """
    g = _as_planes(grad_out)
    if absolute:
        g = np.abs(g)
    planes, out_h, out_w, ch = g.shape
    iy, wy, _, _ = axis_taps(in_h, out_h, filt, a)
    ix, wx, _, _ = axis_taps(in_w, out_w, filt, a)
    if absolute:
        wy, wx = np.abs(wy), np.abs(wx)
    gs = np.zeros((planes, in_h, in_w, ch), dtype=np.float64)
    k = iy.shape[1]
    for j in range(k):
        for i in range(k):
            wgt = wy[:, j][:, None] * wx[:, i][None, :]
            rows_idx = np.broadcast_to(iy[:, j][:, None], (out_h, out_w))
            cols_idx = np.broadcast_to(ix[:, i][None, :], (out_h, out_w))
            np.add.at(gs, (slice(None), rows_idx, cols_idx), wgt[None, :, :, None] * g)
    return gs


def axis_matrix(n_in: int, n_out: int, filt: int, a: float = KEYS_A) -> np.ndarray:
    """Dense (n_out, n_in) interpolation matrix of one axis: A[x, idx] += w."""
    idx, w, _, _ = axis_taps(n_in, n_out, filt, a)
    m = np.zeros((n_out, n_in), dtype=np.float64)
    for j in range(idx.shape[1]):
        np.add.at(m, (np.arange(n_out), idx[:, j]), w[:, j])
    return m


def quantize_u8(v) -> np.ndarray:
    """Round half to even, then clamp to [0, 255] (uint8 storage)."""
    return np.clip(np.rint(np.asarray(v, dtype=np.float64)), 0.0, 255.0).astype(np.uint8)


def quantize_f16(v) -> np.ndarray:
    """Round to nearest even float16 directly from float64."""
    return np.asarray(v, dtype=np.float64).astype(np.float16)


def needed_rows(in_h: int, out_h: int, row0: int, rows: int, filt: int):
    """Inclusive range of clamped source rows that output rows [row0, row0+rows) read."""
    iy, _, _, _ = axis_taps(in_h, out_h, filt)
    sel = iy[row0:row0 + rows]
    return int(sel.min()), int(sel.max())

