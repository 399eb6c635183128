"""FP64 reference resampler.

TEST INFRASTRUCTURE ONLY. This module is the oracle that the HIP library is
checked against. Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the library itself never does, and it shares no
code, header, table or constant with the HIP path.

What it computes (paper section II.B, eqs. 1-5, generalised to 4x4 taps):

For an image of size N_in along one axis resized to N_out, the source
coordinate of output index x is taken at pixel centres,

    s(x) = ((2x + 1) N_in - N_out) / (2 N_out)        (eq. 1, half-pixel reading)

or, with mapping=CORNER, as eq. 1 prints it, s(x) = x N_in / N_out.

the base tap is x0 = floor(s) and the fractional offset t = s - x0
(eqs. 2-4, with int() read as floor). Bilinear uses taps x0, x0+1 with weights
(1 - t, t); Keys bicubic uses taps x0-1 .. x0+2 with weights K(t - j) for
j = -1..2 (Keys 1981, parameter a, -0.5 by default). Every tap index is clamped
to [0, N_in - 1] (replicate edge). An output value is

    v = sum_j sum_i wy_j wx_i src[clamp(y0 + j)][clamp(x0 + i)]

(eq. 5, with the second bracket's weight read as (1 - offsetX) so that the four
weights sum to one). Everything is evaluated in float64. The adjoint scatters
wy_j wx_i g[y][x] onto the same clamped taps. Nearest neighbour (named among
the paper's interpolation methods in section II) takes the one source pixel
whose area contains the mapped point.

Images are arrays of shape (planes, height, width, channels).

Parity status: every function below is pinned in tests/test_oracle.py against
brute force in exact rational arithmetic, closed forms, invariants and
independent library routines (torch, PIL).
"""

from __future__ import annotations

import numpy as np

BILINEAR = 0
BICUBIC = 1
NEAREST = 2
KEYS_A = -0.5

HALF_PIXEL = 0  # pixel centres aligned: s = (x + 1/2) n_in / n_out - 1/2
CORNER = 1      # eq. 1 as printed: s = x_f / scale with scale = n_out / n_in


def source_coordinate(x, n_in: int, n_out: int, mapping: int = HALF_PIXEL):
    """Source coordinate of output index x (eq. 1), in float64.

    HALF_PIXEL: s = ((2x+1) n_in - n_out) / (2 n_out) (pixel centres aligned);
    CORNER:     s = x n_in / n_out (eq. 1 as printed, x_p = x_f / scale, the
                scale taken from the two sizes).
    The numerator and denominator are exact integers, so s carries a single
    rounding.
    """
    x = np.asarray(x, dtype=np.int64)
    if mapping == HALF_PIXEL:
        num, den = (2 * x + 1) * int(n_in) - int(n_out), 2 * int(n_out)
    elif mapping == CORNER:
        num, den = x * int(n_in), int(n_out)
    else:
        raise ValueError(f"unknown mapping {mapping}")
    return num.astype(np.float64) / float(den)


def nearest_index(x, n_in: int, n_out: int, mapping: int = HALF_PIXEL):
    """Nearest neighbour: the source pixel whose area contains the mapped
    point. Pixel i covers [i - 1/2, i + 1/2) in half-pixel coordinates and
    [i, i + 1) in the corner convention, so the index is floor(s + 1/2),
    respectively floor(s), from exact integers; clamped to [0, n_in - 1]."""
    x = np.asarray(x, dtype=np.int64)
    if mapping == HALF_PIXEL:
        idx = ((2 * x + 1) * int(n_in)) // (2 * int(n_out))  # floor(s + 1/2)
    elif mapping == CORNER:
        idx = (x * int(n_in)) // int(n_out)                    # floor(s)
    else:
        raise ValueError(f"unknown mapping {mapping}")
    return np.clip(idx, 0, int(n_in) - 1)


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


def axis_taps(n_in: int, n_out: int, filt: int, a: float = KEYS_A, mapping: int = HALF_PIXEL):
    """Per output index: clamped tap indices and float64 weights.

    Returns (idx, w, x0, t) with idx, w of shape (n_out, k), k = 1 (nearest),
    2 (bilinear) or 4 (bicubic); idx[x, j] is the clamped source index of tap
    j and w[x, j] its weight; x0 = floor(s) and t = s - x0 (eqs. 2-4).
    """
    if filt == NEAREST:
        idx = nearest_index(np.arange(n_out), n_in, n_out, mapping)
        return idx[:, None], np.ones((n_out, 1)), idx, np.zeros(n_out)
    s = source_coordinate(np.arange(n_out), n_in, n_out, mapping)
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


BILINEAR_AA = 3
BICUBIC_AA = 4
AA_RADIUS = {BILINEAR_AA: 1, BICUBIC_AA: 2}


def axis_taps_antialiased(n_in: int, n_out: int, filt: int, a: float = KEYS_A):
    """Antialiased taps (not in the paper; the usual remedy for aliasing when
    shrinking): the filter is stretched by sigma = max(1, n_in / n_out), so
    output x (pixel-centre s(x)) reads every source pixel i with
    |i - s| < R sigma (R = 1 bilinear, 2 Keys), weight K((i - s) / sigma);
    taps outside the image are dropped (not clamped) and the weights are
    divided by their sum. The tap range comes from exact integers:
    i > s - R sigma and i <= s + R sigma.

    Returns (idx, w) of shape (n_out, kmax), unused slots with weight 0.
    """
    n_in, n_out = int(n_in), int(n_out)
    r = AA_RADIUS[filt]
    down = n_in > n_out
    rows_idx, rows_w = [], []
    for x in range(n_out):
        num = (2 * x + 1) * n_in - n_out  # s = num / (2 n_out)
        if down:  # sigma = n_in / n_out: s -/+ R sigma = (num -/+ 2 R n_in) / (2 n_out)
            lo = (num - 2 * r * n_in) // (2 * n_out) + 1
            hi = (num + 2 * r * n_in) // (2 * n_out)
        else:     # sigma = 1
            lo = (num - 2 * r * n_out) // (2 * n_out) + 1
            hi = (num + 2 * r * n_out) // (2 * n_out)
        lo, hi = max(lo, 0), min(hi, n_in - 1)
        i = np.arange(lo, hi + 1, dtype=np.int64)
        s = num / (2.0 * n_out)
        sigma = n_in / n_out if down else 1.0
        d = (i - s) / sigma
        k = np.maximum(1.0 - np.abs(d), 0.0) if filt == BILINEAR_AA else keys_kernel(d, a)
        rows_idx.append(i)
        rows_w.append(k / k.sum())
    kmax = max(len(i) for i in rows_idx)
    idx = np.zeros((n_out, kmax), dtype=np.int64)
    w = np.zeros((n_out, kmax))
    for x in range(n_out):
        idx[x, :len(rows_idx[x])] = rows_idx[x]
        w[x, :len(rows_w[x])] = rows_w[x]
    return idx, w


def resize_antialiased(img, out_h: int, out_w: int, filt: int, rows=None, a: float = KEYS_A,
                       absolute: bool = False) -> np.ndarray:
    """Antialiased resize (BILINEAR_AA or BICUBIC_AA), pixel centres, float64,
    shape (P, len(rows), out_w, C): the same double sum as ``resize_rows``
    with the taps of ``axis_taps_antialiased``."""
    src = _as_planes(img)
    if absolute:
        src = np.abs(src)
    _, in_h, in_w, _ = src.shape
    rows = np.arange(out_h) if rows is None else np.asarray(rows, dtype=np.int64)
    iy, wy = axis_taps_antialiased(in_h, out_h, filt, a)
    ix, wx = axis_taps_antialiased(in_w, out_w, filt, a)
    iy, wy = iy[rows], wy[rows]
    if absolute:
        wy, wx = np.abs(wy), np.abs(wx)
    out = np.zeros((src.shape[0], rows.size, out_w, src.shape[3]), dtype=np.float64)
    for j in range(iy.shape[1]):
        src_rows = src[:, iy[:, j]]
        for i in range(ix.shape[1]):
            wgt = wy[:, j][:, None] * wx[:, i][None, :]
            out += wgt[None, :, :, None] * src_rows[:, :, ix[:, i]]
    return out


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
                absolute: bool = False, mapping: int = HALF_PIXEL) -> np.ndarray:
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
    iy, wy, _, _ = axis_taps(in_h, out_h, filt, a, mapping)
    ix, wx, _, _ = axis_taps(in_w, out_w, filt, a, mapping)
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


def resize(img, out_h: int, out_w: int, filt: int, a: float = KEYS_A,
           mapping: int = HALF_PIXEL) -> np.ndarray:
    """Whole-image resize, float64, shape (P, out_h, out_w, C)."""
    return resize_rows(img, out_h, out_w, np.arange(out_h), filt, a, mapping=mapping)


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


def axis_matrix(n_in: int, n_out: int, filt: int, a: float = KEYS_A,
                mapping: int = HALF_PIXEL) -> np.ndarray:
    """Dense (n_out, n_in) interpolation matrix of one axis: A[x, idx] += w."""
    idx, w, _, _ = axis_taps(n_in, n_out, filt, a, mapping)
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


def needed_rows(in_h: int, out_h: int, row0: int, rows: int, filt: int,
                mapping: int = HALF_PIXEL):
    """Inclusive range of clamped source rows that output rows [row0, row0+rows) read."""
    iy, _, _, _ = axis_taps(in_h, out_h, filt, mapping=mapping)
    sel = iy[row0:row0 + rows]
    return int(sel.min()), int(sel.max())

