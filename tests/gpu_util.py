"""Shared helpers of the GPU parity tests: comparison rules against the oracle.

Tolerances (derived from the float32 evaluation order):
* uint8, dyadic scale ratios (every weight k / 2^m): the float32 sums are exact,
  so the GPU must equal rint-half-even + clamp of the float64 oracle on every
  pixel, rounding ties included;
* uint8, other ratios: a pixel may differ from the oracle's rounding only by
  one, and only where the float64 value lies within U8_EPS of a .5 boundary:
  there both roundings are within float32 error of the exact value (ratios
  with exact ties, such as t = 1/3 weights, produce many such pixels; the
  rounding mode itself is pinned by the dyadic cases, which must be exact);
* float16: |gpu - oracle| <= 1e-3 (values in [0, 1]) and at most one float16
  ulp away from the oracle's own float16 rounding;
* float32: |gpu - oracle| <= 1e-5 * sum |w_y w_x v| per pixel;
* float16 gradients (sums of unbounded size): half a float16 ulp at the
  value's magnitude + the float32 bound.
"""

import numpy as np

from oracle import ref_resize as R

U8_EPS = 2.0 ** -10
F16_MAX_ABS = 1e-3
F32_REL = 1e-5


def is_dyadic_ratio(n_in: int, n_out: int, mapping: int = R.HALF_PIXEL) -> bool:
    """True when every offset t of the axis is a multiple of 1/4.

    Then the bilinear weights are multiples of 1/4 and the Keys weights
    multiples of 1/128, and every float32 partial sum over uint8 pixels is an
    exact multiple of 2^-14 below 2^23: the GPU's float32 value equals the
    exact one, so its rounding must match the oracle's everywhere.
    """
    x = np.arange(n_out, dtype=np.int64)
    if mapping == R.HALF_PIXEL:
        rem, den = ((2 * x + 1) * n_in - n_out) % (2 * n_out), 2 * n_out
    else:
        rem, den = (x * n_in) % n_out, n_out
    return bool(np.all((4 * rem) % den == 0))


def check_u8(gpu: np.ndarray, ref: np.ndarray, exact: bool, what: str = ""):
    want = R.quantize_u8(ref)
    gpu = np.asarray(gpu)
    assert gpu.shape == want.shape, (gpu.shape, want.shape)
    if exact:
        bad = np.argwhere(gpu != want)
        assert bad.size == 0, (f"{what}: {len(bad)} u8 mismatches on a dyadic ratio, first at "
                               f"{bad[:3].tolist()}: gpu {gpu[tuple(bad[0])]} want {want[tuple(bad[0])]} "
                               f"ref {ref[tuple(bad[0])]!r}")
        return 0
    diff = gpu.astype(np.int32) - want.astype(np.int32)
    bad = diff != 0
    n_bad = int(bad.sum())
    if n_bad:
        frac = np.abs(ref[bad] - np.floor(ref[bad]) - 0.5)
        assert np.all(np.abs(diff[bad]) == 1), f"{what}: u8 mismatch larger than 1"
        assert np.all(frac <= U8_EPS), f"{what}: u8 mismatch away from a .5 boundary (max {frac.max()})"
    return n_bad


def check_f16(gpu: np.ndarray, ref: np.ndarray, what: str = ""):
    g = np.asarray(gpu).astype(np.float64)
    err = np.abs(g - ref)
    assert err.max() <= F16_MAX_ABS, f"{what}: float16 max abs error {err.max()}"
    want = R.quantize_f16(ref).astype(np.float64)
    ulp = np.spacing(np.abs(want).astype(np.float16)).astype(np.float64)
    assert np.all(np.abs(g - want) <= ulp + 1e-30), f"{what}: more than one float16 ulp from the oracle"
    return float(err.max())


def check_f16_sum(gpu: np.ndarray, ref: np.ndarray, scale: np.ndarray, what: str = ""):
    """float16 storage of a float32 sum of unbounded size (gradients): the
    float32 value lies within 1e-5 * sum |w v| of the exact one and is then
    rounded once to float16, so |gpu - exact| <= half a float16 ulp at that
    magnitude + the float32 bound."""
    g = np.asarray(gpu).astype(np.float64)
    err = np.abs(g - ref)
    f32 = F32_REL * scale
    mag = (np.abs(ref) + f32).astype(np.float16)
    lim = 0.5 * np.spacing(mag).astype(np.float64) + f32 + 1e-30
    worst = float((err / lim).max())
    assert worst <= 1.0, f"{what}: float16 error {worst:.3g} x (half ulp + float32 bound)"
    return worst


def check_f32(gpu: np.ndarray, ref: np.ndarray, scale: np.ndarray, what: str = ""):
    g = np.asarray(gpu).astype(np.float64)
    err = np.abs(g - ref)
    lim = F32_REL * scale + 1e-30
    worst = float((err / lim).max())
    assert worst <= 1.0, f"{what}: float32 error {worst:.3g} x the 1e-5 * sum|w v| bound"
    return worst


def compare(gpu: np.ndarray, src_np: np.ndarray, out_h: int, out_w: int, filt: int, rows=None,
            what: str = "", use_c: bool = True, mapping: int = R.HALF_PIXEL):
    """Compare GPU output rows (P, R, W, C) with the oracle on the same rows.
    Nearest neighbour copies source values, so it must match exactly in every
    storage type; the C oracle covers the pixel-centre map with 2 or 4 taps."""
    from oracle import ref_c

    if mapping != R.HALF_PIXEL or filt not in (R.BILINEAR, R.BICUBIC):
        use_c = False
    aa = filt in (R.BILINEAR_AA, R.BICUBIC_AA)

    planes = src_np if src_np.ndim == 4 else (src_np[None] if src_np.ndim == 3 else src_np[None, :, :, None])
    in_h, in_w = planes.shape[1], planes.shape[2]
    if rows is None:
        rows = np.arange(out_h)
    gpu = np.asarray(gpu)
    if gpu.ndim == 2:
        gpu = gpu[None, :, :, None]
    elif gpu.ndim == 3:
        gpu = gpu[None]
    if aa:
        ref = R.resize_antialiased(planes, out_h, out_w, filt, rows=rows)
    elif use_c:
        ref = ref_c.resize_rows(planes, out_h, out_w, rows, filt)
    else:
        ref = R.resize_rows(planes, out_h, out_w, rows, filt, mapping=mapping)
    if filt == R.NEAREST:
        want = ref.astype(planes.dtype)
        np.testing.assert_array_equal(np.asarray(gpu).reshape(want.shape).view(np.uint8),
                                      want.view(np.uint8), err_msg=f"{what}: nearest is not an exact copy")
        return 0
    if planes.dtype == np.uint8:
        # antialiased weights are normalised in float32: never exact
        exact = (not aa) and is_dyadic_ratio(in_w, out_w, mapping) and is_dyadic_ratio(in_h, out_h, mapping)
        return check_u8(gpu, ref, exact, what)
    if planes.dtype == np.float16:
        return check_f16(gpu, ref, what)
    scale = (R.resize_antialiased(planes, out_h, out_w, filt, rows=rows, absolute=True) if aa
             else R.resize_rows(planes, out_h, out_w, rows, filt, absolute=True, mapping=mapping))
    return check_f32(gpu, ref, scale, what)
