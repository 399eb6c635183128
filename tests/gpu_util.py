"""Shared helpers of the GPU parity tests: comparison rules against the oracle.

Tolerances (derived from the float32 evaluation order):
* uint8, dyadic scale ratios (every offset t a multiple of 1/4, so every
  weight is k / 2^m): every float32 partial sum is exact, so the GPU must
  equal rint-half-even + clamp of the oracle on every pixel, ties included;
* uint8, other ratios: the float32 value differs from the exact one by at
  most B = 1.25 (e_x + e_y + n_x + n_y) u S (u = 2^-24, S = sum |w_y w_x v|
  over the taps, e the weights' relative error in units of u, n the taps per
  axis; see ``f32_units``). Its rounding can therefore differ from the
  exact value's only where that value lies within B of a .5 boundary. Every
  mismatch is judged on the exact rational value (``oracle.exact``):
  - it must be a +-1 step across the boundary k + 1/2 next to the exact
    value, and the exact value must lie within B of it;
  - exact ties (value exactly k + 1/2, possible when the weights have small
    odd denominators) may round either way: the exact value is the tie, the
    float32 one is not;
  - the share of mismatches that are not exact ties is gated at 1e-4 of the
    compared values (the reading of the stated 1e-6 band, which is narrower
    than a float32 ulp at 128-255): the count must not exceed the Poisson
    quantile of mean 1e-4 N at false-alarm rate 1e-6, so small cases are not
    failed by chance and large ones are held to the share;
* float16: |gpu - oracle| <= 1e-3 (values in [0, 1]) and at most one float16
  ulp away from the oracle's own float16 rounding;
* float32: |gpu - oracle| <= 1e-5 * sum |w_y w_x v| per pixel (the derived
  bound above is at most 40 u S = 2.4e-6 S for bicubic weights);
* float16 gradients (sums of unbounded size): half a float16 ulp at the
  value's magnitude + the float32 bound.
"""

import math
from fractions import Fraction

import numpy as np

from oracle import exact as EX
from oracle import ref_resize as R

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


U = 2.0 ** -24
U8_SHARE = 1e-4


def f32_units(filt: int, n_in: int, n_out: int):
    """(e, n) of one axis: the float32 weights' relative error bound in units
    of u, and the taps per output index. Bilinear: t and 1 - t are each one
    correctly rounded quotient (e = 1). Keys a = -1/2 in its factored forms:
    at most 16 u (the K(t) factor 2 + t (2 - 3t), whose inner difference may
    cancel, contributes about 13 u absolute on a value >= 1). Antialiased:
    kernel values (8 u), their sum over n taps (n u, amplified at most 1.2x
    by the negative lobes) and the reciprocal and product (2 u), bounded by
    10 + 2n."""
    n = EX.taps_per_axis(n_in, n_out, filt)
    if filt == R.NEAREST:
        return 0, 1
    if filt == R.BILINEAR:
        return 1, 2
    if filt == R.BICUBIC:
        return 16, 4
    return 10 + 2 * n, n


def _poisson_upper(mean: float, alpha: float = 1e-6) -> int:
    """Smallest k with P(Poisson(mean) > k) <= alpha."""
    k, term = 0, math.exp(-mean)
    cdf = term
    while 1.0 - cdf > alpha:
        k += 1
        term *= mean / k
        cdf += term
    return k


def check_u8(gpu: np.ndarray, ref: np.ndarray, exact: bool, what: str = "", ctx=None):
    """uint8 output (P, R, W, C) against the float64 oracle values `ref` of
    the same rows. `ctx` = (planes, out_h, out_w, filt, rows, mapping)
    identifies the workload, for the exact value of each mismatch. Returns a
    dict of counts (and prints it when anything differs)."""
    want = R.quantize_u8(ref)
    gpu = np.asarray(gpu)
    assert gpu.shape == want.shape, (gpu.shape, want.shape)
    n_values = int(gpu.size)
    if exact:
        bad = np.argwhere(gpu != want)
        assert bad.size == 0, (f"{what}: {len(bad)} u8 mismatches on a dyadic ratio, first at "
                               f"{bad[:3].tolist()}: gpu {gpu[tuple(bad[0])]} want {want[tuple(bad[0])]} "
                               f"ref {ref[tuple(bad[0])]!r}")
        return {"values": n_values, "ties": 0, "non_ties": 0}
    assert ctx is not None, "non-dyadic uint8 comparisons need the workload to judge mismatches exactly"
    planes, out_h, out_w, filt, rows, mapping = ctx
    in_h, in_w = planes.shape[1], planes.shape[2]
    ex, nx = f32_units(filt, in_w, out_w)
    ey, ny = f32_units(filt, in_h, out_h)
    units = Fraction(5, 4) * (ex + ey + nx + ny)
    ties = non_ties = 0
    worst = Fraction(0)
    for p, k, x, c in np.argwhere(gpu != want):
        y = int(rows[k])
        v = EX.value(planes, out_h, out_w, filt, int(p), y, int(x), int(c), mapping)
        g = int(gpu[p, k, x, c])
        # the exact value's own rounding (half to even, clamped)
        fl = v.__floor__()
        rne = fl + 1 if (v - fl > Fraction(1, 2) or (v - fl == Fraction(1, 2) and fl % 2 == 1)) else fl
        rne = min(max(rne, 0), 255)
        if v - fl == Fraction(1, 2) and 0 <= fl and fl + 1 <= 255:
            assert g in (fl, fl + 1), f"{what}: u8 {g} at an exact tie {float(v)} at {(p, y, x, c)}"
            ties += 1
            continue
        if g == rne:
            continue  # the float64 oracle itself rounded across a boundary it lies within 1e-13 of
        assert abs(g - rne) == 1, f"{what}: u8 {g} vs exact rounding {rne} at {(p, y, x, c)}"
        boundary = Fraction(g + rne, 2)
        b = units * Fraction(U) * EX.abs_scale(planes, out_h, out_w, filt, int(p), y, int(x), int(c), mapping)
        dist = abs(v - boundary)
        assert dist <= b, (f"{what}: u8 {g} vs {rne} at {(p, y, x, c)}: exact value {float(v)!r} is "
                           f"{float(dist):.3g} from the boundary, beyond the float32 bound {float(b):.3g}")
        worst = max(worst, dist / b)
        non_ties += 1
    limit = _poisson_upper(U8_SHARE * n_values)
    res = {"values": n_values, "ties": ties, "non_ties": non_ties, "share": non_ties / max(n_values, 1),
           "limit": limit, "worst_dist_over_bound": float(worst)}
    if ties or non_ties:
        print(f"u8 flips {what}: {res}", flush=True)
    assert non_ties <= limit, (f"{what}: {non_ties} non-tie u8 flips in {n_values} values exceed the "
                               f"share {U8_SHARE} (limit {limit})")
    return res


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
        return check_u8(gpu, ref, exact, what, ctx=(planes, out_h, out_w, filt, np.asarray(rows), mapping))
    if planes.dtype == np.float16:
        return check_f16(gpu, ref, what)
    scale = (R.resize_antialiased(planes, out_h, out_w, filt, rows=rows, absolute=True) if aa
             else R.resize_rows(planes, out_h, out_w, rows, filt, absolute=True, mapping=mapping))
    return check_f32(gpu, ref, scale, what)
