"""Exact rational evaluation of single output values of the resize.

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: the parity tests use it to
judge the few uint8 pixels where a float32 evaluation may round to the other
side of a .5 boundary. The library never imports it.

It computes the same definition as ``ref_resize`` (paper section II.B, eqs.
1-5, read with pixel centres or the printed map, floor for int(), every tap
index clamped to the image; Keys a = -1/2 for the bicubic; the antialiased
variant with the stretched, renormalised kernel), but in Python ``Fraction``
arithmetic, so the value and the distance to a rounding boundary are exact:

    s   = ((2x + 1) n_in - n_out) / (2 n_out)  or  x n_in / n_out   (eq. 1)
    x0  = floor(s), t = s - x0                                       (eqs. 2-4)
    v   = sum_j sum_i wy_j wx_i src[clamp(y0 + j)][clamp(x0 + i)]   (eq. 5)

``abs_scale`` is the same double sum over |wy_j| |wx_i| |src|, tap by tap: the
scale of the rounding error of any evaluation of the sum in that tap order.

Parity status: pinned in tests/test_oracle.py against the exact all-taps brute
force (a separate derivation) and against ``ref_resize`` in float64.
"""

from __future__ import annotations

from fractions import Fraction
from typing import List, Tuple

BILINEAR = 0
BICUBIC = 1
NEAREST = 2
BILINEAR_AA = 3
BICUBIC_AA = 4
HALF_PIXEL = 0
CORNER = 1

KEYS_A = Fraction(-1, 2)


def keys(d: Fraction, a: Fraction = KEYS_A) -> Fraction:
    """Keys (1981) cubic convolution kernel K(d), exact."""
    d = abs(d)
    if d <= 1:
        return (a + 2) * d ** 3 - (a + 3) * d ** 2 + 1
    if d < 2:
        return a * d ** 3 - 5 * a * d ** 2 + 8 * a * d - 4 * a
    return Fraction(0)


def tent(d: Fraction) -> Fraction:
    d = abs(d)
    return 1 - d if d < 1 else Fraction(0)


def axis_taps(x: int, n_in: int, n_out: int, filt: int, mapping: int = HALF_PIXEL) -> List[Tuple[int, Fraction]]:
    """(clamped source index, exact weight) of every tap of output index x,
    in ascending tap order (duplicates after clamping are kept apart)."""
    if filt in (BILINEAR_AA, BICUBIC_AA):
        return _axis_taps_aa(x, n_in, n_out, filt)
    if mapping == HALF_PIXEL:
        s = Fraction((2 * x + 1) * n_in - n_out, 2 * n_out)
    elif mapping == CORNER:
        s = Fraction(x * n_in, n_out)
    else:
        raise ValueError(f"unknown mapping {mapping}")
    if filt == NEAREST:
        # the pixel whose area contains s: [i - 1/2, i + 1/2) with pixel
        # centres, [i, i + 1) with the printed map
        i = (s + Fraction(1, 2)).__floor__() if mapping == HALF_PIXEL else s.__floor__()
        return [(min(max(i, 0), n_in - 1), Fraction(1))]
    x0 = s.__floor__()
    t = s - x0
    if filt == BILINEAR:
        offs = (0, 1)
        w = (1 - t, t)
    elif filt == BICUBIC:
        offs = (-1, 0, 1, 2)
        w = tuple(keys(t - j) for j in offs)
    else:
        raise ValueError(f"unknown filter {filt}")
    return [(min(max(x0 + j, 0), n_in - 1), wj) for j, wj in zip(offs, w)]


def _axis_taps_aa(x: int, n_in: int, n_out: int, filt: int) -> List[Tuple[int, Fraction]]:
    """Antialiased taps: sigma = max(1, n_in / n_out); every source i inside
    the image with |i - s| < R sigma (R = 1 tent, 2 Keys), weight
    K((i - s) / sigma) divided by the sum of those weights."""
    r = 1 if filt == BILINEAR_AA else 2
    s = Fraction((2 * x + 1) * n_in - n_out, 2 * n_out)
    sigma = Fraction(n_in, n_out) if n_in > n_out else Fraction(1)
    reach = r * sigma
    lo = max((s - reach).__floor__() + 1, 0)
    hi = min((s + reach).__floor__(), n_in - 1)
    kern = tent if filt == BILINEAR_AA else keys
    vals = [(i, kern((i - s) / sigma)) for i in range(lo, hi + 1)]
    total = sum(v for _, v in vals)
    return [(i, v / total) for i, v in vals]


def value(img, out_h: int, out_w: int, filt: int, p: int, y: int, x: int, c: int,
          mapping: int = HALF_PIXEL) -> Fraction:
    """Exact output value at plane p, row y, column x, channel c of the resize
    of img (P, H, W, C) whose samples are exact binary fractions (integers,
    float16 or float32 values)."""
    in_h, in_w = img.shape[1], img.shape[2]
    ty = axis_taps(y, in_h, out_h, filt, mapping)
    tx = axis_taps(x, in_w, out_w, filt, mapping)
    v = Fraction(0)
    for r, wy in ty:
        for q, wx in tx:
            v += wy * wx * Fraction(float(img[p, r, q, c]))
    return v


def abs_scale(img, out_h: int, out_w: int, filt: int, p: int, y: int, x: int, c: int,
              mapping: int = HALF_PIXEL) -> Fraction:
    """sum over the taps of |wy_j| |wx_i| |src| at one output value, exact."""
    in_h, in_w = img.shape[1], img.shape[2]
    ty = axis_taps(y, in_h, out_h, filt, mapping)
    tx = axis_taps(x, in_w, out_w, filt, mapping)
    v = Fraction(0)
    for r, wy in ty:
        for q, wx in tx:
            v += abs(wy) * abs(wx) * abs(Fraction(float(img[p, r, q, c])))
    return v


def taps_per_axis(n_in: int, n_out: int, filt: int) -> int:
    """Largest number of taps of any output index on this axis."""
    if filt == NEAREST:
        return 1
    if filt == BILINEAR:
        return 2
    if filt == BICUBIC:
        return 4
    # antialiased: at most floor(2 R sigma) + 1 sources lie within R sigma of s
    r = 1 if filt == BILINEAR_AA else 2
    return (2 * r * n_in) // n_out + 1 if n_in > n_out else 2 * r + 1
