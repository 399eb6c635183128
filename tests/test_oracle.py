"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* exact rational brute force ("all-i" form: every source sample weighted by the
  kernel evaluated at its distance, no floor and no tap selection);
* closed forms of the Keys weights and a hand-worked bilinear example
  (tests/golden/), plus invariants (partition of unity, moment reproduction);
* special cases: identity size, constants, ramps, quadratics;
* independent library routines: torch interpolate (bilinear; bicubic with
  a = -3/4; nearest-exact and nearest for the nearest filter under the two
  maps) and its backward, PIL float-mode bicubic in the interior;
* the paper's printed map (eq. 1, x_p = x_f / scale): exact brute force, the
  x2 closed form, and eqs. 1-5 evaluated literally pixel by pixel;
* the antialiased variant: PIL float-mode resize on whole images (edges
  renormalised alike), the x0.5 bilinear closed form, the plain filters in the
  interior when growing, partition of unity;
* adjoint by finite differences, by <Ax, y> = <x, A^T y> and by mass conservation;
* a mutation check: plausible mistakes planted into a copy of the oracle must
  be caught by the brute-force pin.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref_c
from oracle import ref_resize as R
from synth import fields

HALF = Fraction(1, 2)


# ---------------------------------------------------------------------------
# exact rational brute force, written independently of the oracle
# ---------------------------------------------------------------------------

def _kernel_exact(d: Fraction, filt: int, a: Fraction) -> Fraction:
    ad = abs(d)
    if filt == R.BILINEAR:
        return 1 - ad if ad < 1 else Fraction(0)
    if ad <= 1:
        return (a + 2) * ad ** 3 - (a + 3) * ad ** 2 + 1
    if ad < 2:
        return a * ad ** 3 - 5 * a * ad ** 2 + 8 * a * ad - 4 * a
    return Fraction(0)


def _axis_exact(n_in: int, n_out: int, filt: int, a: Fraction, corner: bool = False):
    """Dense exact (n_out, n_in) matrix from the all-i form: every integer i in a
    generous window contributes K(s - i) to column clamp(i). s is the pixel
    centre map, or with `corner` the paper's printed map x * n_in / n_out."""
    m = [[Fraction(0)] * n_in for _ in range(n_out)]
    for x in range(n_out):
        if corner:
            s = Fraction(x * n_in, n_out)
        else:
            s = Fraction((2 * x + 1) * n_in - n_out, 2 * n_out)
        lo = int(s) - 6
        for i in range(lo, lo + 13):
            w = _kernel_exact(s - i, filt, a)
            if w:
                m[x][min(max(i, 0), n_in - 1)] += w
    return m


def _brute_resize(img2d, out_h, out_w, filt, a=Fraction(-1, 2), corner=False):
    in_h, in_w = len(img2d), len(img2d[0])
    ay = _axis_exact(in_h, out_h, filt, a, corner)
    ax = _axis_exact(in_w, out_w, filt, a, corner)
    out = []
    for y in range(out_h):
        row = []
        for x in range(out_w):
            v = Fraction(0)
            for r in range(in_h):
                if ay[y][r] == 0:
                    continue
                for c in range(in_w):
                    if ax[x][c]:
                        v += ay[y][r] * ax[x][c] * Fraction(int(img2d[r][c]))
            row.append(v)
        out.append(row)
    return out


def _brute_adjoint(g2d, in_h, in_w, filt, a=Fraction(-1, 2)):
    out_h, out_w = len(g2d), len(g2d[0])
    ay = _axis_exact(in_h, out_h, filt, a)
    ax = _axis_exact(in_w, out_w, filt, a)
    gs = [[Fraction(0)] * in_w for _ in range(in_h)]
    for y in range(out_h):
        for x in range(out_w):
            gv = Fraction(int(g2d[y][x]))
            for r in range(in_h):
                if ay[y][r] == 0:
                    continue
                for c in range(in_w):
                    if ax[x][c]:
                        gs[r][c] += ay[y][r] * ax[x][c] * gv
    return gs


SHAPES = [  # (in_h, in_w, out_h, out_w): dyadic, non-dyadic, mixed up/down, non-square
    (8, 8, 16, 16),
    (8, 8, 4, 4),
    (8, 8, 13, 11),
    (7, 9, 5, 20),
    (8, 6, 3, 17),
    (5, 8, 2, 2),
    (1, 6, 3, 5),
]


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("shape", SHAPES)
def test_brute_force_exact(shape, filt):
    in_h, in_w, out_h, out_w = shape
    img = fields.uniform_u8((in_h, in_w), seed=11 + in_h * 31 + in_w)
    exact = _brute_resize(img.tolist(), out_h, out_w, filt)
    got = R.resize(img, out_h, out_w, filt)[0, :, :, 0]
    want = np.array([[float(v) for v in row] for row in exact])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    got_c = ref_c.resize(img, out_h, out_w, filt)[0, :, :, 0]
    np.testing.assert_allclose(got_c, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("shape", SHAPES)
def test_brute_force_exact_corner_mapping(shape, filt):
    in_h, in_w, out_h, out_w = shape
    img = fields.uniform_u8((in_h, in_w), seed=13 + in_h * 31 + in_w)
    exact = _brute_resize(img.tolist(), out_h, out_w, filt, corner=True)
    got = R.resize(img, out_h, out_w, filt, mapping=R.CORNER)[0, :, :, 0]
    want = np.array([[float(v) for v in row] for row in exact])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("shape", SHAPES[:5])
def test_brute_force_adjoint_exact(shape, filt):
    in_h, in_w, out_h, out_w = shape
    g = fields.uniform_u8((out_h, out_w), seed=5 + out_h * 7 + out_w).astype(np.int64) - 128
    exact = _brute_adjoint(g.tolist(), in_h, in_w, filt)
    want = np.array([[float(v) for v in row] for row in exact])
    got = R.adjoint(g.astype(np.float64), in_h, in_w, filt)[0, :, :, 0]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-10)
    got_c = ref_c.adjoint(g.astype(np.float32), in_h, in_w, filt)[0, :, :, 0]
    np.testing.assert_allclose(got_c, want, rtol=0, atol=1e-10)


# ---------------------------------------------------------------------------
# closed forms and the hand-worked example
# ---------------------------------------------------------------------------

def _read_golden(path):
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_keys_weights_closed_form(golden_dir):
    for a_s, t_s, *ws in _read_golden(os.path.join(golden_dir, "keys_weights.txt")):
        a, t = float(Fraction(a_s)), Fraction(t_s)
        want = [float(Fraction(w)) for w in ws]
        got = R.keys_kernel(float(t) - np.array([-1.0, 0.0, 1.0, 2.0]), a)
        np.testing.assert_array_equal(got, want)
        # and through the tap path of a size pair that produces this t
        if a == -0.5 and t == Fraction(1, 4):
            _, w, x0, tt = R.axis_taps(8, 16, R.BICUBIC)
            assert tt[1] == 0.25 and x0[1] == 0
            np.testing.assert_array_equal(w[1], want)


def test_bilinear_hand_worked(golden_dir):
    rows = [list(map(float, r)) for r in _read_golden(os.path.join(golden_dir, "bilinear_2x2_to_4x4.txt"))]
    img = np.array(rows[:2])
    want = np.array(rows[2:])
    np.testing.assert_array_equal(R.resize(img, 4, 4, R.BILINEAR)[0, :, :, 0], want)
    np.testing.assert_array_equal(ref_c.resize(img.astype(np.float32), 4, 4, R.BILINEAR)[0, :, :, 0], want)


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
def test_weight_moments(filt):
    rng = np.random.default_rng(3)
    for n_in, n_out in [(17, 40), (40, 17), (8, 16), (1000, 333)]:
        _, w, x0, t = R.axis_taps(n_in, n_out, filt)
        offs = np.arange(w.shape[1]) - (1 if filt == R.BICUBIC else 0)
        d = offs[None, :] - t[:, None]
        np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-15)            # partition of unity
        np.testing.assert_allclose((w * d).sum(1), 0.0, atol=1e-14)      # linear reproduction
        if filt == R.BICUBIC:                                            # quadratic (a = -1/2)
            np.testing.assert_allclose((w * d * d).sum(1), 0.0, atol=1e-14)
        assert np.all((t >= 0) & (t < 1))
    t = rng.random(1000)
    for j_sum in [R.keys_kernel(t[:, None] - np.array([-1, 0, 1, 2])[None, :], -0.5).sum(1)]:
        np.testing.assert_allclose(j_sum, 1.0, atol=1e-15)


def test_floor_not_truncation():
    # x2 upscale: s(0) = -1/4 must give x0 = -1, t = 3/4 (floor), not x0 = 0, t = -1/4.
    _, _, x0, t = R.axis_taps(8, 16, R.BILINEAR)
    assert x0[0] == -1 and t[0] == 0.75
    s = R.source_coordinate(np.arange(16), 8, 16)
    np.testing.assert_array_equal(s, (2 * np.arange(16) - 1) / 4.0)


# ---------------------------------------------------------------------------
# special cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
def test_identity_size(filt):
    img = fields.uniform_u8((2, 13, 29, 4), seed=7)
    np.testing.assert_array_equal(R.resize(img, 13, 29, filt), img.astype(np.float64))
    np.testing.assert_array_equal(ref_c.resize(img, 13, 29, filt), img.astype(np.float64))


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("out", [(37, 19), (5, 3), (64, 64)])
def test_constant_image(filt, out):
    img = np.full((1, 23, 17, 1), 173.0)
    got = R.resize(img, out[0], out[1], filt)
    np.testing.assert_allclose(got, 173.0, rtol=0, atol=1e-12)


def _interior(n_in, n_out, lo, hi_off):
    s = R.source_coordinate(np.arange(n_out), n_in, n_out)
    return s, (s >= lo) & (s <= n_in - 1 - hi_off)


@pytest.mark.parametrize("sizes", [(13, 17, 29, 23), (40, 31, 17, 12), (16, 16, 32, 32)])
def test_bilinear_reproduces_ramps(sizes):
    in_h, in_w, out_h, out_w = sizes
    yy, xx = np.mgrid[0:in_h, 0:in_w].astype(np.float64)
    img = 3.0 + 1.75 * xx - 0.5 * yy
    got = R.resize(img, out_h, out_w, R.BILINEAR)[0, :, :, 0]
    sy, my = _interior(in_h, out_h, 0, 0)
    sx, mx = _interior(in_w, out_w, 0, 0)
    want = 3.0 + 1.75 * sx[None, :] - 0.5 * sy[:, None]
    m = my[:, None] & mx[None, :]
    assert m.sum() > 0
    np.testing.assert_allclose(got[m], want[m], rtol=0, atol=1e-11)


@pytest.mark.parametrize("sizes", [(13, 17, 29, 23), (40, 31, 17, 12), (16, 16, 32, 32)])
def test_bicubic_reproduces_quadratics(sizes):
    in_h, in_w, out_h, out_w = sizes
    yy, xx = np.mgrid[0:in_h, 0:in_w].astype(np.float64)

    def f(y, x):
        return 2.0 + 0.5 * x - 0.25 * y + 0.03 * x * x - 0.02 * y * y + 0.015 * x * y

    img = f(yy, xx)
    got = R.resize(img, out_h, out_w, R.BICUBIC)[0, :, :, 0]
    sy, my = _interior(in_h, out_h, 1, 1)
    sx, mx = _interior(in_w, out_w, 1, 1)
    m = my[:, None] & mx[None, :]
    assert m.sum() > 0
    want = f(sy[:, None], sx[None, :])
    np.testing.assert_allclose(got[m], want[m], rtol=0, atol=1e-10)
    # bilinear does not reproduce the curvature: the pin must be able to fail
    bil = R.resize(img, out_h, out_w, R.BILINEAR)[0, :, :, 0]
    assert np.abs(bil[m] - want[m]).max() > 1e-3


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
def test_dense_separable_form(filt):
    img = fields.uniform_u8((2, 11, 14, 3), seed=9)
    out_h, out_w = 23, 9
    ay = R.axis_matrix(11, out_h, filt)
    ax = R.axis_matrix(14, out_w, filt)
    got = R.resize(img, out_h, out_w, filt)
    for p in range(2):
        for c in range(3):
            want = ay @ img[p, :, :, c].astype(np.float64) @ ax.T
            np.testing.assert_allclose(got[p, :, :, c], want, rtol=0, atol=1e-11)


# ---------------------------------------------------------------------------
# library routines
# ---------------------------------------------------------------------------

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _torch_interp(img2d, out_h, out_w, mode):
    t = torch.from_numpy(np.asarray(img2d, dtype=np.float64))[None, None]
    return F.interpolate(t, size=(out_h, out_w), mode=mode, align_corners=False)[0, 0].numpy()


@pytest.mark.parametrize("sizes", [(16, 16, 32, 32), (13, 17, 29, 23), (40, 31, 17, 12), (9, 9, 9, 9)])
def test_torch_bilinear_pin(sizes):
    in_h, in_w, out_h, out_w = sizes
    img = fields.normal_f32((in_h, in_w), seed=21).astype(np.float64)
    want = _torch_interp(img, out_h, out_w, "bilinear")
    np.testing.assert_allclose(R.resize(img, out_h, out_w, R.BILINEAR)[0, :, :, 0], want,
                               rtol=0, atol=1e-13)


@pytest.mark.parametrize("sizes", [(16, 16, 32, 32), (13, 17, 29, 23), (40, 31, 17, 12)])
def test_torch_bicubic_pin_a075(sizes):
    in_h, in_w, out_h, out_w = sizes
    img = fields.normal_f32((in_h, in_w), seed=22).astype(np.float64)
    want = _torch_interp(img, out_h, out_w, "bicubic")
    got = R.resize(img, out_h, out_w, R.BICUBIC, a=-0.75)[0, :, :, 0]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    got_c = ref_c.resize(img.astype(np.float32), out_h, out_w, R.BICUBIC, a=-0.75)[0, :, :, 0]
    want32 = _torch_interp(img.astype(np.float32).astype(np.float64), out_h, out_w, "bicubic")
    np.testing.assert_allclose(got_c, want32, rtol=0, atol=1e-12)


@pytest.mark.parametrize("sizes", [(16, 16, 32, 32), (13, 17, 29, 23), (40, 31, 17, 12)])
def test_torch_bilinear_backward_pin(sizes):
    in_h, in_w, out_h, out_w = sizes
    g = fields.normal_f32((out_h, out_w), seed=23).astype(np.float64)
    x = torch.zeros((1, 1, in_h, in_w), dtype=torch.float64, requires_grad=True)
    y = F.interpolate(x, size=(out_h, out_w), mode="bilinear", align_corners=False)
    y.backward(torch.from_numpy(g)[None, None])
    want = x.grad[0, 0].numpy()
    np.testing.assert_allclose(R.adjoint(g, in_h, in_w, R.BILINEAR)[0, :, :, 0], want,
                               rtol=0, atol=1e-13)


@pytest.mark.parametrize("sizes", [(16, 16, 32, 32), (13, 17, 29, 23), (40, 31, 17, 12), (9, 9, 9, 9),
                                   (7, 30, 50, 4), (1, 5, 3, 11)])
def test_torch_nearest_pins(sizes):
    """Nearest neighbour: pixel-centre map == torch 'nearest-exact', the
    paper's printed map == torch 'nearest' (both FP64, exact copies)."""
    in_h, in_w, out_h, out_w = sizes
    img = fields.normal_f32((in_h, in_w), seed=23).astype(np.float64)
    t = torch.from_numpy(img)[None, None]
    exact = F.interpolate(t, size=(out_h, out_w), mode="nearest-exact")[0, 0].numpy()
    legacy = F.interpolate(t, size=(out_h, out_w), mode="nearest")[0, 0].numpy()
    np.testing.assert_array_equal(R.resize(img, out_h, out_w, R.NEAREST)[0, :, :, 0], exact)
    np.testing.assert_array_equal(
        R.resize(img, out_h, out_w, R.NEAREST, mapping=R.CORNER)[0, :, :, 0], legacy)


@pytest.mark.parametrize("n", [1, 2, 7, 16])
def test_corner_mapping_x2_closed_form(n):
    """Eq. 1 as printed at x2: s = x / 2, so even outputs copy source pixel
    x / 2 (t = 0) and odd outputs sit halfway (t = 1/2): bilinear averages
    the two neighbours, Keys a = -1/2 weighs four by (-1, 9, 9, -1) / 16,
    taps clamped to the image."""
    row = fields.uniform_u8((1, n), seed=n).astype(np.float64)[0]
    img = np.tile(row, (3, 1))  # constant columns: only the x axis matters

    def px(i):
        return row[min(max(i, 0), n - 1)]

    bil = R.resize(img, 3, 2 * n, R.BILINEAR, mapping=R.CORNER)[0, 1, :, 0]
    bic = R.resize(img, 3, 2 * n, R.BICUBIC, mapping=R.CORNER)[0, 1, :, 0]
    for x in range(2 * n):
        m = x // 2
        if x % 2 == 0:
            assert bil[x] == row[m] and bic[x] == row[m]
        else:
            assert bil[x] == (px(m) + px(m + 1)) / 2
            assert abs(bic[x] - (-px(m - 1) + 9 * px(m) + 9 * px(m + 1) - px(m + 2)) / 16) < 1e-12


@pytest.mark.parametrize("sizes", [(8, 8, 20, 20), (9, 7, 5, 13), (6, 6, 6, 6)])
def test_paper_eq5_with_printed_map(sizes):
    """Eqs. 1-5 evaluated as the paper writes them, pixel by pixel: x_p = x_f /
    scale, P1 = (int x_p, int y_p), P2 its right, P3 its lower and P4 its
    lower-right neighbour (clamped to the image), offsets the fractional
    parts, and eq. 5 with (1 - offsetX) on P1 and P3."""
    in_h, in_w, out_h, out_w = sizes
    img = fields.uniform_u8((in_h, in_w), seed=in_h * 7 + in_w).astype(np.float64)
    got = R.resize(img, out_h, out_w, R.BILINEAR, mapping=R.CORNER)[0, :, :, 0]
    for yf in range(out_h):
        for xf in range(out_w):
            xp, yp = Fraction(xf * in_w, out_w), Fraction(yf * in_h, out_h)
            x1, y1 = int(xp), int(yp)
            ox, oy = xp - x1, yp - y1
            x2, y2 = min(x1 + 1, in_w - 1), min(y1 + 1, in_h - 1)
            p1, p2, p3, p4 = (Fraction(int(img[y1, x1])), Fraction(int(img[y1, x2])),
                              Fraction(int(img[y2, x1])), Fraction(int(img[y2, x2])))
            want = (1 - oy) * ((1 - ox) * p1 + ox * p2) + oy * ((1 - ox) * p3 + ox * p4)
            assert abs(got[yf, xf] - float(want)) < 1e-12, (yf, xf)


def test_pil_bicubic_interior():
    Image = pytest.importorskip("PIL.Image")
    for in_h, in_w, out_h, out_w in [(16, 16, 32, 32), (21, 13, 50, 37)]:
        img = fields.field_u8(in_h, in_w, 1, seed=31)[:, :, 0].astype(np.float32)
        pil = Image.fromarray(img, mode="F").resize((out_w, out_h), resample=Image.BICUBIC)
        want = np.asarray(pil, dtype=np.float64)
        got = R.resize(img, out_h, out_w, R.BICUBIC)[0, :, :, 0]
        sy, my = _interior(in_h, out_h, 1, 1)
        sx, mx = _interior(in_w, out_w, 1, 1)
        # all four taps inside the image on both axes (PIL renormalises at edges)
        my &= (np.floor(sy) - 1 >= 0) & (np.floor(sy) + 2 <= in_h - 1)
        mx &= (np.floor(sx) - 1 >= 0) & (np.floor(sx) + 2 <= in_w - 1)
        m = my[:, None] & mx[None, :]
        assert m.sum() > 0
        # PIL keeps its intermediate rows in float32
        np.testing.assert_allclose(got[m], want[m], rtol=0, atol=2e-4)


@pytest.mark.parametrize("filt", [R.BILINEAR_AA, R.BICUBIC_AA])
@pytest.mark.parametrize("sizes", [(64, 64, 32, 32), (50, 37, 13, 20), (40, 90, 17, 11), (33, 33, 33, 33),
                                   (16, 12, 40, 30), (9, 300, 5, 19)])
def test_pil_antialiased_pin(filt, sizes):
    """PIL's float-mode resize stretches its filters by the shrink factor and
    renormalises the taps it keeps at the edges: the whole image, edges
    included, must match (PIL keeps its intermediate rows in float32)."""
    Image = pytest.importorskip("PIL.Image")
    in_h, in_w, out_h, out_w = sizes
    img = fields.field_u8(in_h, in_w, 1, seed=in_h + in_w)[:, :, 0].astype(np.float32)
    pil_filter = Image.BILINEAR if filt == R.BILINEAR_AA else Image.BICUBIC
    want = np.asarray(Image.fromarray(img, mode="F").resize((out_w, out_h), resample=pil_filter),
                      dtype=np.float64)
    got = R.resize_antialiased(img, out_h, out_w, filt)[0, :, :, 0]
    np.testing.assert_allclose(got, want, rtol=0, atol=3e-4)


def test_antialiased_closed_form_bilinear_half():
    """x0.5 bilinear, antialiased: s = 2x + 1/2, sigma = 2, taps 2x-1 .. 2x+2
    at distances (-3/4, -1/4, 1/4, 3/4), weights (1, 3, 3, 1) / 8."""
    idx, w = R.axis_taps_antialiased(16, 8, R.BILINEAR_AA)
    for x in range(1, 7):
        assert idx[x].tolist() == [2 * x - 1, 2 * x, 2 * x + 1, 2 * x + 2]
        np.testing.assert_allclose(w[x], np.array([1, 3, 3, 1]) / 8, rtol=0, atol=1e-15)
    # at the left edge tap -1 is dropped and the rest renormalised: (3, 3, 1) / 7
    assert idx[0].tolist()[:3] == [0, 1, 2]
    np.testing.assert_allclose(w[0][:3], np.array([3, 3, 1]) / 7, rtol=0, atol=1e-15)


@pytest.mark.parametrize("filt, plain", [(R.BILINEAR_AA, R.BILINEAR), (R.BICUBIC_AA, R.BICUBIC)])
def test_antialiased_upscale_interior_is_plain(filt, plain):
    """sigma = 1 when growing: away from the edges every tap is inside the
    image, the weights already sum to one, and the plain filter results."""
    img = fields.uniform_u8((21, 17), seed=5).astype(np.float64)
    got = R.resize_antialiased(img, 50, 41, filt)[0, :, :, 0]
    want = R.resize(img, 50, 41, plain)[0, :, :, 0]
    sy, my = _interior(21, 50, 1, 1)
    sx, mx = _interior(17, 41, 1, 1)
    r = 2 if plain == R.BICUBIC else 1
    my &= (np.floor(sy) - (r - 1) >= 0) & (np.floor(sy) + r <= 20)
    mx &= (np.floor(sx) - (r - 1) >= 0) & (np.floor(sx) + r <= 16)
    m = my[:, None] & mx[None, :]
    assert m.sum() > 0
    np.testing.assert_allclose(got[m], want[m], rtol=0, atol=1e-12)


@pytest.mark.parametrize("filt", [R.BILINEAR_AA, R.BICUBIC_AA])
def test_antialiased_constant_and_sum(filt):
    for n_in, n_out in [(100, 7), (37, 29), (5, 9), (64, 1)]:
        _, w = R.axis_taps_antialiased(n_in, n_out, filt)
        np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    img = np.full((30, 40), 77.0)
    np.testing.assert_allclose(R.resize_antialiased(img, 7, 9, filt), 77.0, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
def test_adjoint_finite_differences(filt):
    full = fields.normal_f32((64, 64), seed=1004).astype(np.float64)
    crop = full[20:36, 8:24]  # 16 x 16 x 1 crop, treated as a standalone image
    out_h, out_w = 32, 32
    n = crop.size
    base = R.resize(crop, out_h, out_w, filt).ravel()
    jac = np.empty((base.size, n))
    h = 1.0  # the map is linear, so central differences are exact up to rounding
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        plus = R.resize(crop + e.reshape(crop.shape), out_h, out_w, filt).ravel()
        minus = R.resize(crop - e.reshape(crop.shape), out_h, out_w, filt).ravel()
        jac[:, k] = (plus - minus) / (2 * h)
    g = fields.normal_f32((out_h, out_w), seed=1005).astype(np.float64)
    want = (jac.T @ g.ravel()).reshape(crop.shape)
    np.testing.assert_allclose(R.adjoint(g, 16, 16, filt)[0, :, :, 0], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ref_c.adjoint(g.astype(np.float32), 16, 16, filt)[0, :, :, 0],
                               (jac.T @ g.astype(np.float32).astype(np.float64).ravel()).reshape(16, 16),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
def test_adjoint_identity_and_mass(filt):
    x = fields.normal_f32((3, 37, 45, 1), seed=41).astype(np.float64)
    y = fields.normal_f32((3, 70, 29, 1), seed=42).astype(np.float64)
    ax = R.resize(x, 70, 29, filt)
    aty = R.adjoint(y, 37, 45, filt)
    lhs, rhs = float(np.dot(ax.ravel(), y.ravel())), float(np.dot(x.ravel(), aty.ravel()))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    np.testing.assert_allclose(aty.sum(axis=(1, 2, 3)), y.sum(axis=(1, 2, 3)), rtol=1e-12)


def test_adjoint_constant_upstream_x2():
    g = np.ones((1, 32, 32, 1))
    gs = R.adjoint(g, 16, 16, R.BILINEAR)[0, :, :, 0]
    np.testing.assert_array_equal(gs[1:-1, 1:-1], 4.0)
    assert gs.sum() == 32 * 32


# ---------------------------------------------------------------------------
# storage rounding
# ---------------------------------------------------------------------------

def test_u8_rounding_half_even_and_clamp():
    v = np.array([0.5, 1.5, 2.5, 3.49999, 254.5, 255.5, -0.5, -3.0, 300.0, 127.5, 128.5])
    np.testing.assert_array_equal(R.quantize_u8(v), [0, 2, 2, 3, 254, 255, 0, 0, 255, 128, 128])


def test_f16_rounding_is_direct_from_f64():
    one = 1.0
    # 1 + 2^-11 + 2^-40 is above the midpoint of [1, 1 + 2^-10]: direct RNE gives 1 + 2^-10,
    # a detour through float32 would round to the midpoint first and then to 1.
    v = np.array([one + 2.0 ** -11 + 2.0 ** -40, one + 2.0 ** -11, one + 3 * 2.0 ** -11])
    got = R.quantize_f16(v).astype(np.float64)
    np.testing.assert_array_equal(got, [one + 2.0 ** -10, one, one + 2 * 2.0 ** -10])


# ---------------------------------------------------------------------------
# the two oracle implementations agree, and band helpers are consistent
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32])
def test_c_oracle_matches_numpy(filt, dtype):
    if dtype == np.uint8:
        img = fields.uniform_u8((2, 33, 47, 4), seed=51)
    else:
        img = fields.normal_f32((2, 33, 47, 4), seed=52).astype(dtype)
    rows = np.array([0, 1, 17, 40, 58, 59])
    want = R.resize_rows(img, 60, 23, rows, filt)
    got = ref_c.resize_rows(img, 60, 23, rows, filt, threads=2)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_needed_rows_cover_band():
    for filt in (R.BILINEAR, R.BICUBIC):
        lo, hi = R.needed_rows(16, 32, 0, 32, filt)
        assert (lo, hi) == (0, 15)
    # rows 8..15 of a 16 -> 32 resize: s = 3.75 .. 7.25, so y0 = 3 .. 7
    assert R.needed_rows(16, 32, 8, 8, R.BICUBIC) == (2, 9)
    assert R.needed_rows(16, 32, 8, 8, R.BILINEAR) == (3, 8)


# ---------------------------------------------------------------------------
# mutation check: the brute-force pin must catch plausible oracle mistakes
# ---------------------------------------------------------------------------

def _mutant_taps(kind):
    orig = R.axis_taps

    def taps(n_in, n_out, filt, a=R.KEYS_A, mapping=R.HALF_PIXEL):
        idx, w, x0, t = orig(n_in, n_out, filt, a, mapping)
        idx, w = idx.copy(), w.copy()
        if kind == "trunc":          # int() read as truncation toward zero
            s = R.source_coordinate(np.arange(n_out), n_in, n_out)
            x0 = np.trunc(s).astype(np.int64)
            t = s - x0
            offs = np.arange(w.shape[1]) - (1 if filt == R.BICUBIC else 0)
            idx = np.clip(x0[:, None] + offs[None, :], 0, n_in - 1)
            w = (np.stack([1 - t, t], 1) if filt == R.BILINEAR
                 else R.keys_kernel(t[:, None] - offs[None, :], a))
        elif kind == "swap_weights":  # weights attached to the wrong taps
            w = w[:, ::-1]
        elif kind == "no_clamp":      # wrap instead of replicate
            idx = np.mod(x0[:, None] + (np.arange(w.shape[1]) - (1 if filt == R.BICUBIC else 0)), n_in)
        elif kind == "drop_tap":      # a dropped term
            w[:, -1] = 0.0
        elif kind == "corner_aligned":  # eq. 1 as printed, without half-pixel centres
            s = np.arange(n_out) * (n_in / n_out)
            x0 = np.floor(s).astype(np.int64)
            t = s - x0
            offs = np.arange(w.shape[1]) - (1 if filt == R.BICUBIC else 0)
            idx = np.clip(x0[:, None] + offs[None, :], 0, n_in - 1)
            w = (np.stack([1 - t, t], 1) if filt == R.BILINEAR
                 else R.keys_kernel(t[:, None] - offs[None, :], a))
        return idx, w, x0, t

    return taps


@pytest.mark.parametrize("kind", ["trunc", "swap_weights", "no_clamp", "drop_tap", "corner_aligned"])
def test_pins_catch_planted_mistakes(kind, monkeypatch):
    img = fields.uniform_u8((8, 8), seed=77)
    caught = False
    for filt in (R.BILINEAR, R.BICUBIC):
        for shape in [(8, 8, 16, 16), (8, 8, 13, 11), (8, 6, 3, 17)]:
            in_h, in_w, out_h, out_w = shape
            exact = np.array([[float(v) for v in row]
                              for row in _brute_resize(img[:in_h, :in_w].tolist(), out_h, out_w, filt)])
            with monkeypatch.context() as m:
                m.setattr(R, "axis_taps", _mutant_taps(kind))
                got = R.resize(img[:in_h, :in_w], out_h, out_w, filt)[0, :, :, 0]
            if np.abs(got - exact).max() > 1e-9:
                caught = True
    assert caught, f"planted mistake {kind!r} went unnoticed"


def test_pins_catch_transposed_axes():
    # using the row taps on columns (and vice versa) must be visible on a non-square case
    img = fields.uniform_u8((7, 9), seed=78)
    exact = np.array([[float(v) for v in row] for row in _brute_resize(img.tolist(), 5, 20, R.BICUBIC)])
    iy, wy, _, _ = R.axis_taps(9, 5, R.BICUBIC)   # swapped n_in between axes
    ix, wx, _, _ = R.axis_taps(7, 20, R.BICUBIC)
    src = img.astype(np.float64)
    got = np.zeros((5, 20))
    for j in range(4):
        for i in range(4):
            got += (wy[:, j][:, None] * wx[:, i][None, :]) * src[np.clip(iy[:, j], 0, 6)][:, np.clip(ix[:, i], 0, 8)]
    assert np.abs(got - exact).max() > 1e-6


# ---------------------------------------------------------------------------
# the exact single-value evaluator (oracle/exact.py) and the error scale
# (absolute=True) of the float64 oracle
# ---------------------------------------------------------------------------

from oracle import exact as EX  # noqa: E402


def _abs_brute(img2d, out_h, out_w, filt, a=Fraction(-1, 2)):
    """sum over every integer sample position i, j of |K(s_y - i)| |K(s_x - j)|
    |v[clamp(i)][clamp(j)]| (all-taps form, no tap selection, exact): the
    float32 rounding-error scale of a tap-by-tap evaluation, including the
    clamped duplicate taps at the edges, which are not merged."""
    in_h, in_w = len(img2d), len(img2d[0])

    def taps(x, n_in, n_out):
        s = Fraction((2 * x + 1) * n_in - n_out, 2 * n_out)
        lo = int(s) - 6
        return [(min(max(i, 0), n_in - 1), abs(_kernel_exact(s - i, filt, a))) for i in range(lo, lo + 13)
                if _kernel_exact(s - i, filt, a) != 0]

    out = []
    for y in range(out_h):
        row = []
        for x in range(out_w):
            v = Fraction(0)
            for r, wy in taps(y, in_h, out_h):
                for c, wx in taps(x, in_w, out_w):
                    v += wy * wx * abs(Fraction(float(img2d[r][c])))
            row.append(v)
        out.append(row)
    return out


def _signed_img(h, w, seed):
    """Signed samples that are exact in float64 (multiples of 1/8)."""
    rng = np.random.default_rng(seed)
    return np.round(rng.normal(0.0, 4.0, (h, w)) * 8) / 8


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("shape", SHAPES)
def test_exact_values_match_brute_force(shape, filt):
    in_h, in_w, out_h, out_w = shape
    img = fields.uniform_u8((in_h, in_w), seed=in_h * 31 + in_w)
    want = _brute_resize(img.tolist(), out_h, out_w, filt)
    planes = img[None, :, :, None]
    for y in range(out_h):
        for x in range(out_w):
            assert EX.value(planes, out_h, out_w, filt, 0, y, x, 0) == want[y][x]


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("shape", SHAPES[2:6])
def test_exact_values_match_brute_force_corner_map(shape, filt):
    in_h, in_w, out_h, out_w = shape
    img = fields.uniform_u8((in_h, in_w), seed=in_h * 37 + in_w)
    want = _brute_resize(img.tolist(), out_h, out_w, filt, corner=True)
    planes = img[None, :, :, None]
    for y in range(out_h):
        for x in range(out_w):
            assert EX.value(planes, out_h, out_w, filt, 0, y, x, 0, mapping=EX.CORNER) == want[y][x]


@pytest.mark.parametrize("filt", [R.BILINEAR_AA, R.BICUBIC_AA])
@pytest.mark.parametrize("sizes", [(20, 17, 7, 5), (9, 12, 13, 4), (16, 16, 4, 4)])
def test_exact_antialiased_values(filt, sizes):
    """Exact antialiased values: against a brute force over every source
    index of the image (weight K((i - s) / sigma) when |i - s| < R sigma,
    then divided by the sum), and against the float64 oracle."""
    in_h, in_w, out_h, out_w = sizes
    img = fields.uniform_u8((in_h, in_w), seed=in_h + 5 * in_w)
    r = 1 if filt == R.BILINEAR_AA else 2
    base = R.BILINEAR if filt == R.BILINEAR_AA else R.BICUBIC

    def weights(x, n_in, n_out):
        s = Fraction((2 * x + 1) * n_in - n_out, 2 * n_out)
        sig = max(Fraction(n_in, n_out), Fraction(1))
        ws = [(i, _kernel_exact((i - s) / sig, base, Fraction(-1, 2))) for i in range(n_in)
              if abs(i - s) < r * sig]
        tot = sum(w for _, w in ws)
        return [(i, w / tot) for i, w in ws]

    planes = img[None, :, :, None]
    f64 = R.resize_antialiased(planes, out_h, out_w, filt)[0, :, :, 0]
    for y in range(out_h):
        wy = weights(y, in_h, out_h)
        for x in range(out_w):
            wx = weights(x, in_w, out_w)
            want = sum(a * b * int(img[i, j]) for i, a in wy for j, b in wx)
            got = EX.value(planes, out_h, out_w, filt, 0, y, x, 0)
            assert got == want
            assert abs(float(got) - f64[y, x]) <= 1e-12 * max(1.0, abs(f64[y, x]))


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("shape", SHAPES)
def test_absolute_scale_pin(shape, filt):
    """resize_rows(absolute=True) and exact.abs_scale against the all-taps
    brute force over |w_y| |w_x| |v| on signed data (negative Keys lobes and
    negative samples make any dropped absolute value visible)."""
    in_h, in_w, out_h, out_w = shape
    img = _signed_img(in_h, in_w, seed=in_h * 7 + in_w)
    want = _abs_brute(img.tolist(), out_h, out_w, filt)
    planes = img[None, :, :, None]
    got = R.resize_rows(planes, out_h, out_w, np.arange(out_h), filt, absolute=True)[0, :, :, 0]
    plain = R.resize_rows(planes, out_h, out_w, np.arange(out_h), filt)[0, :, :, 0]
    for y in range(out_h):
        for x in range(out_w):
            w = float(want[y][x])
            assert abs(got[y, x] - w) <= 1e-13 * max(1.0, w)
            assert EX.abs_scale(planes, out_h, out_w, filt, 0, y, x, 0) == want[y][x]
            assert abs(plain[y, x]) <= got[y, x] * (1 + 1e-13) + 1e-300


@pytest.mark.parametrize("filt", [R.BILINEAR_AA, R.BICUBIC_AA])
def test_absolute_scale_pin_antialiased(filt):
    in_h, in_w, out_h, out_w = 19, 23, 6, 9
    img = _signed_img(in_h, in_w, seed=11)
    planes = img[None, :, :, None]
    got = R.resize_antialiased(planes, out_h, out_w, filt, absolute=True)[0, :, :, 0]
    for y in range(out_h):
        ty = EX.axis_taps(y, in_h, out_h, filt)
        for x in range(out_w):
            tx = EX.axis_taps(x, in_w, out_w, filt)
            want = sum(abs(a) * abs(b) * abs(Fraction(float(img[i, j]))) for i, a in ty for j, b in tx)
            assert abs(got[y, x] - float(want)) <= 1e-12 * float(want)
            assert EX.abs_scale(planes, out_h, out_w, filt, 0, y, x, 0) == want


@pytest.mark.parametrize("filt", [R.BILINEAR, R.BICUBIC])
@pytest.mark.parametrize("shape", SHAPES[:5])
def test_absolute_scale_pin_adjoint(shape, filt):
    """adjoint(absolute=True) against a brute force that scatters
    |K(s_y - i)| |K(s_x - j)| |g| from every output onto clamp(i), clamp(j)."""
    in_h, in_w, out_h, out_w = shape
    g = _signed_img(out_h, out_w, seed=out_h * 5 + out_w)
    a = Fraction(-1, 2)
    gs = [[Fraction(0)] * in_w for _ in range(in_h)]
    for y in range(out_h):
        sy = Fraction((2 * y + 1) * in_h - out_h, 2 * out_h)
        for x in range(out_w):
            sx = Fraction((2 * x + 1) * in_w - out_w, 2 * out_w)
            gv = abs(Fraction(float(g[y, x])))
            for i in range(int(sy) - 6, int(sy) + 7):
                wy = abs(_kernel_exact(sy - i, filt, a))
                if not wy:
                    continue
                for j in range(int(sx) - 6, int(sx) + 7):
                    wx = abs(_kernel_exact(sx - j, filt, a))
                    if wx:
                        gs[min(max(i, 0), in_h - 1)][min(max(j, 0), in_w - 1)] += wy * wx * gv
    got = R.adjoint(g[None, :, :, None], in_h, in_w, filt, absolute=True)[0, :, :, 0]
    for r in range(in_h):
        for c in range(in_w):
            w = float(gs[r][c])
            assert abs(got[r, c] - w) <= 1e-13 * max(1.0, w)
