"""GPU parity of the adjoint (xr_resize_backward) and of the autograd wrapper.

* small shapes of every filter and channel count (exact x2 with its border
  pass, other upscales, shrinking, identity, one-row and one-column sources)
  against the FP64 oracle adjoint, within 1e-5 * sum |w_y w_x g| per pixel;
* the finite-difference Jacobian of the oracle forward on a 16 x 16 x 1 crop;
* the 32 x 3 x 1024^2 -> 2048^2 float32 workload: forward rows, adjoint
  planes, the adjoint identity <Ax, y> = <x, A^T y> and mass conservation;
* float16 gradients (float32 sums, one rounding) on the same shapes, equal bit
  for bit to the float32 result rounded to float16 wherever both run the
  owner-computes kernel, and repeat runs bitwise identical (fixed order).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1001_1718_amd as xr  # noqa: E402
from gpu_util import check_f16_sum, check_f32, compare  # noqa: E402
from oracle import ref_c  # noqa: E402
from oracle import ref_resize as R  # noqa: E402
from synth import fields  # noqa: E402

DEV = "cuda:0"
MODES = {"bilinear": 0, "bicubic": 1}


def _adjoint_gpu(g_nchw: np.ndarray, in_h: int, in_w: int, mode: str) -> np.ndarray:
    gs = xr.resize_backward(torch.from_numpy(g_nchw).to(DEV), (in_h, in_w), mode)
    torch.cuda.synchronize()
    return gs.cpu().numpy()


SHAPES = [
    ((37, 53), (74, 106)),   # x2 up, ragged
    ((20, 300), (90, 610)),  # several tiles in both directions
    ((37, 53), (61, 29)),    # mixed: shrink along x
    ((64, 96), (32, 48)),    # x0.5
    ((33, 21), (33, 21)),    # identity
    ((1, 5), (40, 7)),       # one source row, strong vertical upscale (narrow tiles)
    ((300, 280), (21, 17)),  # strong shrink: source pixels that no output touches
    ((40, 700), (311, 1400)),  # several column tiles, non-dyadic rows
    ((1, 6), (2, 12)),       # x2 with a single source row (border pass only)
    ((5, 1), (10, 2)),       # x2 with a single source column
    ((2, 2), (4, 4)),        # x2, every pixel on the border
    ((48, 2050), (96, 4100)),  # x2, ragged last column block, several strips
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0][0]}x{s[0][1]}-{s[1][0]}x{s[1][1]}")
@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_adjoint_small_nchw(shape, mode):
    (in_h, in_w), (out_h, out_w) = shape
    g = fields.normal_f32((2, 3, out_h, out_w), seed=out_h * 31 + out_w)
    got = _adjoint_gpu(g, in_h, in_w, mode)
    planes = g.reshape(6, out_h, out_w, 1)
    ref = R.adjoint(planes, in_h, in_w, MODES[mode]).reshape(2, 3, in_h, in_w)
    scale = R.adjoint(planes, in_h, in_w, MODES[mode], absolute=True).reshape(2, 3, in_h, in_w)
    check_f32(got, ref, scale, what=f"adjoint {shape} {mode}")


@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_adjoint_rgba_interleaved(mode):
    g = fields.normal_f32((2, 66, 90, 4), seed=9)
    gs = xr.resize_backward(torch.from_numpy(g).to(DEV), (33, 45), mode, layout="hwc")
    torch.cuda.synchronize()
    ref = R.adjoint(g, 33, 45, MODES[mode])
    scale = R.adjoint(g, 33, 45, MODES[mode], absolute=True)
    check_f32(gs.cpu().numpy(), ref, scale, what=f"adjoint rgba {mode}")


@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_adjoint_matches_finite_differences(mode):
    full = fields.normal_f32((64, 64), seed=1004).astype(np.float64)
    crop = full[20:36, 8:24]
    n = crop.size
    jac = np.empty((32 * 32, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        plus = R.resize(crop + e.reshape(16, 16), 32, 32, MODES[mode]).ravel()
        minus = R.resize(crop - e.reshape(16, 16), 32, 32, MODES[mode]).ravel()
        jac[:, k] = (plus - minus) / 2.0
    g = fields.normal_f32((1, 1, 32, 32), seed=1005)
    want = (jac.T @ g.astype(np.float64).ravel()).reshape(16, 16)
    got = _adjoint_gpu(g, 16, 16, mode)[0, 0]
    scale = (np.abs(jac).T @ np.abs(g.astype(np.float64)).ravel()).reshape(16, 16)
    check_f32(got, want, scale, what="finite differences")


def test_autograd_function():
    x = torch.from_numpy(fields.normal_f32((2, 3, 24, 40), seed=6)).to(DEV).requires_grad_(True)
    y = xr.ResizeFn.apply(x, (48, 80), "bilinear")
    g = torch.from_numpy(fields.normal_f32((2, 3, 48, 80), seed=8)).to(DEV)
    y.backward(g)
    torch.cuda.synchronize()
    gp = g.cpu().numpy().reshape(6, 48, 80, 1)
    ref = R.adjoint(gp, 24, 40, 0).reshape(2, 3, 24, 40)
    scale = R.adjoint(gp, 24, 40, 0, absolute=True).reshape(2, 3, 24, 40)
    check_f32(x.grad.cpu().numpy(), ref, scale, what="autograd")
    fwd = R.resize(x.detach().cpu().numpy().reshape(6, 24, 40, 1), 48, 80, 0).reshape(2, 3, 48, 80)
    fscale = R.resize_rows(x.detach().cpu().numpy().reshape(6, 24, 40, 1), 48, 80, np.arange(48), 0,
                           absolute=True).reshape(2, 3, 48, 80)
    check_f32(y.detach().cpu().numpy(), fwd, fscale, what="autograd forward")


def test_c4_full_size():
    """32x3x1024^2 -> 2048^2 bilinear, float32 NCHW: forward + adjoint."""
    x_np = fields.normal_f32((32, 3, 1024, 1024), seed=1004)
    g_np = fields.normal_f32((32, 3, 2048, 2048), seed=1005)
    x = torch.from_numpy(x_np).to(DEV)
    g = torch.from_numpy(g_np).to(DEV)
    y = xr.resize(x, (2048, 2048), "bilinear", layout="nchw")
    gs = xr.resize_backward(g, (1024, 1024), "bilinear")
    torch.cuda.synchronize()

    # forward: sampled rows of sampled planes
    rng = np.random.default_rng(4)
    rows = np.unique(np.concatenate([[0, 1, 2047], rng.integers(0, 2048, 12)]))
    for p in [0, 47, 95]:
        n, c = divmod(p, 3)
        got = y[n, c][torch.from_numpy(rows).to(DEV)].cpu().numpy()
        compare(got[None, :, :, None], x_np[n, c][None, :, :, None], 2048, 2048, 0, rows=rows,
                what=f"C4 forward plane {p}")

    # adjoint: whole planes against the C oracle
    for p in [0, 95]:
        n, c = divmod(p, 3)
        gp = g_np[n, c][None, :, :, None]
        ref = ref_c.adjoint(gp, 1024, 1024, 0)[0, :, :, 0]
        scale = R.adjoint(gp, 1024, 1024, 0, absolute=True)[0, :, :, 0]
        check_f32(gs[n, c].cpu().numpy(), ref, scale, what=f"C4 adjoint plane {p}")

    # adjoint identity <Ax, y> = <x, A^T y> over the whole tensor, float64 dots
    lhs = torch.sum(y.double() * g.double()).item()
    rhs = torch.sum(x.double() * gs.double()).item()
    assert abs(lhs - rhs) <= 1e-6 * max(1.0, abs(lhs)), (lhs, rhs)
    # mass conservation per plane: sum grad_src = sum grad_dst
    np.testing.assert_allclose(gs.double().sum(dim=(2, 3)).cpu().numpy(),
                               g.double().sum(dim=(2, 3)).cpu().numpy(), rtol=1e-5, atol=1e-2)


def test_adjoint_overwrites_output():
    g = torch.from_numpy(fields.normal_f32((1, 1, 80, 64), seed=2)).to(DEV)
    out = torch.full((1, 1, 40, 32), 123.0, device=DEV)
    xr.resize_backward(g, (40, 32), "bicubic", out=out)
    first = out.clone()
    xr.resize_backward(g, (40, 32), "bicubic", out=out)
    torch.cuda.synchronize()
    ref = R.adjoint(g.cpu().numpy().reshape(1, 80, 64, 1), 40, 32, 1)[0, :, :, 0]
    scale = R.adjoint(g.cpu().numpy().reshape(1, 80, 64, 1), 40, 32, 1, absolute=True)[0, :, :, 0]
    check_f32(first[0, 0].cpu().numpy(), ref, scale, what="first call")
    check_f32(out[0, 0].cpu().numpy(), ref, scale, what="second call")


def test_adjoint_rejects_extreme_upscale():
    g = torch.zeros((1, 1, 30000, 4), device=DEV)
    with pytest.raises(xr.XResizeError) as e:
        xr.resize_backward(g, (1, 4), "bicubic")
    assert e.value.code == 2


def _is_up2(shape):
    (in_h, in_w), (out_h, out_w) = shape
    return out_h == 2 * in_h and out_w == 2 * in_w


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0][0]}x{s[0][1]}-{s[1][0]}x{s[1][1]}")
@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_adjoint_float16(shape, mode):
    (in_h, in_w), (out_h, out_w) = shape
    g16 = fields.normal_f32((2, 3, out_h, out_w), seed=out_h * 17 + out_w).astype(np.float16)
    gd = torch.from_numpy(g16).to(DEV)
    got = xr.resize_backward(gd, (in_h, in_w), mode)
    assert got.dtype == torch.float16
    again = xr.resize_backward(gd, (in_h, in_w), mode)
    torch.cuda.synchronize()
    got_np = got.cpu().numpy()
    np.testing.assert_array_equal(again.cpu().numpy().view(np.uint16), got_np.view(np.uint16))
    planes = g16.astype(np.float64).reshape(6, out_h, out_w, 1)
    ref = R.adjoint(planes, in_h, in_w, MODES[mode]).reshape(2, 3, in_h, in_w)
    scale = R.adjoint(planes, in_h, in_w, MODES[mode], absolute=True).reshape(2, 3, in_h, in_w)
    check_f16_sum(got_np, ref, scale, what=f"adjoint f16 {shape} {mode}")
    if not _is_up2(shape):  # same kernel and order in float32: one rounding apart
        f32 = xr.resize_backward(gd.float(), (in_h, in_w), mode)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(f32.cpu().numpy().astype(np.float16).view(np.uint16),
                                      got_np.view(np.uint16))


@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_adjoint_float16_rgba_and_autograd(mode):
    g16 = fields.normal_f32((2, 50, 70, 4), seed=21).astype(np.float16)
    gs = xr.resize_backward(torch.from_numpy(g16).to(DEV), (33, 45), mode, layout="hwc")
    torch.cuda.synchronize()
    ref = R.adjoint(g16.astype(np.float64), 33, 45, MODES[mode])
    scale = R.adjoint(g16.astype(np.float64), 33, 45, MODES[mode], absolute=True)
    check_f16_sum(gs.cpu().numpy(), ref, scale, what=f"adjoint f16 rgba {mode}")
    x = torch.from_numpy(fields.field_unit(24, 40, 3, seed=5, dtype=np.float16).transpose(2, 0, 1)[None].copy())
    x = x.to(DEV).requires_grad_(True)
    y = xr.ResizeFn.apply(x, (61, 29), mode)
    g = torch.from_numpy(fields.normal_f32((1, 3, 61, 29), seed=8).astype(np.float16)).to(DEV)
    y.backward(g)
    torch.cuda.synchronize()
    assert x.grad.dtype == torch.float16
    gp = g.cpu().numpy().astype(np.float64).reshape(3, 61, 29, 1)
    ref = R.adjoint(gp, 24, 40, MODES[mode]).reshape(1, 3, 24, 40)
    scale = R.adjoint(gp, 24, 40, MODES[mode], absolute=True).reshape(1, 3, 24, 40)
    check_f16_sum(x.grad.cpu().numpy(), ref, scale, what=f"autograd f16 {mode}")


def test_adjoint_owner_is_deterministic_at_size():
    """Non-x2 float32 adjoint over many tiles: two runs bitwise equal, and a
    slice of the batch gives the same bits as the whole tensor."""
    g = torch.from_numpy(fields.normal_f32((4, 3, 1500, 1100), seed=12)).to(DEV)
    a = xr.resize_backward(g, (1024, 800), "bicubic")
    b = xr.resize_backward(g, (1024, 800), "bicubic")
    part = xr.resize_backward(g[1:3].contiguous(), (1024, 800), "bicubic")
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a[1:3], part)
    p = g[2, 1].cpu().numpy()[None, :, :, None]
    ref = ref_c.adjoint(p, 1024, 800, 1)[0, :, :, 0]
    scale = R.adjoint(p, 1024, 800, 1, absolute=True)[0, :, :, 0]
    check_f32(a[2, 1].cpu().numpy(), ref, scale, what="owner adjoint at size")


def test_adjoint_rejects_mixed_dtypes():
    g = torch.zeros((1, 1, 8, 8), device=DEV, dtype=torch.float16)
    out = torch.empty((1, 1, 4, 4), device=DEV, dtype=torch.float32)
    with pytest.raises(xr.XResizeError) as e:
        xr.resize_backward(g, (4, 4), "bilinear", out=out)
    assert e.value.code == 3
    with pytest.raises(xr.XResizeError) as e:
        xr.resize_backward(torch.zeros((1, 1, 8, 8), device=DEV, dtype=torch.uint8), (4, 4), "bilinear")
    assert e.value.code == 3
