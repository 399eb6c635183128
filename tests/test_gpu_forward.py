"""GPU parity of the forward resize against the FP64 oracle (through the C ABI).

Cases: the 512x512 -> 1024x1024 uint8 bilinear workload in full; every dtype x
channel count x filter x kernel on small ragged images (several tiles plus a
ragged tail, dyadic and non-dyadic ratios, shrinking, identity, 1-pixel
sides); bitwise equality of every launch shape; row bands; and the
4096x4096 RGBA bicubic x2 / x0.5 workload on sampled rows.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU only under -m gpu
    pytest.skip("no GPU", allow_module_level=True)

import paper_1001_1718_amd as xr  # noqa: E402
from gpu_util import compare  # noqa: E402
from synth import fields  # noqa: E402

DEV = "cuda:0"
MODES = {"bilinear": 0, "bicubic": 1, "nearest": 2, "bilinear_aa": 3, "bicubic_aa": 4}
R_MAP = {"half_pixel": 0, "paper": 1}

TILES = {
    "auto": None,
    "gather8x8": xr.tile(xr.XR_KERNEL_GATHER, 8, 8),
    "gather32x4": xr.tile(xr.XR_KERNEL_GATHER, 32, 4),
    "strip": xr.tile(xr.XR_KERNEL_STRIP, 64, 4, 0, 7),      # ppt_x filled per case
    "strip_any": xr.tile(xr.XR_KERNEL_STRIP_ANY, 128, 2, 0, 5),
    "strip_xcd": xr.tile(xr.XR_KERNEL_STRIP, 512, 1, 0, 9, 1),
    "strip_any_xcd": xr.tile(xr.XR_KERNEL_STRIP_ANY, 64, 2, 0, 3, 1),
    "strip_row1": xr.tile(xr.XR_KERNEL_STRIP, 64, 1, 0, 1),     # one output row per thread
    "strip_row2_xcd": xr.tile(xr.XR_KERNEL_STRIP, 128, 2, 0, 2, 1),
    "strip_lds": xr.tile(xr.XR_KERNEL_STRIP_LDS, 64, 1, 0, 7),
    "strip_lds_xcd": xr.tile(xr.XR_KERNEL_STRIP_LDS, 256, 1, 0, 3, 1),
}


def _tile_for(name, channels):
    t = TILES[name]
    if t is None or t.kernel == xr.XR_KERNEL_GATHER:
        return t
    t = xr.XrTile(*t.as_tuple())
    t.ppt_x = 4 if channels == 4 else 8
    return t


def _lds_stageable(t, in_w, out_w, mode, dtype, channels):
    """The staging rule of XR_KERNEL_STRIP_LDS: a workgroup's source segment
    of at most floor((cols - 1) * in_w / out_w) + K + 1 pixels, moved in
    chunks of max(pixel, 4) bytes, must need at most 64 / chunk chunks per
    lane and three row buffers of at most 64 KiB; pixels under 4 bytes need
    rows of whole 4-byte words."""
    pb = channels * np.dtype(dtype).itemsize
    cb = max(pb, 4)
    k = 4 if mode == "bicubic" else 2
    cols = min(t.block_w * t.ppt_x, out_w)
    seg = (cols - 1) * in_w // out_w + k + 1
    chunks = -(-(seg * pb + cb - pb) // cb)
    need = -(-chunks // t.block_w)
    return need <= 64 // cb and 3 * (-(-chunks * cb // 16) * 16) <= 65536 and (pb >= 4 or (in_w * pb) % 4 == 0)


def _input(dtype, h, w, c, seed):
    if dtype == np.uint8:
        return fields.uniform_u8((h, w, c), seed)
    if dtype == np.float16:
        return fields.field_unit(h, w, c, seed, np.float16)
    return fields.normal_f32((h, w, c), seed)


def _gpu(src_np, out_h, out_w, mode, tile=None):
    x = torch.from_numpy(src_np).to(DEV)
    y = xr.resize(x, (out_h, out_w), mode, tile=tile)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_c1_bilinear_x2_u8_full():
    img = fields.uniform_u8((512, 512), seed=1001)
    out = _gpu(img, 1024, 1024, "bilinear")
    res = compare(out, img, 1024, 1024, 0, what="C1")
    assert res["ties"] == 0 and res["non_ties"] == 0


SHAPES = [
    ((37, 53), (74, 106)),   # exact x2, ragged
    ((40, 32), (80, 64)),    # exact x2, aligned
    ((37, 53), (61, 29)),    # non-dyadic up / down
    ((64, 96), (32, 48)),    # exact x0.5
    ((74, 262), (37, 131)),  # exact x0.5, ragged, several strips
    ((2, 2), (1, 1)),        # exact x0.5, every tap clamped
    ((33, 21), (33, 21)),    # identity
    ((1, 5), (3, 7)),        # one-row source
    ((9, 1), (20, 2)),       # one-column source
    ((150, 70), (41, 263)),  # several tiles, mixed
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0][0]}x{s[0][1]}-{s[1][0]}x{s[1][1]}")
@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32], ids=["u8", "f16", "f32"])
@pytest.mark.parametrize("channels", [1, 4])
@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_small_all_kernels(shape, dtype, channels, mode):
    (in_h, in_w), (out_h, out_w) = shape
    img = _input(dtype, in_h, in_w, channels, seed=in_h * 1000 + in_w + channels)
    outs = {}
    for name in TILES:
        t = _tile_for(name, channels)
        if name.startswith("strip_lds") and not _lds_stageable(t, in_w, out_w, mode, dtype, channels):
            # refused (XR_ERR_ARG), never read past a row or the LDS budget
            with pytest.raises(xr.XResizeError) as e:
                _gpu(img, out_h, out_w, mode, t)
            assert e.value.code == 11
            continue
        outs[name] = _gpu(img, out_h, out_w, mode, t)
    compare(outs["auto"], img, out_h, out_w, MODES[mode], what=f"{shape} {mode}")
    for name, o in outs.items():
        np.testing.assert_array_equal(o.view(np.uint8), outs["auto"].view(np.uint8),
                                      err_msg=f"kernel {name} differs from the default")


MAP_SHAPES = [
    ((37, 53), (74, 106)),   # x2: the printed map gives t in {0, 1/2}
    ((37, 53), (61, 29)),    # non-dyadic up / down
    ((64, 96), (32, 48)),    # x0.5
    ((150, 70), (41, 263)),  # several tiles, mixed
    ((1, 5), (3, 7)),        # one-row source
]
MODES_MAPS = [("nearest", "half_pixel"), ("nearest", "paper"), ("bilinear", "paper"),
              ("bicubic", "paper")]


@pytest.mark.parametrize("shape", MAP_SHAPES, ids=lambda s: f"{s[0][0]}x{s[0][1]}-{s[1][0]}x{s[1][1]}")
@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32], ids=["u8", "f16", "f32"])
@pytest.mark.parametrize("channels", [1, 4])
@pytest.mark.parametrize("mode_map", MODES_MAPS, ids=lambda m: f"{m[0]}-{m[1]}")
def test_nearest_and_printed_map(shape, dtype, channels, mode_map):
    """Nearest neighbour and eq. 1 as printed, every kernel kind: bitwise equal
    to each other and within the storage rule of the FP64 oracle (nearest:
    exact copies)."""
    mode, mapping = mode_map
    (in_h, in_w), (out_h, out_w) = shape
    img = _input(dtype, in_h, in_w, channels, seed=in_h * 1000 + in_w + channels + 7)
    x = torch.from_numpy(img).to(DEV)
    outs = {}
    for name in TILES:
        t = _tile_for(name, channels)
        if name.startswith("strip_lds") and not _lds_stageable(t, in_w, out_w, mode, dtype, channels):
            continue
        y = xr.resize(x, (out_h, out_w), mode, tile=t, mapping=mapping)
        torch.cuda.synchronize()
        outs[name] = y.cpu().numpy()
    m = R_MAP[mapping]
    compare(outs["auto"], img, out_h, out_w, MODES[mode], what=f"{shape} {mode} {mapping}", mapping=m)
    for name, o in outs.items():
        np.testing.assert_array_equal(o.view(np.uint8), outs["auto"].view(np.uint8),
                                      err_msg=f"kernel {name} differs from the default")


@pytest.mark.parametrize("mode", ["nearest", "bilinear", "bicubic"])
def test_printed_map_bands_match_whole_image(mode):
    img = fields.field_unit(41, 30, 1, seed=8, dtype=np.float32)[:, :, 0]
    out_h, out_w = 97, 50
    whole = _gpu_map(img, out_h, out_w, mode, "paper")
    x = torch.from_numpy(img).to(DEV)
    bands = []
    for row0, row1 in [(0, 30), (30, 31), (31, 97)]:
        first, last = xr.needed_rows(41, out_h, row0, row1 - row0, mode, mapping="paper")
        dst = torch.empty((row1 - row0, out_w), dtype=x.dtype, device=DEV)
        xr.resize_into(x[first:last + 1].contiguous(), dst, mode, src_row0=first, src_height=41,
                       dst_row0=row0, dst_height=out_h, mapping="paper")
        bands.append(dst)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(torch.cat(bands).cpu().numpy().view(np.uint32), whole.view(np.uint32))


def _gpu_map(src_np, out_h, out_w, mode, mapping):
    y = xr.resize(torch.from_numpy(src_np).to(DEV), (out_h, out_w), mode, mapping=mapping)
    torch.cuda.synchronize()
    return y.cpu().numpy()


AA_SHAPES = [
    ((64, 96), (32, 48)),     # x0.5
    ((150, 70), (41, 23)),    # strong, non-dyadic shrink
    ((37, 53), (61, 29)),     # grow rows, shrink columns
    ((33, 21), (33, 21)),     # identity
    ((300, 17), (19, 17)),    # ~x16 rows
    ((5, 9), (12, 20)),       # grow: edges renormalised
]
AA_TILES = [None, xr.tile(xr.XR_KERNEL_GATHER, 8, 8), xr.tile(xr.XR_KERNEL_GATHER, 32, 4),
            xr.tile(xr.XR_KERNEL_GATHER, 256, 1), xr.tile(xr.XR_KERNEL_STRIP, 64, 4, 4, 7),
            xr.tile(xr.XR_KERNEL_STRIP_LDS, 16, 2, 1, 1), xr.tile(xr.XR_KERNEL_STRIP_LDS, 64, 4, 1, 1),
            xr.tile(xr.XR_KERNEL_STRIP_LDS, 16, 16, 1, 1), xr.tile(xr.XR_KERNEL_STRIP_LDS, 128, 2, 1, 1),
            xr.tile(xr.XR_KERNEL_STRIP_LDS, 7, 3, 1, 1)]


@pytest.mark.parametrize("shape", AA_SHAPES, ids=lambda s: f"{s[0][0]}x{s[0][1]}-{s[1][0]}x{s[1][1]}")
@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32], ids=["u8", "f16", "f32"])
@pytest.mark.parametrize("channels", [1, 4])
@pytest.mark.parametrize("mode", ["bilinear_aa", "bicubic_aa"])
def test_antialiased(shape, dtype, channels, mode):
    """The antialiased kernels (gather and LDS-tiled): every block shape
    bitwise equal (a strip tile means the default tile), within the storage
    rule of the FP64 antialiased oracle (float32 weights: never bit-exact for
    uint8). An LDS block whose source window exceeds the budget is refused;
    the 16 x 2 one fits every shape here."""
    (in_h, in_w), (out_h, out_w) = shape
    img = _input(dtype, in_h, in_w, channels, seed=in_h * 1000 + in_w + channels + 11)
    x = torch.from_numpy(img).to(DEV)
    outs = []
    for t in AA_TILES:
        try:
            y = xr.resize(x, (out_h, out_w), mode, tile=t)
        except xr.XResizeError as e:
            assert t is not None and t.kernel == xr.XR_KERNEL_STRIP_LDS and (t.block_w, t.block_h) != (16, 2)
            assert e.code == 11 and "LDS" in str(e)
            continue
        torch.cuda.synchronize()
        outs.append(y.cpu().numpy())
    compare(outs[0], img, out_h, out_w, MODES[mode], what=f"{shape} {mode}")
    for o in outs[1:]:
        np.testing.assert_array_equal(o.view(np.uint8), outs[0].view(np.uint8))


AA_WIDE = [
    ((1000, 1234), (250, 301), np.uint8, 4, "bilinear_aa"),   # ~x0.25, ragged blocks
    ((777, 1500), (389, 751), np.float16, 4, "bicubic_aa"),   # ~x0.5
    ((640, 2048), (91, 300), np.float32, 1, "bicubic_aa"),    # ~x1/7
    ((300, 400), (500, 900), np.uint8, 1, "bilinear_aa"),     # upscale: plain taps
]


@pytest.mark.parametrize("case", AA_WIDE, ids=lambda c: f"{c[0][1]}-{c[1][1]}-c{c[3]}-{c[4]}")
def test_antialiased_tiled_matches_gather_on_many_blocks(case):
    """LDS-tiled and gather kernels bitwise equal over many workgroups with
    ragged right and bottom blocks; sampled rows against the oracle."""
    (in_h, in_w), (out_h, out_w), dtype, channels, mode = case
    img = _input(dtype, in_h, in_w, channels, seed=in_w + 7 * channels)
    x = torch.from_numpy(img).to(DEV)
    ref = xr.resize(x, (out_h, out_w), mode, tile=xr.tile(xr.XR_KERNEL_GATHER, 64, 4))
    for bw, bh in [(64, 4), (32, 8), (16, 2), (48, 5)]:
        try:
            y = xr.resize(x, (out_h, out_w), mode, tile=xr.tile(xr.XR_KERNEL_STRIP_LDS, bw, bh, 1, 1))
        except xr.XResizeError as e:
            assert e.code == 11 and (bw, bh) != (16, 2)
            continue
        torch.cuda.synchronize()
        np.testing.assert_array_equal(y.cpu().numpy().view(np.uint8), ref.cpu().numpy().view(np.uint8))
    torch.cuda.synchronize()
    got = ref.cpu().numpy()
    rows = sorted({0, 1, out_h // 3, out_h - 2, out_h - 1})
    compare(got[rows], img, out_h, out_w, MODES[mode], rows=rows, what=f"{case}")


@pytest.mark.parametrize("dtype", [np.float16, np.float32], ids=["f16", "f32"])
@pytest.mark.parametrize("mode", ["bilinear_aa", "bicubic_aa"])
def test_antialiased_planar(dtype, mode):
    """NCHW tensors (planes = N x C): every plane against the oracle, and the
    LDS-tiled kernel bitwise equal to the gather."""
    n, c, in_h, in_w, out_h, out_w = 2, 3, 91, 130, 30, 41
    x_np = np.ascontiguousarray(
        fields.field_unit(in_h, in_w, n * c, seed=77, dtype=dtype).transpose(2, 0, 1)).reshape(n, c, in_h, in_w)
    x = torch.from_numpy(x_np).to(DEV)
    y = xr.resize(x, (out_h, out_w), mode, layout="nchw")
    g = xr.resize(x, (out_h, out_w), mode, layout="nchw", tile=xr.tile(xr.XR_KERNEL_GATHER, 32, 4))
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint8), g.cpu().numpy().view(np.uint8))
    planes = x_np.reshape(n * c, in_h, in_w, 1)
    compare(got.reshape(n * c, out_h, out_w, 1), planes, out_h, out_w, MODES[mode], what=f"planar {mode}")


@pytest.mark.parametrize("mode", ["bilinear_aa", "bicubic_aa"])
def test_antialiased_bands_and_limits(mode):
    img = fields.field_unit(120, 64, 4, seed=3, dtype=np.float32)
    out_h, out_w = 37, 29
    whole = _gpu(img, out_h, out_w, mode)
    x = torch.from_numpy(img).to(DEV)
    bands = []
    for row0, row1 in [(0, 10), (10, 11), (11, 37)]:
        first, last = xr.needed_rows(120, out_h, row0, row1 - row0, mode)
        dst = torch.empty((row1 - row0, out_w, 4), dtype=x.dtype, device=DEV)
        xr.resize_into(x[first:last + 1].contiguous(), dst, mode, src_row0=first, src_height=120,
                       dst_row0=row0, dst_height=out_h)
        bands.append(dst)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(torch.cat(bands).cpu().numpy().view(np.uint32), whole.view(np.uint32))
    # weight tables beyond the LDS budget are refused
    big = torch.zeros((8, 30000), dtype=torch.float32, device=DEV)
    with pytest.raises(xr.XResizeError) as e:
        xr.resize(big, (8, 10), mode, tile=xr.tile(xr.XR_KERNEL_GATHER, 256, 1))
    assert e.value.code == 11
    with pytest.raises(xr.XResizeError) as e:  # pixel-centre map only
        xr.resize(x, (out_h, out_w), mode, mapping="paper")
    assert e.value.code == 11


def test_antialiased_multi_tile_bands_planar():
    """The LDS-tiled kernel walks several tiles down a tile column when the
    grid is large: 2 x 3 float32 planes, 1000 x 1750 -> 400 x 700 bicubic_aa
    (64 x 4 blocks: 4 tiles per workgroup on the whole image, 2 on the bands
    below, whose last workgroups hold one ragged tile).
    Whole image, three uneven row bands and the gather kernel agree bit for
    bit; sampled rows against the oracle."""
    mode, in_h, in_w, out_h, out_w = "bicubic_aa", 1000, 1750, 400, 700
    x_np = np.ascontiguousarray(
        fields.field_unit(in_h, in_w, 6, seed=91, dtype=np.float32).transpose(2, 0, 1)).reshape(2, 3, in_h, in_w)
    x = torch.from_numpy(x_np).to(DEV)
    lds = xr.tile(xr.XR_KERNEL_STRIP_LDS, 64, 4, 1, 1)
    whole = xr.resize(x, (out_h, out_w), mode, layout="nchw", tile=lds)
    gather = xr.resize(x, (out_h, out_w), mode, layout="nchw", tile=xr.tile(xr.XR_KERNEL_GATHER, 64, 4))
    banded = torch.empty_like(whole)
    for row0, row1 in [(0, 133), (133, 263), (263, 400)]:
        first, last = xr.needed_rows(in_h, out_h, row0, row1 - row0, mode)
        xr.resize_into(x[:, :, first:last + 1], banded[:, :, row0:row1], mode, layout="nchw", tile=lds,
                       src_row0=first, src_height=in_h, dst_row0=row0, dst_height=out_h)
    torch.cuda.synchronize()
    w = whole.cpu().numpy()
    np.testing.assert_array_equal(w.view(np.uint32), gather.cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(w.view(np.uint32), banded.cpu().numpy().view(np.uint32))
    rows = [0, 1, 132, 133, 262, 263, 398, 399]
    for p in (0, 5):
        n, c = divmod(p, 3)
        compare(w[n, c][rows][None, :, :, None], x_np[n, c][:, :, None], out_h, out_w, MODES[mode], rows=rows,
                what=f"multi-tile plane {p}")


LDS_CASES = [
    ((300, 2201), (97, 1290), np.uint8, 4, 256),     # non-dyadic shrink, several workgroups, ragged
    ((130, 1537), (290, 4100), np.float32, 1, 128),  # non-dyadic upscale, ragged right edge
    ((64, 4096), (40, 1024), np.uint8, 1, 256),      # x0.25 across: 16 chunks per lane
    ((50, 3001), (77, 1801), np.float16, 4, 64),     # ~x0.6, narrow workgroups
    ((40, 700), (40, 5600), np.float32, 4, 512),     # x8 across: one chunk per lane
]


@pytest.mark.parametrize("case", LDS_CASES, ids=lambda c: f"{c[0][1]}-{c[1][1]}-c{c[3]}-bw{c[4]}")
@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_lds_strip_wide_images(case, mode):
    (in_h, in_w), (out_h, out_w), dtype, channels, bw = case
    img = _input(dtype, in_h, in_w, channels, seed=in_w + channels)
    ppx = 4 if channels == 4 else 8
    lds = _gpu(img, out_h, out_w, mode, xr.tile(xr.XR_KERNEL_STRIP_LDS, bw, 1, ppx, 13, 1))
    ref = _gpu(img, out_h, out_w, mode, xr.tile(xr.XR_KERNEL_STRIP_ANY, 64, 1, ppx, 13))
    np.testing.assert_array_equal(lds.view(np.uint8), ref.view(np.uint8))
    rng = np.random.default_rng(in_w)
    rows = np.unique(np.concatenate([[0, out_h - 1], rng.integers(0, out_h, 6)]))
    compare(lds[rows], img, out_h, out_w, MODES[mode], rows=rows, what=f"LDS {case} {mode}")


def test_lds_strip_rejects_what_it_cannot_stage():
    x = torch.zeros((4, 32768), dtype=torch.float32, device=DEV)
    with pytest.raises(xr.XResizeError) as e:  # segment beyond the LDS budget
        xr.resize(x, (4, 64), "bicubic", tile=xr.tile(xr.XR_KERNEL_STRIP_LDS, 512, 1, 8, 4))
    assert e.value.code == 11
    u = torch.zeros((8, 37), dtype=torch.uint8, device=DEV)  # rows of 37 bytes: not whole words
    with pytest.raises(xr.XResizeError) as e:
        xr.resize(u, (16, 74), "bicubic", tile=xr.tile(xr.XR_KERNEL_STRIP_LDS, 64, 1, 8, 4))
    assert e.value.code == 11
    # the default shape never picks what the source cannot use
    out = xr.resize(u, (16, 74), "bicubic")
    torch.cuda.synchronize()
    assert int(out.sum()) == 0


@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
@pytest.mark.parametrize("out_hw", [(194, 160), (48, 40)], ids=["x2", "x0.5"])
def test_bands_match_whole_image(mode, out_hw):
    img = fields.field_unit(97, 80, 1, seed=5, dtype=np.float16)[:, :, 0]
    if out_hw[0] < 97:
        img = img[:96]
    out_h, out_w = out_hw
    whole = _gpu(img, out_h, out_w, mode)
    x = torch.from_numpy(img).to(DEV)
    in_h = img.shape[0]
    bands = []
    cuts = [0, 61, 62, 132, 194] if out_h == 194 else [0, 13, 14, 31, 48]
    for row0, row1 in zip(cuts[:-1], cuts[1:]):
        rows = row1 - row0
        first, last = xr.needed_rows(in_h, out_h, row0, rows, mode)
        src_band = x[first:last + 1].contiguous()
        dst_band = torch.empty((rows, out_w), dtype=x.dtype, device=DEV)
        xr.resize_into(src_band, dst_band, mode, src_row0=first, src_height=in_h, dst_row0=row0,
                       dst_height=out_h)
        bands.append(dst_band)
    torch.cuda.synchronize()
    got = torch.cat(bands).cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint16), whole.view(np.uint16))


def test_band_missing_halo_rejected():
    x = torch.zeros((10, 8), dtype=torch.uint8, device=DEV)
    dst = torch.empty((4, 16), dtype=torch.uint8, device=DEV)
    with pytest.raises(xr.XResizeError) as e:
        # output rows 8..11 of 40 read source rows 2..7; the band holds rows 4..13
        xr.resize_into(x, dst, "bicubic", src_row0=4, src_height=20, dst_row0=8, dst_height=40)
    assert e.value.code == 6


# the benchmark's timed launch shape for the x2 workload (and the default)
BENCH_TILE_X2 = xr.tile(xr.XR_KERNEL_STRIP, 256, 1, 4, 22, 0)


@pytest.mark.parametrize("direction,tile", [("up", None), ("up", BENCH_TILE_X2), ("down", None)],
                         ids=["up-default", "up-bench-tile", "down-default"])
def test_c2_rgba_u8_bicubic_sampled(direction, tile):
    img = fields.field_u8(4096, 4096, 4, seed=1002)
    out = 8192 if direction == "up" else 2048
    x = torch.from_numpy(img).to(DEV)
    y = xr.resize(x, (out, out), "bicubic", tile=tile)
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([[0, 1, 2, out - 2, out - 1], rng.integers(0, out, 40)]))
    got = y[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    res = compare(got[None], img, out, out, 1, rows=rows, what=f"C2 {direction}")
    assert res["ties"] == 0 and res["non_ties"] == 0


def test_autotune_choice_does_not_change_results():
    img = fields.uniform_u8((300, 260, 4), seed=17)
    x = torch.from_numpy(img).to(DEV)
    before = xr.resize(x, (600, 520), "bicubic").cpu().numpy()
    srcs = [x, x.clone()]
    dsts = [torch.empty((600, 520, 4), dtype=torch.uint8, device=DEV) for _ in range(2)]
    cands = xr.tune_candidates("bicubic", xr.XR_U8, 4, 260, 300, 520, 600)
    best, ms = xr.autotune(srcs, dsts, "bicubic", candidates=cands, reps=2, groups=2)
    assert ms > 0 and best.kernel in (xr.XR_KERNEL_GATHER, xr.XR_KERNEL_STRIP)
    assert xr.get_tile("bicubic", xr.XR_U8, 4, 260, 300, 520, 600).as_tuple() == best.as_tuple()
    after = xr.resize(x, (600, 520), "bicubic").cpu().numpy()
    np.testing.assert_array_equal(after, before)
    for d in dsts:
        np.testing.assert_array_equal(d.cpu().numpy(), before)
    xr.set_tile("bicubic", xr.XR_U8, 4, 260, 300, 520, 600, xr.tile(xr.XR_KERNEL_AUTO))


EXACT_SHAPES = [
    ((37, 53), (74, 106)),   # x2, ragged
    ((3, 3), (6, 6)),        # x2, image narrower than one thread's run
    ((1, 70), (2, 140)),     # x2, one source row
    ((74, 262), (37, 131)),  # x0.5, ragged
    ((6, 10), (3, 5)),       # x0.5, narrower than a run
    ((130, 2), (65, 1)),     # x0.5, one output column
]


@pytest.mark.parametrize("shape", EXACT_SHAPES, ids=lambda s: f"{s[0][0]}x{s[0][1]}-{s[1][0]}x{s[1][1]}")
@pytest.mark.parametrize("dtype", [np.uint8, np.float16, np.float32], ids=["u8", "f16", "f32"])
@pytest.mark.parametrize("channels", [1, 4])
@pytest.mark.parametrize("mode", ["bilinear", "bicubic"])
def test_exact_ratio_walks_every_width(shape, dtype, channels, mode):
    """The exact x2 and x0.5 walks with every built run width (direct and
    LDS-exchanged run stores, edge runs rebuilt in registers or loaded pixel
    by pixel), strip heights that split the image unevenly and both workgroup
    orders: bitwise equal
    to each other and to the one-pixel gather, and within the oracle rule."""
    (in_h, in_w), (out_h, out_w) = shape
    img = _input(dtype, in_h, in_w, channels, seed=in_h * 31 + in_w * 7 + channels)
    ref = _gpu(img, out_h, out_w, mode, xr.tile(xr.XR_KERNEL_GATHER, 64, 1))
    compare(ref, img, out_h, out_w, MODES[mode], what=f"{shape} {mode}")
    widths = (1, 2, 4, 8) if channels == 4 else (4, 8, 16)
    for ppx in widths:
        for bw, bh, ppy in ((64, 1, 8), (128, 2, 16), (64, 4, 2)):
            for order in (0, 1):
                got = _gpu(img, out_h, out_w, mode, xr.tile(xr.XR_KERNEL_STRIP, bw, bh, ppx, ppy, order))
                np.testing.assert_array_equal(got.view(np.uint8), ref.view(np.uint8),
                                              err_msg=f"ppx {ppx} block {bw}x{bh} rows {ppy} order {order}")
