"""CPU-only checks of the C ABI: the library loads and exports every symbol the
header declares, the struct layouts agree with the C compiler, every argument
error is reported before any HIP call, and the host geometry helpers follow
eqs. 1-4 and 6 exactly."""

import ctypes
import os
import re
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import paper_1001_1718_amd as xr
from paper_1001_1718_amd import _lib
from oracle import ref_resize as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xresize.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xr_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = _declared_functions()
    assert len(names) >= 16
    lib = ctypes.CDLL(_lib.LIBRARY)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIBRARY], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (xr_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(xr_image), offsetof(xr_image, width),
         offsetof(xr_image, row_pitch), offsetof(xr_image, planes), offsetof(xr_image, plane_pitch),
         offsetof(xr_image, row0), offsetof(xr_image, rows), sizeof(xr_tile), sizeof(xr_job),
         offsetof(xr_job, filter));
  return 0;
}}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(prog), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                       check=True).stdout.split()))
    want = [ctypes.sizeof(_lib.XrImage), _lib.XrImage.width.offset, _lib.XrImage.row_pitch.offset,
            _lib.XrImage.planes.offset, _lib.XrImage.plane_pitch.offset, _lib.XrImage.row0.offset,
            _lib.XrImage.rows.offset, ctypes.sizeof(_lib.XrTile), ctypes.sizeof(_lib.XrJob),
            _lib.XrJob.filter.offset]
    assert got == want


FAKE = 0x7F0000000000  # never dereferenced: every call below fails validation


def _img(w=16, h=16, c=1, dtype=0, data=FAKE, pitch=None, planes=1, plane_pitch=0, row0=0, rows=None):
    es = {0: 1, 1: 2, 2: 4}.get(dtype, 1)
    im = _lib.XrImage()
    im.data = data
    im.width, im.height, im.channels, im.dtype = w, h, c, dtype
    im.row_pitch = w * c * es if pitch is None else pitch
    im.planes = planes
    im.plane_pitch = plane_pitch
    im.row0 = row0
    im.rows = h if rows is None else rows
    return im


def _fwd(src, dst, tile=None, mode=0):
    fn = _lib.lib.xr_resize_bicubic if mode else _lib.lib.xr_resize_bilinear
    return fn(ctypes.byref(src) if src is not None else None,
              ctypes.byref(dst) if dst is not None else None,
              ctypes.byref(tile) if tile is not None else None, None)


D2 = FAKE + (1 << 30)  # a second, non-overlapping fake buffer

CASES = [
    ("null src", lambda: _fwd(None, _img(32, 32, data=D2)), 1),
    ("null data", lambda: _fwd(_img(data=0), _img(32, 32, data=D2)), 1),
    ("zero width", lambda: _fwd(_img(w=0), _img(32, 32, data=D2)), 2),
    ("too wide", lambda: _fwd(_img(w=40000), _img(32, 32, data=D2)), 2),
    ("no planes", lambda: _fwd(_img(planes=0), _img(32, 32, data=D2)), 2),
    ("plane mismatch", lambda: _fwd(_img(planes=2, plane_pitch=256), _img(32, 32, data=D2)), 2),
    ("bad dtype", lambda: _fwd(_img(dtype=7), _img(32, 32, data=D2)), 3),
    ("dtype mismatch", lambda: _fwd(_img(dtype=1), _img(32, 32, data=D2)), 3),
    ("3 channels", lambda: _fwd(_img(c=3), _img(32, 32, c=3, data=D2)), 4),
    ("channel mismatch", lambda: _fwd(_img(c=4), _img(32, 32, data=D2)), 4),
    ("short pitch", lambda: _fwd(_img(pitch=15), _img(32, 32, data=D2)), 5),
    ("pitch not pixel multiple", lambda: _fwd(_img(c=4, pitch=66), _img(32, 32, c=4, data=D2)), 5),
    ("misaligned data", lambda: _fwd(_img(c=4, data=FAKE + 2), _img(32, 32, c=4, data=D2)), 5),
    ("short plane pitch", lambda: _fwd(_img(planes=2, plane_pitch=100),
                                       _img(32, 32, planes=2, plane_pitch=1024, data=D2)), 5),
    ("band past end", lambda: _fwd(_img(), _img(32, 32, data=D2, row0=30, rows=4)), 6),
    ("band missing halo", lambda: _fwd(_img(row0=4, rows=10, h=20), _img(32, 40, data=D2, row0=8, rows=4), mode=1), 6),
    ("alias", lambda: _fwd(_img(), _img(32, 32, data=FAKE + 100)), 7),
    ("bad tile kind", lambda: _fwd(_img(), _img(32, 32, data=D2), tile=xr.tile(9, 64, 1, 1, 1)), 11),
    ("gather too many threads", lambda: _fwd(_img(), _img(32, 32, data=D2),
                                             tile=xr.tile(xr.XR_KERNEL_GATHER, 64, 32)), 11),
    ("strip block not wave multiple", lambda: _fwd(_img(), _img(32, 32, data=D2),
                                                   tile=xr.tile(xr.XR_KERNEL_STRIP, 32, 4, 8, 8)), 11),
    ("strip ppt not built", lambda: _fwd(_img(), _img(32, 32, data=D2),
                                         tile=xr.tile(xr.XR_KERNEL_STRIP, 64, 4, 3, 8)), 11),
    ("strip too many threads", lambda: _fwd(_img(), _img(32, 32, data=D2),
                                            tile=xr.tile(xr.XR_KERNEL_STRIP, 512, 2, 8, 8)), 11),
    ("bad order", lambda: _fwd(_img(), _img(32, 32, data=D2),
                               tile=xr.tile(xr.XR_KERNEL_STRIP, 64, 4, 8, 8, 2)), 11),
    ("gather with order", lambda: _fwd(_img(), _img(32, 32, data=D2),
                                       tile=xr.tile(xr.XR_KERNEL_GATHER, 8, 8, 1, 1, 1)), 11),
]


@pytest.mark.parametrize("name,call,code", CASES, ids=[c[0] for c in CASES])
def test_validation_codes(name, call, code):
    assert call() == code, _lib.last_error()
    assert _lib.last_error()


def test_backward_validation():
    f = _lib.lib.xr_resize_backward
    g = _img(32, 32, dtype=2, data=D2)
    s = _img(16, 16, dtype=2)
    assert f(ctypes.byref(g), ctypes.byref(_img(16, 16, dtype=0)), 0, None) == 3
    assert f(ctypes.byref(g), ctypes.byref(s), 5, None) == 11
    assert f(ctypes.byref(_img(32, 32, dtype=2, data=D2, row0=4, rows=8)), ctypes.byref(s), 0, None) == 6
    assert f(ctypes.byref(g), ctypes.byref(_img(16, 16, dtype=2, data=D2 + 64)), 0, None) == 7
    assert f(None, ctypes.byref(s), 0, None) == 1
    # float16 gradients are accepted only in pairs; uint8 never
    g16 = _img(32, 32, dtype=1, data=D2)
    assert f(ctypes.byref(g16), ctypes.byref(s), 0, None) == 3
    assert f(ctypes.byref(_img(32, 32, dtype=0, data=D2)), ctypes.byref(_img(16, 16, dtype=0)), 0, None) == 3


def test_batch_validation():
    lib = _lib.lib
    jobs = (_lib.XrJob * 2)()
    jobs[0].src, jobs[0].dst, jobs[0].filter = _img(), _img(32, 32, data=D2), 0
    jobs[1].src, jobs[1].dst, jobs[1].filter = _img(), _img(32, 32, data=D2 + 4096), 1
    need = lib.xr_batch_workspace_bytes(2)
    assert need >= 256 + 2 * 64 and lib.xr_batch_workspace_bytes(0) == 0
    ws = FAKE + (2 << 30)
    assert lib.xr_batch_prepare(None, 2, None, ws, need, None) == 1
    assert lib.xr_batch_prepare(jobs, 0, None, ws, need, None) == 11
    assert lib.xr_batch_prepare(jobs, 2, None, None, need, None) == 8
    assert lib.xr_batch_prepare(jobs, 2, None, ws + 8, need, None) == 8
    assert lib.xr_batch_prepare(jobs, 2, None, ws, need - 1, None) == 8
    # the batch autotuner validates before any HIP call
    tune = lib.xr_batch_autotune
    assert tune(None, 2, None, 0, 3, 3, ws, need, None, None, None) == 1
    assert tune(jobs, 0, None, 0, 3, 3, ws, need, None, None, None) == 11
    assert tune(jobs, 2, None, 0, 0, 3, ws, need, None, None, None) == 11
    assert tune(jobs, 2, None, 0, 3, 0, ws, need, None, None, None) == 11
    gather = (_lib.XrTile * 1)(_lib.tile(_lib.XR_KERNEL_GATHER, 8, 8))
    assert tune(jobs, 2, gather, 1, 3, 3, ws, need, None, None, None) == 11
    strip = (_lib.XrTile * 1)(_lib.tile(_lib.XR_KERNEL_STRIP, 256, 1, 4, 14))
    assert tune(jobs, 2, strip, 0, 3, 3, ws, need, None, None, None) == 11
    assert tune(jobs, 2, strip, 1, 3, 3, None, need, None, None, None) == 8
    jobs[1].filter = 4
    assert lib.xr_batch_prepare(jobs, 2, None, ws, need, None) == 11
    jobs[1].filter = 1
    jobs[1].dst = _img(32, 32, data=D2 + 100)  # overlaps job 0's output
    assert lib.xr_batch_prepare(jobs, 2, None, ws, need, None) == 7
    assert lib.xr_resize_batched(None, 2, None) == 8
    assert lib.xr_resize_batched(ws + 4096 * 256, 2, None) == 8  # never prepared


def test_resize_with_mapping_validates_first():
    f = _lib.lib.xr_resize
    s, d = _img(), _img(32, 32, data=D2)
    assert f(ctypes.byref(s), ctypes.byref(d), 7, 0, None, None) == 11   # unknown filter
    assert f(ctypes.byref(s), ctypes.byref(d), 4, 1, None, None) == 11   # antialiased + printed map
    assert f(ctypes.byref(s), ctypes.byref(d), 2, 2, None, None) == 11   # unknown mapping
    assert f(None, ctypes.byref(d), 2, 1, None, None) == 1


@pytest.mark.parametrize("filt", [3, 4])
def test_needed_rows_antialiased_match_oracle(filt):
    from oracle import ref_resize as R

    for in_h, out_h in [(17, 40), (40, 17), (300, 71), (64, 4), (9, 9)]:
        idx, w = R.axis_taps_antialiased(in_h, out_h, filt)
        for row0, rows in [(0, 1), (0, out_h), (out_h // 3, max(1, out_h // 4)), (out_h - 1, 1)]:
            sel = [idx[y][w[y] != 0] for y in range(row0, row0 + rows)]
            first, last = ctypes.c_int32(), ctypes.c_int32()
            assert _lib.lib.xr_needed_rows_map(in_h, out_h, row0, rows, filt, 0, ctypes.byref(first),
                                               ctypes.byref(last)) == 0
            # the library's range holds every tap with a nonzero weight ...
            assert first.value <= min(int(t.min()) for t in sel)
            assert last.value >= max(int(t.max()) for t in sel)
            # ... and no row outside (s - R sigma, s + R sigma] of its end rows
            r = 2 if filt == 4 else 1
            sigma = max(1.0, in_h / out_h)
            s0 = (row0 + 0.5) * in_h / out_h - 0.5
            s1 = (row0 + rows - 1 + 0.5) * in_h / out_h - 0.5
            assert first.value >= max(0, int(np.floor(s0 - r * sigma)) + 1)
            assert last.value <= min(in_h - 1, int(np.floor(s1 + r * sigma)))


@pytest.mark.parametrize("filt", [0, 1, 2])
@pytest.mark.parametrize("mapping", [0, 1])
def test_needed_rows_map_match_oracle(filt, mapping):
    from oracle import ref_resize as R

    for in_h, out_h in [(17, 40), (40, 17), (9, 9), (1, 5), (300, 71)]:
        for row0, rows in [(0, 1), (0, out_h), (out_h // 3, max(1, out_h // 4)), (out_h - 1, 1)]:
            first, last = ctypes.c_int32(), ctypes.c_int32()
            assert _lib.lib.xr_needed_rows_map(in_h, out_h, row0, rows, filt, mapping, ctypes.byref(first),
                                               ctypes.byref(last)) == 0
            assert (first.value, last.value) == R.needed_rows(in_h, out_h, row0, rows, filt, mapping)
    first, last = ctypes.c_int32(), ctypes.c_int32()
    assert _lib.lib.xr_needed_rows_map(8, 8, 0, 1, filt, 5, ctypes.byref(first), ctypes.byref(last)) == 11


def test_strerror_all_codes():
    for code in range(12):
        assert _lib.strerror(code) and _lib.strerror(code) != "unknown error code"
    assert _lib.strerror(99) == "unknown error code"
    assert _lib.lib.xr_version() >= 100


@pytest.mark.parametrize("n_in,n_out", [(512, 1024), (4096, 2048), (37, 61), (1, 7), (32768, 1),
                                        (1, 32768), (32768, 32767), (1537, 3211)])
def test_source_taps_exact(n_in, n_out):
    xs = sorted(x for x in set([0, 1, n_out // 2, n_out - 1] + list(range(0, n_out, max(1, n_out // 50)))) if x < n_out)
    for x in xs:
        x0, num, den = xr.source_taps(n_in, n_out, x)
        s = Fraction((2 * x + 1) * n_in - n_out, 2 * n_out)          # eq. 1, half-pixel
        assert x0 == s.__floor__() and Fraction(num, den) == s - x0  # eqs. 2-4 with floor
        assert 0 <= num < den


def test_needed_rows_matches_oracle():
    rng = np.random.default_rng(0)
    for _ in range(200):
        in_h, out_h = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        row0 = int(rng.integers(0, out_h))
        rows = int(rng.integers(1, out_h - row0 + 1))
        for mode in (0, 1):
            assert xr.needed_rows(in_h, out_h, row0, rows, mode) == \
                R.needed_rows(in_h, out_h, row0, rows, mode)


def test_eq6_worked_example(golden_dir):
    rows = [ln.split() for ln in open(os.path.join(golden_dir, "eq6_worked_example.txt"))
            if ln.strip() and not ln.startswith("#")]
    for bw, bh, px, py, bx, by, tx, ty in (map(int, r) for r in rows):
        t = xr.tile(xr.XR_KERNEL_GATHER, bw, bh)
        assert xr.thread_of_pixel(t, px, py) == (bx, by, tx, ty, 0, 0)
    # with pixels per thread the block size is block * ppt and eq. 6 still holds
    t = xr.tile(xr.XR_KERNEL_STRIP, 64, 4, 4, 32)
    bx, by, tx, ty, sx, sy = xr.thread_of_pixel(t, 1000, 300)
    assert bx * 256 + tx * 4 + sx == 1000 and by * 128 + ty * 32 + sy == 300


def test_tune_candidates_include_paper_shapes():
    cands = xr.tune_candidates("bilinear", xr.XR_U8, 1, 800, 800, 1600, 1600)
    gathers = {(c.block_w, c.block_h) for c in cands if c.kernel == xr.XR_KERNEL_GATHER}
    assert {(8, 8), (32, 4), (32, 16), (4, 8), (8, 4)} <= gathers
    assert any(c.kernel == xr.XR_KERNEL_STRIP for c in cands)


def test_get_set_tile_roundtrip():
    key = ("bicubic", xr.XR_F16, 1, 100, 100, 300, 300)
    default = xr.get_tile(*key)
    t = xr.tile(xr.XR_KERNEL_STRIP, 128, 2, 8, 16)
    xr.set_tile(*key, t)
    assert xr.get_tile(*key).as_tuple() == t.as_tuple()
    xr.set_tile(*key, xr.tile(xr.XR_KERNEL_AUTO))
    assert xr.get_tile(*key).as_tuple() == default.as_tuple()
    with pytest.raises(xr.XResizeError):
        xr.set_tile(*key, xr.tile(xr.XR_KERNEL_STRIP, 100, 1, 8, 16))


def test_tuned_shape_keyed_by_output_size():
    """A shape stored for a large output is not used for a small output of the
    same filter, storage, channels and scale, and vice versa; outputs in the
    same size class share it."""
    big = ("bicubic", xr.XR_U8, 4, 4096, 4096, 8192, 8192)      # 2^26 px: class 3
    small = ("bicubic", xr.XR_U8, 4, 64, 64, 128, 128)          # 2^14 px: class 0
    near = ("bicubic", xr.XR_U8, 4, 3000, 3000, 6000, 6000)     # class 3 too
    d_small = xr.get_tile(*small).as_tuple()
    t = xr.tile(xr.XR_KERNEL_STRIP, 512, 1, 2, 24)
    xr.set_tile(*big, t)
    try:
        assert xr.get_tile(*big).as_tuple() == t.as_tuple()
        assert xr.get_tile(*near).as_tuple() == t.as_tuple()
        assert xr.get_tile(*small).as_tuple() == d_small
    finally:
        xr.set_tile(*big, xr.tile(xr.XR_KERNEL_AUTO))
