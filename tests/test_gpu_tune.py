"""GPU tests of persisted launch shapes (xr_tune_save / xr_tune_load): a saved
table loads back on the same GPU and build; a file headed by another build or
architecture loads nothing; resizes with a loaded shape are bitwise unchanged."""

import os

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1001_1718_amd as xr  # noqa: E402

KEY = ("bilinear", xr.XR_U8, 4, 300, 200, 450, 300)


def test_save_load_roundtrip(tmp_path):
    assert xr.get_tile(*KEY).as_tuple() != xr.tile(xr.XR_KERNEL_STRIP, 256, 2, 2, 6).as_tuple()
    t = xr.tile(xr.XR_KERNEL_STRIP, 256, 2, 2, 6)
    xr.set_tile(*KEY, t)
    path = str(tmp_path / "tiles.txt")
    xr.tune_save(path)
    xr.set_tile(*KEY, xr.tile(xr.XR_KERNEL_AUTO))
    n = xr.tune_load(path)
    assert n >= 1
    assert xr.get_tile(*KEY).as_tuple() == t.as_tuple()
    # results with the loaded shape equal those of the default shape
    src = torch.randint(0, 256, (200, 300, 4), dtype=torch.uint8, device="cuda:0")
    a = xr.resize(src, (300, 450), "bilinear")
    xr.set_tile(*KEY, xr.tile(xr.XR_KERNEL_AUTO))
    b = xr.resize(src, (300, 450), "bilinear")
    assert torch.equal(a, b)


def test_foreign_file_loads_nothing(tmp_path):
    t = xr.tile(xr.XR_KERNEL_STRIP, 256, 2, 2, 6)
    xr.set_tile(*KEY, t)
    path = str(tmp_path / "tiles.txt")
    xr.tune_save(path)
    xr.set_tile(*KEY, xr.tile(xr.XR_KERNEL_AUTO))
    lines = open(path).read().splitlines()
    for bad in (lines[1].replace(" build ", " build x"), lines[1].replace(" cus ", " cus 1")):
        with open(path, "w") as f:
            f.write("\n".join([lines[0], bad] + lines[2:]) + "\n")
        assert xr.tune_load(path) == 0
    assert xr.get_tile(*KEY).as_tuple() != t.as_tuple()
    with pytest.raises(xr.XResizeError):
        xr.tune_load(os.path.join(str(tmp_path), "missing.txt"))
