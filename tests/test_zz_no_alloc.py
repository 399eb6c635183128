"""GPU test of xr_resize_batched_static, the batched launch whose workspace is
the library's static device array: called through the C-ABI twice in a row
(the second batch smaller), every output must equal, bit for bit, what
xr_batch_prepare + xr_resize_batched write for the same jobs; a batch over
the static limit is refused before any launch."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1001_1718_amd as xr  # noqa: E402
from paper_1001_1718_amd import _lib  # noqa: E402
from synth import fields  # noqa: E402

DEV = "cuda:0"


def _jobs(seed, count, side_hi, dtype=torch.uint8):
    rng = np.random.default_rng(seed)
    pairs = []
    for j in fields.batch_jobs(seed, count=count, side_hi=side_hi):
        if dtype == torch.uint8:
            s = torch.from_numpy(rng.integers(0, 256, (j.in_h, j.in_w, j.channels), dtype=np.uint8)).to(DEV)
        else:
            s = torch.from_numpy(rng.random((j.in_h, j.in_w, j.channels)).astype(np.float32)).to(dtype).to(DEV)
        pairs.append((s, torch.empty((j.out_h, j.out_w, j.channels), dtype=dtype, device=DEV), j.filter))
    return pairs


def _static_call(pairs, tile=None):
    n = len(pairs)
    arr = (_lib.XrJob * n)()
    for k, (s, d, f) in enumerate(pairs):
        arr[k].src = xr.image(s)
        arr[k].dst = xr.image(d)
        arr[k].filter = xr.filter_code(f)
    stream = torch.cuda.current_stream().cuda_stream
    return _lib.lib.xr_resize_batched_static(arr, n, xr._tile_ptr(tile), ctypes.c_void_p(stream))


@pytest.mark.parametrize("dtype", [torch.uint8, torch.float16], ids=["u8", "f16"])
def test_static_batch_equals_workspace_batch_twice(dtype):
    # first call: a larger batch; second call: a smaller one on the same
    # static array (its earlier contents must not leak into the result)
    for seed, count, side_hi in ((41, 40, 700), (42, 6, 150)):
        pairs = _jobs(seed, count, side_hi, dtype)
        b = xr.Batch(pairs)
        b.run()
        torch.cuda.synchronize()
        ref = [d.clone() for _, d, _ in pairs]
        for _, d, _ in pairs:
            d.fill_(0)
        torch.cuda.synchronize()
        rc = _static_call(pairs)
        torch.cuda.synchronize()
        assert rc == 0, _lib.last_error()
        for k, ((_, d, _), r) in enumerate(zip(pairs, ref)):
            assert torch.equal(d, r), f"seed {seed}: job {k} differs from the workspace launch"


def test_static_batch_explicit_tile_and_limit():
    pairs = _jobs(43, 12, 300)
    tile = xr.tile(xr.XR_KERNEL_STRIP, 64, 4, 0, 30)
    b = xr.Batch(pairs, tile=tile)
    b.run()
    torch.cuda.synchronize()
    ref = [d.clone() for _, d, _ in pairs]
    for _, d, _ in pairs:
        d.fill_(0)
    assert _static_call(pairs, tile) == 0
    torch.cuda.synchronize()
    assert all(torch.equal(d, r) for (_, d, _), r in zip(pairs, ref))
    # over the static limit: refused with XR_ERR_WORKSPACE, nothing launched
    s = torch.zeros((8, 8, 1), dtype=torch.uint8, device=DEV)
    outs = [torch.zeros((4, 4, 1), dtype=torch.uint8, device=DEV) for _ in range(1025)]
    assert _static_call([(s, o, 0) for o in outs]) == _lib.XR_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert all(int(o.sum()) == 0 for o in outs[:4])
