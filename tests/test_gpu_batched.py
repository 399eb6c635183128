"""GPU tests of the persistent batched launch (xr_batch_prepare / xr_resize_batched).

* a batch of uneven uint8 jobs (1 and 4 channels, both filters, scales
  0.25 .. 4): every output bitwise equal to the per-image launch, and within
  the uint8 rule of the FP64 oracle on sampled rows;
* replays from a captured HIP graph, with eager work in between, equal the
  eager result every time (the ticket counter resets itself);
* the full 256-job batch: bitwise equal to 256 per-image launches;
* FP16 interleaved and FP32 planar (NCHW, several planes per job) batches;
* narrow, short and strongly scaled jobs of every kind and storage type
  (taps clamped on both sides of a column, strips of 1 to 256 rows);
* the batch autotuner keeps results bitwise unchanged;
* host-side validation of prepare (capture, workspace, dtype mix).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1001_1718_amd as xr  # noqa: E402
from gpu_util import compare  # noqa: E402
from synth import fields  # noqa: E402

DEV = "cuda:0"
NAMES = {0: "bilinear", 1: "bicubic"}


def _make_batch(seed, count, side_hi, content="uniform"):
    jobs = fields.batch_jobs(seed, count=count, side_hi=side_hi)
    pairs, srcs = [], []
    for j in jobs:
        if content == "uniform":
            s = torch.from_numpy(fields.uniform_u8((j.in_h, j.in_w, j.channels), j.content_seed)).to(DEV)
        else:
            s = fields.field_u8_torch(j.in_h, j.in_w, j.channels, j.content_seed, DEV)
        d = torch.empty((j.out_h, j.out_w, j.channels), dtype=torch.uint8, device=DEV)
        pairs.append((s, d, j.filter))
        srcs.append(s)
    return jobs, pairs


def _per_image(pairs):
    outs = []
    for s, d, f in pairs:
        o = torch.empty_like(d)
        xr.resize_into(s, o, f)
        outs.append(o)
    torch.cuda.synchronize()
    return outs


def test_small_batch_matches_per_image_and_oracle():
    jobs, pairs = _make_batch(seed=11, count=24, side_hi=300)
    ref = _per_image(pairs)
    b = xr.Batch(pairs)
    b.run()
    torch.cuda.synchronize()
    for k, ((s, d, f), r) in enumerate(zip(pairs, ref)):
        assert torch.equal(d, r), f"job {k}: batched output differs from the per-image launch"
    rng = np.random.default_rng(1)
    for k, (j, (s, d, f)) in enumerate(zip(jobs, pairs)):
        rows = np.unique(np.concatenate([[0, j.out_h - 1], rng.integers(0, j.out_h, 3)]))
        got = d[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        compare(got[None], s.cpu().numpy(), j.out_h, j.out_w, f, rows=rows, what=f"job {k}")


def test_batch_replays_and_graph():
    jobs, pairs = _make_batch(seed=12, count=16, side_hi=400)
    ref = _per_image(pairs)
    b = xr.Batch(pairs)
    stream = torch.cuda.Stream()
    # eager replays: the ticket counter must come back to zero after every launch
    for _ in range(3):
        for _, d, _ in pairs:
            d.zero_()
        b.run()
        torch.cuda.synchronize()
        for (_, d, _), r in zip(pairs, ref):
            assert torch.equal(d, r)
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            b.run(stream=stream)
    torch.cuda.synchronize()
    for rep in range(4):
        for _, d, _ in pairs:
            d.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, ((_, d, _), r) in enumerate(zip(pairs, ref)):
            assert torch.equal(d, r), f"graph replay {rep}: job {k} differs"
        b.run()  # an eager launch between replays
        torch.cuda.synchronize()


def test_full_batch_bitwise_equal_to_per_image():
    jobs, pairs = _make_batch(seed=0, count=256, side_hi=2048, content="field")
    ref = _per_image(pairs)
    b = xr.Batch(pairs)
    b.run()
    torch.cuda.synchronize()
    bad = [k for k, ((_, d, _), r) in enumerate(zip(pairs, ref)) if not torch.equal(d, r)]
    assert not bad, f"jobs {bad[:10]} differ between batched and per-image launches"
    # the oracle on one sampled row of every 8th job
    rng = np.random.default_rng(2)
    for k in range(0, 256, 8):
        j = jobs[k]
        s, d, f = pairs[k]
        rows = rng.integers(0, j.out_h, 1)
        got = d[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        compare(got[None], s.cpu().numpy(), j.out_h, j.out_w, f, rows=rows, what=f"job {k}")


@pytest.mark.parametrize("dtype", [torch.float16, torch.float32], ids=["f16", "f32"])
def test_float_batches(dtype):
    """FP16 interleaved (1 and 4 channels) and FP32 planar NCHW jobs."""
    jobs = fields.batch_jobs(21, count=12, side_hi=260)
    pairs, layout = [], "hwc" if dtype == torch.float16 else "nchw"
    for j in jobs:
        if layout == "hwc":
            s = torch.from_numpy(fields.field_unit(j.in_h, j.in_w, j.channels, j.content_seed,
                                                   np.float16)).to(DEV)
            d = torch.empty((j.out_h, j.out_w, j.channels), dtype=dtype, device=DEV)
        else:  # N = 2 images of C = channels planes
            s = torch.from_numpy(fields.normal_f32((2, j.channels, j.in_h, j.in_w), j.content_seed)).to(DEV)
            d = torch.empty((2, j.channels, j.out_h, j.out_w), dtype=dtype, device=DEV)
        pairs.append((s, d, j.filter))
    ref = []
    for s, d, f in pairs:
        o = torch.empty_like(d)
        xr.resize_into(s, o, f, layout=layout)
        ref.append(o)
    b = xr.Batch(pairs, layout=layout)
    b.run()
    torch.cuda.synchronize()
    for k, ((s, d, f), r) in enumerate(zip(pairs, ref)):
        assert torch.equal(d, r), f"job {k}: batched output differs from the per-image launch"
    rng = np.random.default_rng(5)
    for k, (j, (s, d, f)) in enumerate(zip(jobs, pairs)):
        rows = np.unique(np.concatenate([[0, j.out_h - 1], rng.integers(0, j.out_h, 2)]))
        src = s.cpu().numpy()
        if layout == "hwc":
            got = d[torch.from_numpy(rows).to(DEV)].cpu().numpy()[None]
            compare(got, src, j.out_h, j.out_w, f, rows=rows, what=f"f16 job {k}")
        else:
            planes = src.reshape(-1, j.in_h, j.in_w)[:, :, :, None]
            got = d.reshape(-1, j.out_h, j.out_w)[:, torch.from_numpy(rows).to(DEV)].cpu().numpy()[..., None]
            compare(got, planes, j.out_h, j.out_w, f, rows=rows, what=f"f32 job {k}")


# (in_h, in_w, out_h, out_w): images narrower or shorter than the taps,
# shrinks of 4x and more (row and column windows that do not overlap),
# enlargements of 4x and more, ragged sizes
EDGE_SHAPES = [(1, 1, 5, 7), (2, 3, 9, 4), (3, 2, 1, 1), (5, 3, 17, 2), (7, 1, 3, 40), (64, 5, 16, 300),
               (300, 9, 75, 2), (13, 600, 200, 37), (40, 40, 160, 160), (200, 800, 40, 150),
               (33, 130, 131, 519)]
EDGE_TILES = [None, (64, 4, 1), (256, 1, 256), (128, 2, 64)]


@pytest.mark.parametrize("dtype", [torch.uint8, torch.float16, torch.float32], ids=["u8", "f16", "f32"])
def test_batch_narrow_and_extreme_jobs(dtype):
    rng = np.random.default_rng(31)
    pairs, specs = [], []
    for k, (ih, iw, oh, ow) in enumerate(EDGE_SHAPES):
        for ch in (1, 4):
            for f in (0, 1):
                if dtype == torch.uint8:
                    s = torch.from_numpy(rng.integers(0, 256, (ih, iw, ch), dtype=np.uint8)).to(DEV)
                else:
                    s = torch.from_numpy(rng.random((ih, iw, ch)).astype(np.float32)).to(dtype).to(DEV)
                d = torch.empty((oh, ow, ch), dtype=dtype, device=DEV)
                pairs.append((s, d, f))
                specs.append((ih, iw, oh, ow, ch, f))
    ref = _per_image(pairs)
    for t in EDGE_TILES:
        tile = None if t is None else xr.tile(xr.XR_KERNEL_STRIP, t[0], t[1], 0, t[2])
        b = xr.Batch(pairs, tile=tile)
        for _, d, _ in pairs:
            d.fill_(3)
        b.run()
        torch.cuda.synchronize()
        for k, ((_, d, _), r) in enumerate(zip(pairs, ref)):
            assert torch.equal(d, r), f"tile {t}: job {k} {specs[k]} differs from the per-image launch"
    for k, ((s, d, f), sp) in enumerate(zip(pairs, specs)):
        ih, iw, oh, ow, ch, _ = sp
        rows = np.unique(np.array([0, oh // 2, oh - 1]))
        got = d[torch.from_numpy(rows).to(DEV)].cpu().numpy()[None]
        compare(got, s.cpu().numpy(), oh, ow, f, rows=rows, what=f"job {k} {sp}")


def test_batch_autotune_picks_a_candidate_and_keeps_results():
    jobs, pairs = _make_batch(seed=3, count=24, side_hi=512, content="field")
    ref = _per_image(pairs)
    b = xr.Batch(pairs)
    # the columns per thread are fixed per job kind (ppt_x is ignored)
    cands = [xr.tile(xr.XR_KERNEL_STRIP, 64, 4, 0, 8), xr.tile(xr.XR_KERNEL_STRIP, 256, 1, 0, 14),
             xr.tile(xr.XR_KERNEL_STRIP, 128, 2, 0, 30)]
    best, ms = b.autotune(candidates=cands, reps=2, groups=3)
    assert ms > 0 and best.as_tuple() in [c.as_tuple() for c in cands]
    for _, d, _ in pairs:
        d.zero_()
    b.run()
    torch.cuda.synchronize()
    assert all(torch.equal(d, r) for (_, d, _), r in zip(pairs, ref))
    # the built-in candidate list, then a batch prepared with the tuned default
    best, ms = b.autotune(reps=1, groups=1)
    assert ms > 0 and best.kernel == xr.XR_KERNEL_STRIP and best.ppt_x == 0
    b2 = xr.Batch(pairs)
    for _, d, _ in pairs:
        d.zero_()
    b2.run()
    torch.cuda.synchronize()
    assert all(torch.equal(d, r) for (_, d, _), r in zip(pairs, ref))


def test_prepare_validation():
    s = torch.zeros((8, 8, 1), dtype=torch.uint8, device=DEV)
    d = torch.zeros((16, 16, 1), dtype=torch.uint8, device=DEV)
    d16 = torch.zeros((16, 16, 1), dtype=torch.float16, device=DEV)
    s16 = torch.zeros((8, 8, 1), dtype=torch.float16, device=DEV)
    with pytest.raises(xr.XResizeError) as e:
        xr.Batch([(s, d, 0), (s16, d16, 1)])  # mixed dtypes
    assert e.value.code == 3
    with pytest.raises(xr.XResizeError) as e:
        xr.Batch([(s, d, 0), (s, d, 1)])  # two jobs write the same output
    assert e.value.code == 7
    b = xr.Batch([(s, d, 0)])
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with pytest.raises(xr.XResizeError) as e:
            with torch.cuda.graph(graph, stream=stream):
                xr.Batch([(s, d, 0)], stream=stream)
    assert e.value.code == 9
    torch.cuda.synchronize()
    b.run()
    torch.cuda.synchronize()
