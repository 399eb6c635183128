#!/usr/bin/env python3
"""Benchmark of the resize library on one MI355X.

Headline workload: Keys-bicubic (a = -1/2) x2 upscale of a 4096 x 4096 RGBA
uint8 image (synthetic smooth field) to 8192 x 8192, half-pixel centres,
clamp-to-edge, float32 weights and accumulation. One step = one resize of one
image; inputs and outputs rotate over >= 1 GiB of buffers so the 256 MB
Infinity Cache cannot hold the working set between steps.

Printed JSON line (one):
  value       output Gpixel/s over the K timed steps (wall clock, synchronised),
              submitted as replays of a HIP graph of the rotating launches
              (config.value_eager_launches: K steps launched one by one, each
              between HIP events, over their GPU time)
  roofline    the resize kernel's algorithmic bytes (each input pixel read once,
              each output pixel written once) per launch / its mean launch
              time from HIP event pairs around the eager launches (after an
              untimed pre-roll that leaves the GPU no idle gap), against the
              8 TB/s HBM3E peak; `traffic` is the HBM bytes per launch from
              the rocprofv3 counters in profiles/, or null if those were taken
              on other kernel sources
  cpu_baseline the FP64 C oracle on a bounded sample of output rows, timed on
              all host cores (the value) and on one thread, with the host's
              CPU model; the batched comparison and every extra row carry the
              oracle's rate on a sample of the same workload
  batched     256 uneven uint8 images: one persistent launch replayed from a
              HIP graph vs 256 per-image launches (eager and graph-captured),
              images/s, outputs bitwise identical across the three
  hbm_reference  plain torch fill and copy of 256 MiB: the bandwidth this
              GPU reaches with no arithmetic
  configs     the other configurations: C1 (bilinear x2 of a 512^2 uint8
              image), C2 (bicubic x2 and x0.5 of the 4096^2 RGBA image in
              uint8, float16 and float32), C4 (bilinear x2 of a float32 NCHW
              32x3x1024^2 tensor, forward and adjoint), C5 (bicubic x2 of a
              16384^2 float16 image, whole and in 16 row bands): algorithmic
              bytes, kernel time, fraction of the HBM peak, the oracle's rate;
              with --extras also the other filters and maps

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       [--no-batch] [--no-tune] [--no-configs] [--extras]
       python bench.py --paper-sweep   (the paper's tile experiment only)
       python bench.py --profile WORKLOAD [--steps N] [--tile ...] [--batch-tile ...]
                       (one workload, eager, fixed shape: what rocprofv3 runs)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 78.6  # non-packed FP32 FMA: 256 CUs x 64 lanes x 2 flops x 2.4 GHz
ROTATE_BYTES = 1 << 30
KERNEL_SOURCES = ["xr_forward.hip", "xr_backward.hip", "xr_device.hpp", "xr_buffer.hpp", "xr_internal.h"]
HEADLINE_PROFILE = "c2_bicubic_x2_u8_rgba.md"
# untimed launches before the per-launch statistics (see time_launches)
PREROLL_LAUNCHES = 500


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1001_1718_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_valu(name: str, tile, kernel_s: float):
    """VALU issue time per launch from a committed instruction-counter summary
    (SQ_INSTS_VALU x cycles per instruction / SIMDs / clock, between the
    two-cycle rate of VOP2 multiply-adds and the four-cycle rate of the
    conversions), when it was taken on these kernel sources; else None. The
    summary's launch shape is reported with it."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        if vals.get("kernel_sources_sha256_16") != kernel_hash():
            return None
        # the counters were taken with the summary's launch shape; the
        # instruction count of another strip height differs by its prologue
        insts = int(vals["SQ_INSTS_VALU"])
        per_cycle = int(vals["simds"]) * float(vals["clock_ghz"]) * 1e9
        slow = insts * int(vals["cycles_per_valu_inst"]) / per_cycle
        fast = insts * int(vals["cycles_per_valu_inst_fast"]) / per_cycle
        return {"valu_insts_per_launch": insts, "profile_tile": vals["tile"],
                "issue_us_range": [round(fast * 1e6, 1), round(slow * 1e6, 1)],
                "issue_frac_range": [round(fast / kernel_s, 3), round(slow / kernel_s, 3)]}
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def read_pmc(name: str):
    """HBM traffic per launch from a committed rocprofv3 counter summary."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        if vals.get("kernel_sources_sha256_16") != kernel_hash():
            return None
        fetch = float(vals["fetch_kib_per_dispatch"]) * 1024.0
        write = float(vals["write_kib_per_dispatch"]) * 1024.0
        f_fetch = float(vals["copy_bytes"]) / (float(vals["copy_fetch_kib"]) * 1024.0)
        f_write = float(vals["copy_bytes"]) / (float(vals["copy_write_kib"]) * 1024.0)
        return fetch * f_fetch + write * f_write
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def profile_fields(name, alg, seconds=None):
    """The profiles/ summary of a configuration's kernel: its name and, when it
    was taken on these kernel sources, the HBM bytes per launch it measured
    (traffic), their ratio to the algorithmic bytes and, given the launch
    time, those bytes per second (measured_gbs)."""
    if not name or not os.path.exists(os.path.join(ROOT, "profiles", name)):
        return {}
    traffic = read_pmc(name)
    out = {"profile": name, "traffic": None if traffic is None else int(traffic),
           "traffic_over_alg": None if traffic is None else round(traffic / alg, 3)}
    if traffic is not None and seconds:
        out["measured_gbs"] = round(traffic / seconds / 1e9, 1)
    return out


def time_launches(launch, n_buffers: int, steps: int, warmup: int, torch):
    """Per-launch statistics: at least PREROLL_LAUNCHES (or `warmup`, if
    more) untimed launches, then `steps` launches each bracketed by HIP
    events, rotating over buffers, with no synchronisation between the two
    (the GPU runs about 10-20% slower for the first 10-20 ms after it has
    idled, even briefly: measured on the headline, the first groups of 100
    ran 66-73 us against 52-57 us later whenever a synchronisation preceded
    them, and 51-55 us throughout after 500 launches without one). Returns
    (GPU seconds of the timed launches, first start to last end; list of
    per-launch event times in ms). The events are created (recorded once)
    before the warm-up."""
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for e in starts + ends:
        e.record()
    for i in range(max(warmup, PREROLL_LAUNCHES)):
        launch(i % n_buffers)
    for i in range(steps):
        starts[i].record()
        launch(i % n_buffers)
        ends[i].record()
    torch.cuda.synchronize()
    # GPU time from the first launch's start to the last one's end: for
    # launches of a few microseconds this is the back-to-back rate, which
    # per-launch event pairs (dominated by dispatch latency) overstate
    time_launches.span_ms = starts[0].elapsed_time(ends[-1])
    return time_launches.span_ms / 1e3, [s.elapsed_time(e) for s, e in zip(starts, ends)]


def graph_steps(launch, n_buffers: int, steps: int, torch) -> float:
    """Wall seconds of exactly `steps` launches submitted as replays of one
    HIP graph holding the n_buffers rotating launches (any remainder eager),
    bracketed by device synchronisation; one untimed replay first. The HIP
    events recorded on the replaying stream around the same steps give
    graph_steps.event_ms, their GPU time."""
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            for i in range(n_buffers):
                launch(i)
    torch.cuda.current_stream().wait_stream(stream)
    graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps // n_buffers):
        graph.replay()
    for i in range(steps % n_buffers):
        launch(i)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph_steps.event_ms = e0.elapsed_time(e1)
    del graph
    return wall


def graph_launch_us(launch, n_buffers: int, torch, reps: int = 100) -> float:
    """Microseconds per launch of `reps` launches captured in one HIP graph
    and replayed: no host submission between kernels, so for launches of a
    few microseconds this is the kernel rate that per-launch events (which
    then include the host's submission gap) overstate."""
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            for i in range(reps):
                launch(i % n_buffers)
    torch.cuda.current_stream().wait_stream(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # untimed replays first, with no synchronisation before the timed one
    # (the GPU runs slower for a while after idling; see time_launches)
    for _ in range(5):
        graph.replay()
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    del graph
    return e0.elapsed_time(e1) / reps * 1e3


def group_stats(ms, group: int = 100):
    groups = [ms[i:i + group] for i in range(0, len(ms), group) if len(ms[i:i + group]) == group]
    if not groups:
        groups = [ms]
    means = [sum(g) / len(g) for g in groups]
    return {"groups": len(groups), "median_ms": statistics.median(means), "min_ms": min(means),
            "max_ms": max(means), "mean_ms": sum(ms) / len(ms),
            "group_means_ms": [round(m, 5) for m in means]}


def headline(args, torch, xr, fields):
    dev = torch.device("cuda:0")
    in_hw, out_hw, ch = 4096, 8192, 4
    in_bytes, out_bytes = in_hw * in_hw * ch, out_hw * out_hw * ch
    n_buf = max(1, math.ceil(ROTATE_BYTES / (in_bytes + out_bytes)))
    log(f"generating {n_buf} rotating 4096x4096 RGBA uint8 inputs")
    base = fields.field_u8_torch(in_hw, in_hw, ch, 1002, dev)
    srcs = [base] + [base.clone() for _ in range(n_buf - 1)]
    dsts = [torch.empty((out_hw, out_hw, ch), dtype=torch.uint8, device=dev) for _ in range(n_buf)]

    tile = None
    tune = None
    if args.tile:
        xr.set_tile("bicubic", xr.XR_U8, ch, in_hw, in_hw, out_hw, out_hw,
                    xr.tile(*(int(v) for v in args.tile.split(","))))
    elif not args.no_tune:
        cands = [c for c in xr.tune_candidates("bicubic", xr.XR_U8, ch, in_hw, in_hw, out_hw, out_hw)
                 if c.kernel in (xr.XR_KERNEL_STRIP, xr.XR_KERNEL_STRIP_LDS)]
        t0 = time.perf_counter()
        tile, best_ms = xr.autotune(srcs, dsts, "bicubic", candidates=cands, reps=8, groups=3)
        tune = {"candidates": len(cands), "seconds": round(time.perf_counter() - t0, 2),
                "best_ms": round(best_ms, 5)}
        log(f"autotune picked {tile} at {best_ms * 1e3:.1f} us per launch ({len(cands)} candidates)")
    resolved = xr.get_tile("bicubic", xr.XR_U8, ch, in_hw, in_hw, out_hw, out_hw)

    def launch(i):
        xr.resize_into(srcs[i], dsts[i], "bicubic")

    log(f"timing {args.steps} steps after {args.warmup} warm-up steps")
    # kernel statistics: each launch bracketed by HIP events on its stream
    wall_eager, ms = time_launches(launch, n_buf, args.steps, args.warmup, torch)
    stats = group_stats(ms)
    # the reported value: the same K steps replayed from a HIP graph of the
    # rotating launches (how a serving loop would submit them: no host work
    # between kernels)
    wall = graph_steps(launch, n_buf, args.steps, torch)
    out_px = out_hw * out_hw
    value = out_px * args.steps / wall / 1e9
    # the roofline's launch time: the mean of the HIP event pairs around each
    # eager launch, on its stream (the kernel and its dispatch); the same steps
    # replayed from the graph, timed by events around the replays, run about
    # 3% longer per launch (kernel_ms.graph_replay_mean_ms)
    graph_ms = graph_steps.event_ms / args.steps
    kernel_s = stats["mean_ms"] / 1e3
    alg = in_bytes + out_bytes
    achieved = alg / kernel_s / 1e9
    traffic = read_pmc(HEADLINE_PROFILE)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                # the HBM bytes the counters measured, over the same launch time
                "measured_gbs": None if traffic is None else round(traffic / kernel_s / 1e9, 1),
                "alg_bytes_per_launch": alg,
                "kernel_ms": {"graph_replay_mean_ms": round(graph_ms, 5),
                              "event_pairs": {k: (round(v, 5) if isinstance(v, float) else v)
                                              for k, v in stats.items()}},
                "kernel_gpixel_s": round(out_px / kernel_s / 1e9, 2),
                # the FP32 VALU check: instruction issue time from the counters
                "valu": read_valu(HEADLINE_PROFILE, resolved, kernel_s),
                "profile": HEADLINE_PROFILE,
                # and the algorithmic arithmetic rate: separable Keys x2 takes 24
                # FP32 multiply-adds per output pixel (4 taps x 4 channels
                # vertically, half that horizontally per output row), against
                # the non-packed FP32 peak (256 CUs x 64 lanes x 2 flops x 2.4 GHz)
                "fp32": {"fma_per_px": 24,
                         "achieved_tflops": round(2 * 24 * out_px / kernel_s / 1e12, 2),
                         "peak_tflops": FP32_PEAK_TFLOPS,
                         "frac": round(2 * 24 * out_px / kernel_s / 1e12 / FP32_PEAK_TFLOPS, 4)}}
    return {
        "value": value, "wall": wall, "value_eager": out_px * args.steps / wall_eager / 1e9,
        "roofline": roofline, "tile": repr(resolved), "tune": tune,
        "n_buf": n_buf, "src_host": srcs[0].cpu().numpy(),
    }


def hbm_reference(torch, reps: int = 100):
    """Plain torch kernels as achievable-bandwidth reference lines for this
    GPU: a 256 MiB fill (write only) and a 256 MiB device copy. Two rotating
    buffers exceed the 256 MB Infinity Cache. Timed after 300 untimed calls
    that run straight into the timed ones (the GPU runs slower for a while
    after idling; see time_launches)."""
    dev = torch.device("cuda:0")
    n = 256 << 20
    bufs = [torch.empty(n, dtype=torch.uint8, device=dev) for _ in range(3)]

    def timed(fn):
        for k in range(300):
            fn(k & 1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(reps):
            fn(k & 1)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    res = {}
    t = timed(lambda k: bufs[k].fill_(3))
    res["fill_256MiB_gbs"] = round(n / t / 1e9, 1)
    t = timed(lambda k: bufs[k].copy_(bufs[2]))
    res["copy_256MiB_gbs"] = round(2 * n / t / 1e9, 1)
    del bufs
    torch.cuda.empty_cache()
    return res


def host_cpu() -> dict:
    """The host's CPU model and core count (for the oracle timings)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_baseline_sample(planes, out_h: int, out_w: int, mode: str, target_s: float, threads: int = 0,
                        mapping: str = "half_pixel"):
    """The oracle on evenly spaced output rows of one workload, sized to about
    target_s seconds: returns (output pixels per second, rows, passes, threads).

    planes: host array (P, H, W, C); the rate counts output pixels of one plane
    (H x W x C values make one pixel when C is interleaved). Bilinear and
    bicubic with pixel centres run the C oracle (OpenMP, `threads` = 0: all);
    the other filters and maps run the numpy oracle (one thread)."""
    from oracle import ref_c
    from oracle import ref_resize as R
    from oracle.build import LIBRARY, build_oracle
    import numpy as np

    codes = {"bilinear": 0, "bicubic": 1, "nearest": 2, "bilinear_aa": 3, "bicubic_aa": 4}
    filt = codes[mode]
    use_c = filt in (0, 1) and mapping == "half_pixel"
    if use_c and not os.path.exists(LIBRARY):
        build_oracle()
    used = (ref_c.max_threads() if threads == 0 else threads) if use_c else 1
    if use_c:  # the C oracle reads float32 planes: convert (exactly) once, outside the timing
        planes = np.ascontiguousarray(np.asarray(planes).astype(np.float32))

    def run(n_rows):
        rows = np.linspace(0, out_h - 1, n_rows).astype(np.int64)
        t0 = time.perf_counter()
        if use_c:
            ref_c.resize_rows(planes, out_h, out_w, rows, filt, threads=threads)
        elif filt in (3, 4):
            R.resize_antialiased(planes, out_h, out_w, filt, rows=rows)
        else:
            R.resize_rows(planes, out_h, out_w, rows, filt, mapping=1 if mapping == "paper" else 0)
        return time.perf_counter() - t0

    probe = min(4, out_h)
    t = run(probe)
    n_rows = int(min(out_h, max(probe, probe * target_s / max(t, 1e-6))))
    passes = 1
    if n_rows < out_h:
        t = run(n_rows)
    else:
        t1 = run(out_h)
        passes = max(1, int(target_s / max(t1, 1e-6)))
        t = t1 + sum(run(out_h) for _ in range(passes - 1))
    px = n_rows * out_w * passes * planes.shape[0]
    return px / t, n_rows, passes, used, t


def cpu_baseline_adjoint(grad, in_h: int, in_w: int, mode: str):
    """The oracle adjoint (FP64 C, OpenMP over planes) of as many whole planes
    of the NCHW gradient tensor `grad` as it has threads: gradient pixels per
    second, the cores used and the seconds taken."""
    from oracle import ref_c
    from oracle.build import LIBRARY, build_oracle

    if not os.path.exists(LIBRARY):
        build_oracle()
    k = min(ref_c.max_threads(), grad.shape[0] * grad.shape[1])
    grad_planes = grad.reshape(-1, grad.shape[-2], grad.shape[-1])[:k].float().cpu().numpy()[..., None]
    t0 = time.perf_counter()
    ref_c.adjoint(grad_planes, in_h, in_w, 1 if mode == "bicubic" else 0)
    t = time.perf_counter() - t0
    return grad_planes.shape[0] * in_h * in_w / t, min(ref_c.max_threads(), grad_planes.shape[0]), t


def cpu_baseline_batch(jobs, srcs_host, rows_per_image: int = 2):
    """The oracle on `rows_per_image` evenly spaced output rows of every image
    of a batch, extrapolated to the whole batch: images per second."""
    import numpy as np

    from oracle import ref_c

    total = 0.0
    for j, host in zip(jobs, srcs_host):
        planes = np.ascontiguousarray(host[None].astype(np.float32))  # widened outside the timing
        mode = "bicubic" if j.filter == 1 else "bilinear"
        n = min(rows_per_image, j.out_h)
        rows = np.linspace(0, j.out_h - 1, n).astype(np.int64)
        t0 = time.perf_counter()
        ref_c.resize_rows(planes, j.out_h, j.out_w, rows, 1 if mode == "bicubic" else 0)
        total += (time.perf_counter() - t0) * j.out_h / n
    return len(jobs) / total


def cpu_baseline(src_host, target_s: float = 10.0):
    """The FP64 C oracle on the headline workload: all host cores (the
    reported value), then one thread on a smaller sample."""
    planes = src_host[None]
    rate, n_rows, passes, used, t = cpu_baseline_sample(planes, 8192, 8192, "bicubic", target_s)
    rate1, rows1, _, _, t1 = cpu_baseline_sample(planes, 8192, 8192, "bicubic", target_s / 4, threads=1)
    px = n_rows * 8192 * passes
    what = (f"{n_rows} evenly spaced output rows" if passes == 1 else
            f"the whole 8192 x 8192 output, {passes} passes")
    return {"value": round(rate / 1e9, 6), "unit": "Gpixel/s", "cores": used, "kind": "oracle",
            "seconds": round(t, 2),
            "sample": f"{what} of the bicubic x2 4096x4096 RGBA uint8 workload "
                      f"({px / 1e6:.1f} Mpx), FP64 C oracle, OpenMP, input widened to float32 "
                      f"before timing",
            "one_thread": {"value": round(rate1 / 1e9, 6), "unit": "Gpixel/s", "seconds": round(t1, 2),
                           "sample": f"{rows1} evenly spaced output rows"},
            **host_cpu()}


def touched_rows(n_in: int, n_out: int, taps: int) -> int:
    """Source rows (or columns) that some output row (column) reads: the union over
    output indices y of the clamped taps y0 - lo .. y0 - lo + K - 1 with
    y0 = floor((2 y + 1) n_in / (2 n_out) - 1/2) (eqs. 1-4). Every row when
    the tap windows overlap or touch; fewer when shrinking by more than K."""
    lo = 1 if taps == 4 else 0
    rows = set()
    for y in range(n_out):
        y0 = ((2 * y + 1) * n_in - n_out) // (2 * n_out)
        for j in range(taps):
            rows.add(min(max(y0 - lo + j, 0), n_in - 1))
    return len(rows)


def batch_alg_bytes(jobs) -> int:
    """Algorithmic bytes of a batch: every output pixel written once and every
    source pixel that some output pixel reads read once (the touched rows
    times the touched columns, touched_rows on each axis)."""
    total = 0
    for j in jobs:
        taps = 4 if j.filter == 1 else 2
        touched = touched_rows(j.in_h, j.out_h, taps) * touched_rows(j.in_w, j.out_w, taps)
        total += touched * j.channels + j.out_h * j.out_w * j.channels
    return total


def batched(torch, xr, fields, reps: int = 20, cpu: bool = True):
    dev = torch.device("cuda:0")
    jobs = fields.batch_jobs(0)
    log("generating the 256-image uneven batch (sides 64..2048, scales 0.25..4)")
    pairs = []
    for j in jobs:
        s = fields.field_u8_torch(j.in_h, j.in_w, j.channels, j.content_seed, dev)
        d = torch.empty((j.out_h, j.out_w, j.channels), dtype=torch.uint8, device=dev)
        pairs.append((s, d, j.filter))
    out_px = sum(j.out_h * j.out_w for j in jobs)
    alg = batch_alg_bytes(jobs)

    def per_image():
        for s, d, f in pairs:
            xr.resize_into(s, d, f)

    def timed(run, warm):
        """Seconds per call of `run`: `warm` untimed calls, then `reps`
        calls between HIP events, with no synchronisation in between (the
        GPU runs slower for a while after idling; see time_launches)."""
        for _ in range(warm):
            run()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    res = {}
    # (ii) eager per-image launches
    per_image()
    torch.cuda.synchronize()
    ref = [d.clone() for _, d, _ in pairs]
    res["per_image_eager"] = len(pairs) / timed(per_image, 4)

    stream = torch.cuda.Stream()
    # (iii) the 256 launches captured in one graph
    g_multi = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g_multi, stream=stream):
            for s, d, f in pairs:
                xr.resize_into(s, d, f, stream=stream)
    torch.cuda.synchronize()
    g_multi.replay()
    torch.cuda.synchronize()
    eq_multi = all(torch.equal(d, r) for (_, d, _), r in zip(pairs, ref))
    res["per_image_graph"] = len(pairs) / timed(g_multi.replay, 4)

    # (i) one persistent launch over every tile, shape from the batch
    # autotuner, captured in a graph
    for _, d, _ in pairs:
        d.zero_()
    b = xr.Batch(pairs)
    t0 = time.perf_counter()
    tile, tune_ms = b.autotune()
    tune = {"tile": repr(tile), "best_ms": round(tune_ms, 4), "seconds": round(time.perf_counter() - t0, 2)}
    for _, d, _ in pairs:
        d.zero_()
    g_one = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g_one, stream=stream):
            b.run(stream=stream)
    torch.cuda.synchronize()
    g_one.replay()
    torch.cuda.synchronize()
    eq_one = all(torch.equal(d, r) for (_, d, _), r in zip(pairs, ref))
    launch_s = timed(g_one.replay, 15)
    res["persistent_graph"] = len(pairs) / launch_s
    launch_ms = launch_s * 1e3
    cpu_res = {}
    if cpu:
        log("timing the oracle on 2 rows of every image (extrapolated)")
        ips = cpu_baseline_batch(jobs, [s.cpu().numpy() for s, _, _ in pairs])
        cpu_res = {"cpu_images_per_s": round(ips, 3), "cpu_sample": "2 evenly spaced output rows per image, "
                   "extrapolated to whole images (FP64 C oracle, all host cores)"}
    return {
        **cpu_res,
        "workload": "256 uint8 images (1 or 4 ch), sides U{64..2048}, per-axis scale U(0.25, 4), "
                    "128 bilinear + 128 bicubic, smooth-field content, seed 0",
        "images_per_s": {k: round(v, 1) for k, v in res.items()},
        "speedup_vs_eager": round(res["persistent_graph"] / res["per_image_eager"], 3),
        "speedup_vs_graph": round(res["persistent_graph"] / res["per_image_graph"], 3),
        "bitwise_equal": bool(eq_multi and eq_one),
        "autotune": tune,
        "output_gpixel": round(out_px / 1e9, 3),
        "persistent_ms": round(launch_ms, 4),
        "persistent_gbs": round(alg / (launch_ms / 1e3) / 1e9, 1),
        "alg_bytes": alg,
        "hbm_frac": round(alg / (launch_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        **profile_fields("c3_batch_256_uneven_u8.md", alg, launch_ms / 1e3),
    }


def configs(torch, xr, fields, steps: int = 50, warmup: int = 5, cpu: bool = True, breadth: bool = False):
    """Every configuration of the workload table besides the headline and the
    batch (C1, C2 in three storage types and both directions, C4 forward and
    adjoint, C5 whole and in row bands): per launch the algorithmic bytes,
    the mean kernel time from HIP events, GB/s and the fraction of the HBM
    peak (and that fraction at the per-launch time of a HIP graph replay,
    graph_hbm_frac: per-launch events add microseconds of submission to the
    small kernels), the tuned launch shape, and the oracle's rate on a sample of the
    same workload (about 1 s of host time; `cpu_mpx_s`, the cores it used and
    its sample) unless cpu is False. `profile` names the rocprofv3 summary in
    profiles/ of the configuration's kernel. With breadth, also the other
    filters and maps and two more adjoints."""
    dev = torch.device("cuda:0")
    out = {"C1": {}, "C2": {}, "C4": {}, "C5": {}}
    if breadth:
        out["breadth"] = {}

    def oracle_rate(src, out_hw, mode, layout, mapping="half_pixel"):
        if not cpu:
            return {}
        host = src.cpu().numpy()
        if layout == "hwc":
            planes = host[None] if host.ndim == 3 else host[None, :, :, None]
        else:  # planar: one plane stands for all
            planes = host.reshape(-1, host.shape[-2], host.shape[-1], 1)[:1]
        rate, n_rows, passes, used, _ = cpu_baseline_sample(planes, out_hw[0], out_hw[1], mode, 1.0,
                                                            mapping=mapping)
        return {"cpu_mpx_s": round(rate / 1e6, 3), "cpu_cores": used,
                "cpu_sample": f"{n_rows} rows x {passes} passes" if passes > 1 else f"{n_rows} rows"}

    def measure(group, name, make_src, out_shape, mode, layout="hwc", mapping="half_pixel", rotate=True,
                all_kinds=False, profile=None):
        src0 = make_src()
        in_bytes = src0.numel() * src0.element_size()
        out_bytes = math.prod(out_shape) * src0.element_size()
        # rotate over >= 1 GiB of buffers so the 256 MB Infinity Cache cannot
        # hold the working set between launches (unless rotate is False)
        n_buf = max(1, math.ceil(ROTATE_BYTES / (in_bytes + out_bytes))) if rotate else 1
        srcs = [src0] + [src0.clone() for _ in range(n_buf - 1)]
        dsts = [torch.empty(out_shape, dtype=src0.dtype, device=dev) for _ in range(n_buf)]

        chans = src0.shape[-1] if layout == "hwc" and src0.dim() == 3 else 1
        in_hw = src0.shape[:2] if layout == "hwc" else src0.shape[-2:]
        out_hw = out_shape[:2] if layout == "hwc" else out_shape[-2:]
        # the antialiased filters and tiny images: the library's own list
        # (with the gather shapes); the others: strip shapes
        cands = None if (mode.endswith("_aa") or all_kinds) else [
            c for c in xr.tune_candidates(mode, xr._DTYPES[src0.dtype], chans, in_hw[1], in_hw[0],
                                          out_hw[1], out_hw[0])
            if c.kernel in (xr.XR_KERNEL_STRIP, xr.XR_KERNEL_STRIP_LDS)]
        tile, _ = xr.autotune(srcs, dsts, mode, layout=layout, candidates=cands, reps=4, groups=3)

        def launch(i):
            xr.resize_into(srcs[i], dsts[i], mode, layout=layout, mapping=mapping)

        wall, ms = time_launches(launch, n_buf, steps, warmup, torch)
        k_s = sum(ms) / len(ms) / 1e3
        g_us = graph_launch_us(launch, n_buf, torch)
        # pixels: H * W for interleaved images, N * C * H * W for planar tensors
        px = math.prod(out_shape[:2]) if layout == "hwc" else math.prod(out_shape)
        alg = in_bytes + out_bytes
        out[group][name] = {
            "alg_bytes": alg, "kernel_us": round(k_s * 1e6, 2), "gbs": round(alg / k_s / 1e9, 1),
            "hbm_frac": round(alg / k_s / 1e9 / HBM_PEAK_GBS, 4), "gpixel_s": round(px / k_s / 1e9, 2),
            "tile": repr(tile), "buffers": n_buf,
            "back_to_back_us": round(time_launches.span_ms / steps * 1e3, 2), "graph_us": round(g_us, 2),
            "graph_hbm_frac": round(alg / (g_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            **profile_fields(profile, alg, k_s),
            **oracle_rate(src0, out_hw, mode, layout, mapping)}
        log(f"{group} {name}: {out[group][name]}")
        del srcs, dsts
        torch.cuda.empty_cache()

    measure("C1", "bilinear_x2_u8_512_rotating",
            lambda: torch.randint(0, 256, (512, 512), dtype=torch.uint8, device=dev), (1024, 1024), "bilinear",
            all_kinds=True, profile="c1_bilinear_x2_u8_512.md")
    measure("C1", "bilinear_x2_u8_512_same_buffers",
            lambda: torch.randint(0, 256, (512, 512), dtype=torch.uint8, device=dev), (1024, 1024), "bilinear",
            rotate=False, all_kinds=True)
    fld = fields.smooth_field_torch(4096, 4096, 4, 1002, dev)
    unit = torch.clamp(fld / 255.0, 0.0, 1.0)
    u8 = torch.clamp(torch.round(fld), 0, 255).to(torch.uint8)
    del fld
    for dname, t in [("u8", u8), ("f16", unit.half()), ("f32", unit.float())]:
        for direction, n, tag in [("x2", 8192, "x2"), ("x0.5", 2048, "x05")]:
            measure("C2", f"bicubic_{direction}_{dname}_rgba", lambda t=t: t, (n, n, 4), "bicubic",
                    profile=f"c2_bicubic_{tag}_{dname}_rgba.md")
    if breadth:
        measure("breadth", "nearest_x2_u8_rgba", lambda: u8, (8192, 8192, 4), "nearest")
        measure("breadth", "bicubic_aa_x0.5_u8_rgba", lambda: u8, (2048, 2048, 4), "bicubic_aa")
        measure("breadth", "bilinear_aa_x0.25_u8_rgba", lambda: u8, (1024, 1024, 4), "bilinear_aa")
        measure("breadth", "bilinear_paper_map_x2_u8_rgba", lambda: u8, (8192, 8192, 4), "bilinear",
                mapping="paper")
        measure("breadth", "bicubic_paper_map_x3_u8_rgba", lambda: u8, (12288, 12288, 4), "bicubic",
                mapping="paper")
    del unit, u8
    torch.cuda.empty_cache()
    measure("C4", "bilinear_x2_f32_nchw_forward", lambda: torch.randn((32, 3, 1024, 1024), device=dev),
            (32, 3, 2048, 2048), "bilinear", layout="nchw", profile="c4_bilinear_x2_f32_forward.md")

    # the adjoint: float32 (the configuration); with breadth, float16
    # gradients and a non-dyadic scale (owner-computes kernel)
    def adjoint(group, name, g_shape, in_hw, mode, dtype, profile=None):
        g = torch.randn(g_shape, device=dev).to(dtype)
        gs = torch.empty(g_shape[:2] + in_hw, device=dev, dtype=dtype)

        def bwd(i):
            xr.resize_backward(g, in_hw, mode, out=gs)

        wall, ms = time_launches(bwd, 1, 20, 3, torch)
        k_s = sum(ms) / len(ms) / 1e3
        alg = (g.numel() + gs.numel()) * g.element_size()
        out[group][name] = {
            "alg_bytes": alg, "kernel_us": round(k_s * 1e6, 2), "gbs": round(alg / k_s / 1e9, 1),
            "hbm_frac": round(alg / k_s / 1e9 / HBM_PEAK_GBS, 4), "gpixel_s": round(gs.numel() / k_s / 1e9, 2),
            **profile_fields(profile, alg, k_s)}
        if cpu:
            rate, used, t = cpu_baseline_adjoint(g, in_hw[0], in_hw[1], mode)
            out[group][name].update({"cpu_mpx_s": round(rate / 1e6, 3), "cpu_cores": used,
                                     "cpu_sample": f"{used} whole planes"})
        log(f"{group} {name}: {out[group][name]}")
        del g, gs
        torch.cuda.empty_cache()

    adjoint("C4", "bilinear_x2_f32_nchw_adjoint", (32, 3, 2048, 2048), (1024, 1024), "bilinear", torch.float32,
            profile="c4_bilinear_x2_f32_adjoint.md")
    if breadth:
        adjoint("breadth", "bilinear_x2_f16_nchw_adjoint", (32, 3, 2048, 2048), (1024, 1024), "bilinear",
                torch.float16)
        adjoint("breadth", "bicubic_x1.5_f32_nchw_adjoint", (32, 3, 1536, 1536), (1024, 1024), "bicubic",
                torch.float32)
    # C5: 16384^2 FP16 -> 32768^2, whole image and 16 row bands (the shape
    # tuned on the whole image; the bands share its key)
    src = torch.clamp(fields.smooth_field_torch(16384, 16384, 1, 1005, dev)[:, :, 0] / 255.0, 0, 1).half()
    dst = torch.empty((32768, 32768), dtype=torch.float16, device=dev)
    dst_b = torch.empty_like(dst)
    cands = [c for c in xr.tune_candidates("bicubic", xr.XR_F16, 1, 16384, 16384, 32768, 32768)
             if c.kernel == xr.XR_KERNEL_STRIP]
    c5_tile, _ = xr.autotune(src, dst, "bicubic", candidates=cands, reps=2, groups=3)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # about 15 ms of untimed launches straight into the timed ones (the GPU
    # runs slower for a while after idling; see time_launches)
    for _ in range(30):
        xr.resize_into(src, dst, "bicubic")
    ev[0].record()
    for _ in range(10):
        xr.resize_into(src, dst, "bicubic")
    ev[1].record()
    ev[2].record()
    for b in range(16):
        r0 = b * 2048
        first, last = xr.needed_rows(16384, 32768, r0, 2048, "bicubic")
        xr.resize_into(src[first:last + 1], dst_b[r0:r0 + 2048], "bicubic", src_row0=first,
                       src_height=16384, dst_row0=r0, dst_height=32768)
    ev[3].record()
    torch.cuda.synchronize()
    whole = ev[0].elapsed_time(ev[1]) / 10 / 1e3
    bands = ev[2].elapsed_time(ev[3]) / 1e3
    alg = (src.numel() + dst.numel()) * 2
    out["C5"]["bicubic_x2_f16_16384"] = {
        "alg_bytes": alg, "kernel_us": round(whole * 1e6, 1), "bands16_us": round(bands * 1e6, 1),
        "tile": repr(c5_tile),
        "gbs": round(alg / whole / 1e9, 1), "hbm_frac": round(alg / whole / 1e9 / HBM_PEAK_GBS, 4),
        "bands_gbs": round(alg / bands / 1e9, 1), "bands_bitwise_equal": bool(torch.equal(dst, dst_b)),
        **profile_fields("c5_bicubic_x2_f16_16384.md", alg, whole),
        **oracle_rate(src, (32768, 32768), "bicubic", "hwc")}
    log(f"C5: {out['C5']['bicubic_x2_f16_16384']}")
    del src, dst, dst_b
    torch.cuda.empty_cache()
    return out


def profile_workload(args, torch, xr, fields):
    """One workload launched eagerly `--steps` times with a fixed launch shape
    (the library default, or --tile / --batch-tile; for the 96-plane C4
    tensor the --tile shape is stored by a one-candidate tuning), nothing
    captured in a graph: the command the rocprofv3 summaries in profiles/ are
    taken with. Prints one JSON line with the mean launch time from HIP
    events and the algorithmic bytes per launch."""
    dev = torch.device("cuda:0")
    name = args.profile
    steps = args.steps

    def fix_tile(mode, dtype, channels, in_w, in_h, out_w, out_h):
        if args.tile:
            xr.set_tile(mode, dtype, channels, in_w, in_h, out_w, out_h,
                        xr.tile(*(int(v) for v in args.tile.split(","))))

    if name == "copy":  # counter calibration: a plain 1 GiB device copy
        a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        launch, alg = (lambda i: b.copy_(a)), 2 << 30
    elif name == "batch":
        # every job's source is a crop of one 2048 x 2048 field (the same
        # sizes and work as the benchmark's batch): a few hundred generating
        # dispatches instead of tens of thousands, which rocprofv3 counter
        # collection has not survived
        jobs = fields.batch_jobs(0)
        base = fields.field_u8_torch(2048, 2048, 4, 7, dev)
        pairs = []
        for j in jobs:
            s = base[:j.in_h, :j.in_w, :j.channels].contiguous()
            d = torch.empty((j.out_h, j.out_w, j.channels), dtype=torch.uint8, device=dev)
            pairs.append((s, d, j.filter))
        tile = xr.tile(*(int(v) for v in args.batch_tile.split(","))) if args.batch_tile else None
        b = xr.Batch(pairs, tile=tile)
        launch, alg = (lambda i: b.run()), batch_alg_bytes(jobs)
    elif name in ("c4_fwd", "c4_adjoint"):
        x = torch.randn((32, 3, 1024, 1024), device=dev)
        g = torch.randn((32, 3, 2048, 2048), device=dev)
        if name == "c4_fwd":
            y = torch.empty_like(g)
            if args.tile:  # (a shape for 96 planes: stored by a one-candidate tuning)
                xr.autotune([x], [y], "bilinear", layout="nchw", reps=1, groups=1,
                            candidates=[xr.tile(*(int(v) for v in args.tile.split(",")))])
            launch = lambda i: xr.resize_into(x, y, "bilinear", layout="nchw")
        else:
            gx = torch.empty_like(x)
            launch = lambda i: xr.resize_backward(g, (1024, 1024), "bilinear", out=gx)
        alg = (x.numel() + g.numel()) * 4
    elif name == "c5":
        src = torch.clamp(fields.smooth_field_torch(16384, 16384, 1, 1005, dev)[:, :, 0] / 255.0, 0, 1).half()
        dst = torch.empty((32768, 32768), dtype=torch.float16, device=dev)
        fix_tile("bicubic", xr.XR_F16, 1, 16384, 16384, 32768, 32768)
        launch, alg = (lambda i: xr.resize_into(src, dst, "bicubic")), (src.numel() + dst.numel()) * 2
    elif name == "c1":
        src = torch.randint(0, 256, (512, 512), dtype=torch.uint8, device=dev)
        dst = torch.empty((1024, 1024), dtype=torch.uint8, device=dev)
        fix_tile("bilinear", xr.XR_U8, 1, 512, 512, 1024, 1024)
        launch, alg = (lambda i: xr.resize_into(src, dst, "bilinear")), 512 * 512 + 1024 * 1024
    else:  # C2: x2 / x05, storage u8 / f16 / f32, bicubic RGBA 4096^2
        direction, _, dname = name.partition("_")
        n = {"x2": 8192, "x05": 2048}[direction]
        fld = fields.smooth_field_torch(4096, 4096, 4, 1002, dev)
        if dname in ("", "u8"):
            src = torch.clamp(torch.round(fld), 0, 255).to(torch.uint8)
        else:
            src = torch.clamp(fld / 255.0, 0.0, 1.0).to({"f16": torch.float16, "f32": torch.float32}[dname])
        del fld
        n_buf = max(1, math.ceil(ROTATE_BYTES / (src.numel() * src.element_size() * (1 + (n / 4096) ** 2))))
        srcs = [src] + [src.clone() for _ in range(n_buf - 1)]
        dsts = [torch.empty((n, n, 4), dtype=src.dtype, device=dev) for _ in range(n_buf)]
        fix_tile("bicubic", xr._DTYPES[src.dtype], 4, 4096, 4096, n, n)
        launch = lambda i: xr.resize_into(srcs[i % n_buf], dsts[i % n_buf], "bicubic")
        alg = (4096 * 4096 + n * n) * 4 * src.element_size()
    for i in range(3):
        launch(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        launch(i)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    print(json.dumps({"profile": name, "launches": steps + 3, "timed_launches": steps,
                      "mean_ms": round(ms, 5), "alg_bytes": alg,
                      "gbs": round(alg / ms / 1e6, 1), "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}),
          flush=True)


PAPER_SHAPES = [(8, 8), (32, 4), (32, 16), (4, 8), (8, 4)]


def paper_sweep(torch, xr, fields, reps: int = 10, groups: int = 3):
    """The paper's tile-shape experiment on this GPU: bilinear resize of an
    800 x 800 image (smooth-field stand-in, RGBA uint8) by 2, 4, 6, 8 and 10,
    every output pixel one thread in a block_w x block_h block (the paper's
    own tiling, eq. 6) for the paper's shapes and a few wider ones, next to
    the strip walks. Median of `groups` groups of `reps` launches per shape,
    rotating over enough buffers to exceed the Infinity Cache."""
    dev = torch.device("cuda:0")
    src0 = fields.field_u8_torch(800, 800, 4, 1001, dev)
    gather = PAPER_SHAPES + [(16, 16), (64, 4), (64, 1), (128, 2), (256, 1)]
    out = {}
    for scale in (2, 4, 6, 8, 10):
        n = 800 * scale
        n_buf = max(1, math.ceil(ROTATE_BYTES / (n * n * 4)))
        srcs = [src0.clone() for _ in range(n_buf)]
        dsts = [torch.empty((n, n, 4), dtype=torch.uint8, device=dev) for _ in range(n_buf)]
        times = {}
        for bw, bh in gather:
            _, ms = xr.autotune(srcs, dsts, "bilinear", candidates=[xr.tile(xr.XR_KERNEL_GATHER, bw, bh)],
                                reps=reps, groups=groups)
            times[f"gather {bw}x{bh}"] = ms
        strip = [c for c in xr.tune_candidates("bilinear", xr.XR_U8, 4, 800, 800, n, n)
                 if c.kernel in (xr.XR_KERNEL_STRIP, xr.XR_KERNEL_STRIP_LDS)]
        best_strip, ms = xr.autotune(srcs, dsts, "bilinear", candidates=strip, reps=reps, groups=groups)
        paper = {k: v for k, v in times.items() if tuple(int(x) for x in k.split()[1].split("x")) in PAPER_SHAPES}
        best_paper = min(paper, key=paper.get)
        worst_paper = max(paper, key=paper.get)
        out[f"x{scale}"] = {
            "output": f"{n}x{n}",
            "gather_us": {k: round(v * 1e3, 1) for k, v in times.items()},
            "best_paper_shape": best_paper,
            "paper_spread_worst_over_best": round(paper[worst_paper] / paper[best_paper], 3),
            "best_strip": repr(best_strip),
            "best_strip_us": round(ms * 1e3, 1),
            "strip_speedup_over_best_paper_shape": round(paper[best_paper] / ms, 2),
        }
        log(f"paper sweep x{scale}: {out[f'x{scale}']}")
        del srcs, dsts
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    # 10 groups of 100 timed launches (each group's mean per launch; the
    # median and range over groups are reported)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched comparison")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shape")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (C1, C2 storage types and x0.5, C4, C5)")
    ap.add_argument("--extras", action="store_true",
                    help="also time the other filters and maps and two more adjoints")
    ap.add_argument("--tile", type=str, default=None,
                    help="fixed launch shape KIND,BW,BH,PPX,PPY[,ORDER] (kind 1 gather, 2 strip) instead of tuning")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for hardware counters)")
    ap.add_argument("--profile", type=str, default=None,
                    choices=["x2", "x05", "x2_f16", "x05_f16", "x2_f32", "x05_f32", "c1", "batch", "c4_fwd",
                             "c4_adjoint", "c5", "copy"],
                    help="launch one workload eagerly --steps times with a fixed shape (no graph, no "
                         "tuning; for rocprofv3) and print its mean launch time")
    ap.add_argument("--batch-tile", type=str, default=None,
                    help="fixed batched launch shape KIND,BW,BH,PPX,PPY for --profile batch")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="only run the paper's tile-shape experiment (800x800 bilinear x2..x10) and "
                         "print its JSON line")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1001_1718_amd as xr
    from synth import fields

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.profile:
        if "--steps" not in sys.argv:
            args.steps = 20
        profile_workload(args, torch, xr, fields)
        return
    if args.paper_sweep:
        print(json.dumps({"paper_tile_sweep": paper_sweep(torch, xr, fields), "dtype": "u8",
                          "data": "synthetic"}), flush=True)
        return
    if args.calibrate:
        a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    h = headline(args, torch, xr, fields)
    result = {
        "metric": "output Gpixel/s + % HBM peak, bicubic x2; batched vs per-image launch",
        "value": round(h["value"], 3),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["wall"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "bicubic (Keys a=-0.5) x2 resize, 4096x4096 RGBA uint8 -> 8192x8192, "
                               "half-pixel centres, clamp-to-edge, float32 weights/accumulation",
                   "storage": "u8", "global_batch": 1, "rotating_buffers": h["n_buf"],
                   "tile": h["tile"], "autotune": h["tune"], "parallelism": "single GPU",
                   "submission": "HIP graph of the rotating launches, replayed",
                   "value_eager_launches": round(h["value_eager"], 3)},
        "roofline": h["roofline"],
    }
    result["hbm_reference"] = hbm_reference(torch)
    if not args.no_batch:
        result["batched"] = batched(torch, xr, fields, cpu=not args.no_cpu)
    if not args.no_cpu:
        log("timing the FP64 CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(h["src_host"])
    if not args.no_configs:
        result["configs"] = configs(torch, xr, fields, cpu=not args.no_cpu, breadth=args.extras)
        result["configs"]["C3"] = "the batched entry"
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
