"""Seeded synthetic images and batch job lists (numpy PCG64 everywhere).

The paper's own test image (an unnamed 800x800 picture, section III.B) is not
available, so every workload uses one of these stand-ins:

* ``uniform_u8``   - i.i.d. uniform bytes 0..255 (worst case for rounding ties);
* ``smooth_field`` - a natural-image stand-in: 127.5 + a sum of 8 random 2-D
  sinusoids of amplitude 14 + Gaussian noise of standard deviation 2;
* ``normal_f32``   - N(0, 1) samples for tensors and upstream gradients;
* ``batch_jobs``   - a list of 256 resize jobs of uneven sizes, scales, channel
  counts and filters.

Nothing here computes a resampled value.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BILINEAR = 0
BICUBIC = 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_u8(shape, seed: int) -> np.ndarray:
    """I.i.d. uniform integers in [0, 255] as uint8."""
    return _rng(seed).integers(0, 256, size=tuple(shape), dtype=np.uint8)


def normal_f32(shape, seed: int) -> np.ndarray:
    """I.i.d. standard normal float32 samples."""
    return _rng(seed).standard_normal(size=tuple(shape), dtype=np.float32)


def smooth_field(height: int, width: int, channels: int = 1, seed: int = 0) -> np.ndarray:
    """Float64 field of shape (height, width, channels).

    Channel c draws its parameters from PCG64(seed + 16 c):
    frequencies f_k, g_k ~ U(-32, 32) cycles per image, phases ~ U(0, 2 pi),
    then additive N(0, sigma=2) noise. Each sinusoid is evaluated as
    sin(a + b) = sin(a) cos(b) + cos(a) sin(b) from two 1-D tables, with
    elementwise numpy operations only, so the result does not depend on a
    BLAS library or thread count.
    """
    h, w = int(height), int(width)
    out = np.empty((h, w, channels), dtype=np.float64)
    xs = np.arange(w, dtype=np.float64) / w
    ys = np.arange(h, dtype=np.float64) / h
    tmp = np.empty((h, w), dtype=np.float64)
    for c in range(channels):
        rng = _rng(seed + 16 * c)
        f = rng.uniform(-32.0, 32.0, 8)
        g = rng.uniform(-32.0, 32.0, 8)
        phi = rng.uniform(0.0, 2.0 * math.pi, 8)
        acc = np.full((h, w), 127.5, dtype=np.float64)
        for k in range(8):
            a = 2.0 * math.pi * f[k] * xs + phi[k]
            b = 2.0 * math.pi * g[k] * ys
            np.multiply.outer(14.0 * np.cos(b), np.sin(a), out=tmp)
            acc += tmp
            np.multiply.outer(14.0 * np.sin(b), np.cos(a), out=tmp)
            acc += tmp
        acc += rng.normal(0.0, 2.0, size=(h, w))
        out[:, :, c] = acc
    return out


def field_u8(height: int, width: int, channels: int, seed: int) -> np.ndarray:
    """Smooth field quantised to bytes: clip(rint(S), 0, 255), shape (H, W, C)."""
    s = smooth_field(height, width, channels, seed)
    np.rint(s, out=s)
    np.clip(s, 0.0, 255.0, out=s)
    return s.astype(np.uint8)


def field_unit(height: int, width: int, channels: int, seed: int, dtype=np.float16) -> np.ndarray:
    """Smooth field scaled to [0, 1]: clip(S / 255, 0, 1) stored as ``dtype``."""
    s = smooth_field(height, width, channels, seed)
    s /= 255.0
    np.clip(s, 0.0, 1.0, out=s)
    return s.astype(dtype)


@dataclass(frozen=True)
class BatchJob:
    in_h: int
    in_w: int
    out_h: int
    out_w: int
    channels: int
    filter: int
    content_seed: int


def batch_jobs(seed: int, count: int = 256, side_lo: int = 64, side_hi: int = 2048,
               scale_lo: float = 0.25, scale_hi: float = 4.0) -> list:
    """Uneven batch: sides ~ U{side_lo..side_hi}, per-axis scales ~ U(scale_lo, scale_hi),
    channels ~ U{1, 4}, exactly half bilinear and half bicubic in shuffled order.
    Output side = max(1, floor(in * scale + 0.5)).
    """
    if count % 2:
        raise ValueError("count must be even (half bilinear, half bicubic)")
    rng = _rng(seed)
    w = rng.integers(side_lo, side_hi + 1, count)
    h = rng.integers(side_lo, side_hi + 1, count)
    sx = rng.uniform(scale_lo, scale_hi, count)
    sy = rng.uniform(scale_lo, scale_hi, count)
    ch = rng.choice(np.array([1, 4]), count)
    filt = np.array([BILINEAR] * (count // 2) + [BICUBIC] * (count // 2))
    rng.shuffle(filt)
    jobs = []
    for k in range(count):
        ow = max(1, int(math.floor(int(w[k]) * float(sx[k]) + 0.5)))
        oh = max(1, int(math.floor(int(h[k]) * float(sy[k]) + 0.5)))
        jobs.append(BatchJob(int(h[k]), int(w[k]), oh, ow, int(ch[k]), int(filt[k]),
                             int(seed) * 100000 + k))
    return jobs


def smooth_field_torch(height: int, width: int, channels: int, seed: int, device="cuda"):
    """The smooth field evaluated on ``device`` (torch, float64), shape (H, W, C).

    Same parameter draws as ``smooth_field`` (numpy PCG64, seed + 16 c); the
    noise comes from a torch generator seeded with the same number, so the
    values are a stand-in of the same distribution, not bitwise the numpy ones.
    For large batches whose generation on the host would dominate a run.
    """
    import torch

    h, w = int(height), int(width)
    xs = torch.arange(w, dtype=torch.float64, device=device) / w
    ys = torch.arange(h, dtype=torch.float64, device=device) / h
    out = torch.empty((h, w, channels), dtype=torch.float64, device=device)
    gen = torch.Generator(device=device)
    for c in range(channels):
        rng = _rng(seed + 16 * c)
        f = rng.uniform(-32.0, 32.0, 8)
        g = rng.uniform(-32.0, 32.0, 8)
        phi = rng.uniform(0.0, 2.0 * math.pi, 8)
        acc = torch.full((h, w), 127.5, dtype=torch.float64, device=device)
        for k in range(8):
            a = 2.0 * math.pi * float(f[k]) * xs + float(phi[k])
            b = 2.0 * math.pi * float(g[k]) * ys
            acc += torch.outer(14.0 * torch.cos(b), torch.sin(a))
            acc += torch.outer(14.0 * torch.sin(b), torch.cos(a))
        gen.manual_seed(int(seed) * 7919 + c)
        acc += 2.0 * torch.randn((h, w), generator=gen, dtype=torch.float64, device=device)
        out[:, :, c] = acc
    return out


def field_u8_torch(height: int, width: int, channels: int, seed: int, device="cuda"):
    """``smooth_field_torch`` quantised to uint8 (clip(rint(S), 0, 255))."""
    import torch

    s = smooth_field_torch(height, width, channels, seed, device)
    return torch.clamp(torch.round(s), 0.0, 255.0).to(torch.uint8)
