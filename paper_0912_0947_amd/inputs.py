"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only draws cover bytes,
message bytes, workload shapes and arrival times.  Both the GPU path and the
CPU oracle are fed from here; neither side generates its own inputs.

The paper measures on its own images (an aeroplane cover and a 7x8 payload),
which are not available, so every workload is synthetic:

* ``uniform_cover`` / ``random_bytes``: i.i.d. uniform bytes (PCG64).
* ``smooth_cover``: a per-channel low-frequency sinusoidal gradient plus
  Gaussian noise, rounded half-to-even and clipped to 0..255 -- the texture of
  a natural photograph at large size.
* ``video_frames``: a moving gradient (phase advancing per frame) plus noise,
  generated with torch on the target device so that multi-GB clips need no
  host staging.
* ``batch_shapes`` / ``fill_uniform``: uneven batches of covers.
* ``poisson_arrivals``: open-loop request arrival times.
"""
from __future__ import annotations

import math

import numpy as np


def rng(*seed: int) -> np.random.Generator:
    """PCG64 generator keyed by a tuple of integers."""
    return np.random.default_rng(np.random.SeedSequence(list(seed)))


def random_bytes(n: int, *seed: int) -> np.ndarray:
    return rng(*seed).integers(0, 256, size=n, dtype=np.uint8)


def uniform_cover(shape, *seed: int) -> np.ndarray:
    return rng(*seed).integers(0, 256, size=shape, dtype=np.uint8)


def smooth_cover(height: int, width: int, channels: int = 3,
                 param_seed: int = 201, noise_seed: int = 202,
                 amplitude: float = 64.0, sigma: float = 8.0,
                 rows_per_chunk: int = 256) -> np.ndarray:
    """HWC uint8 cover: 128 + A*sin(2*pi*(a_c*x/W + b_c*y/H) + phi_c) + N(0,
    sigma^2) per channel c, with a_c, b_c ~ U[0.5, 2] and phi_c ~ U[0, 2*pi)."""
    p = rng(param_seed)
    a = p.uniform(0.5, 2.0, size=channels)
    b = p.uniform(0.5, 2.0, size=channels)
    phi = p.uniform(0.0, 2.0 * math.pi, size=channels)
    noise = rng(noise_seed)
    out = np.empty((height, width, channels), dtype=np.uint8)
    x = (np.arange(width, dtype=np.float64) / width)[None, :]
    for y0 in range(0, height, rows_per_chunk):
        y1 = min(height, y0 + rows_per_chunk)
        y = (np.arange(y0, y1, dtype=np.float64) / height)[:, None]
        for c in range(channels):
            phase = (2.0 * math.pi * (a[c] * x + b[c] * y) + phi[c]).astype(np.float32)
            v = np.sin(phase, out=phase)
            v *= np.float32(amplitude)
            v += np.float32(128.0)
            v += noise.standard_normal(size=v.shape, dtype=np.float32) * np.float32(sigma)
            np.clip(np.rint(v, out=v), 0, 255, out=v)
            out[y0:y1, :, c] = v.astype(np.uint8)
    return out


def video_frames(frames: int, height: int, width: int, device="cpu",
                 param_seed: int = 301, noise_seed: int = 302,
                 amplitude: float = 100.0, sigma: float = 8.0, out=None):
    """uint8 torch tensor [frames, H, W, 3]: a moving gradient
    128 + A*sin(2*pi*(a*x/W + b*y/H - f/120) + 2*pi*c/3) plus N(0, sigma^2),
    rounded and clipped.  Generated frame by frame on ``device``."""
    import torch

    p = rng(param_seed)
    a, b = p.uniform(0.5, 2.0, size=2)
    if out is None:
        out = torch.empty((frames, height, width, 3), dtype=torch.uint8, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(noise_seed)
    xs = torch.arange(width, dtype=torch.float32, device=device) / width
    ys = torch.arange(height, dtype=torch.float32, device=device) / height
    base = (a * xs[None, :] + b * ys[:, None])  # [H, W]
    chan = torch.arange(3, dtype=torch.float32, device=device) * (2.0 * math.pi / 3.0)
    for f in range(frames):
        phase = 2.0 * math.pi * (base - f / 120.0)
        v = 128.0 + amplitude * torch.sin(phase[:, :, None] + chan[None, None, :])
        v += torch.randn(v.shape, generator=gen, device=device, dtype=torch.float32) * sigma
        out[f].copy_(v.round_().clamp_(0, 255).to(torch.uint8))
    return out


def batch_shapes(count: int, seed: int = 401, lo: int = 64, hi: int = 4096,
                 ks=(1, 2), frac_lo: float = 0.1, frac_hi: float = 1.0):
    """Uneven batch: width, height ~ U{lo..hi}, channels 1 or 3 (50/50),
    k drawn from ``ks``, message fraction u ~ U[frac_lo, frac_hi].
    Returns a dict of numpy arrays (n = W*H*C cover bytes per job)."""
    g = rng(seed)
    w = g.integers(lo, hi + 1, size=count)
    h = g.integers(lo, hi + 1, size=count)
    c = np.where(g.integers(0, 2, size=count) == 0, 1, 3)
    k = np.asarray(ks)[g.integers(0, len(ks), size=count)]
    u = g.uniform(frac_lo, frac_hi, size=count)
    n = (w * h * c).astype(np.int64)
    return {"w": w, "h": h, "c": c, "k": k.astype(np.int64), "u": u, "n": n}


def fill_uniform(tensor, seed: int) -> None:
    """Fill a uint8 torch tensor (any device) with seeded uniform bytes."""
    import torch

    gen = torch.Generator(device=tensor.device)
    gen.manual_seed(seed)
    flat = tensor.view(-1)
    step = 1 << 30
    for i in range(0, flat.numel(), step):
        part = flat[i:i + step]
        part.random_(0, 256, generator=gen)


def poisson_arrivals(rate: float, count: int, seed: int = 501) -> np.ndarray:
    """Open-loop arrival times in seconds: cumulative Exp(1/rate) gaps."""
    return np.cumsum(rng(seed, int(rate)).exponential(1.0 / rate, size=count))
