"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the filtering method.  It only draws
inputs with the statistics the paper's error model assumes (Section 4.1: a
natural image has a Fourier amplitude spectrum proportional to 1/u), and the
workload mixes (image sizes, channel counts, sigmas, arrival times) that the
batching and serving paths are measured on.

1/f recipe: white Gaussian noise n from numpy's PCG64 with the given seed;
F = exp(i arg FFT2(n)) / rho with rho = sqrt(fx^2 + fy^2) from fftfreq and
F(0, 0) = 0; x = Re IFFT2(F) scaled affinely to [0, 255].  FP32 keeps the
float value, uint8 is rint clipped to [0, 255], FP16/BF16 are round-to-
nearest-even of the FP32 value.  Channel c of a multi-channel image uses the
seed ``seed * 16 + c``; channels are interleaved (H x W x C).
"""
from __future__ import annotations

import math

import numpy as np


def one_over_f(H: int, W: int, seed: int) -> np.ndarray:
    """One H x W float64 field with a 1/f amplitude spectrum, scaled to [0, 255]."""
    rng = np.random.default_rng(seed)
    n = rng.standard_normal((H, W))
    F = np.fft.fft2(n)
    mag = np.abs(F)
    mag[mag == 0] = 1.0
    phase = F / mag
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    rho = np.sqrt(fx * fx + fy * fy)
    rho[0, 0] = 1.0
    amp = 1.0 / rho
    amp[0, 0] = 0.0
    x = np.real(np.fft.ifft2(amp * phase))
    lo, hi = float(x.min()), float(x.max())
    if hi > lo:
        x = (x - lo) * (255.0 / (hi - lo))
    else:
        x = np.zeros_like(x)
    return x


def to_dtype(x: np.ndarray, dtype: str) -> np.ndarray:
    """Convert a [0, 255] float field to the storage dtype.

    Returns uint8 for "u8", float32 for "f32", float16 for "f16" and, for
    "bf16", the raw uint16 bit patterns (round-to-nearest-even of FP32)."""
    if dtype == "u8":
        return np.clip(np.rint(x), 0, 255).astype(np.uint8)
    if dtype == "f32":
        return x.astype(np.float32)
    if dtype == "f16":
        return x.astype(np.float32).astype(np.float16)
    if dtype == "bf16":
        return f32_to_bf16_bits(x.astype(np.float32))
    raise ValueError("unknown dtype %r" % dtype)


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even FP32 -> BF16, returned as uint16 bit patterns."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16
    return u.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Exact BF16 (uint16 bit patterns) -> FP32."""
    return (np.ascontiguousarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def image(H: int, W: int, C: int, dtype: str, seed: int) -> np.ndarray:
    """H x W (C == 1) or H x W x C interleaved 1/f image in the given dtype."""
    if C == 1:
        return to_dtype(one_over_f(H, W, seed), dtype)
    chans = [to_dtype(one_over_f(H, W, seed * 16 + c), dtype) for c in range(C)]
    return np.ascontiguousarray(np.stack(chans, axis=-1))


def crop_pool(H: int, W: int, C: int, dtype: str, seed: int, pool_side: int = 2048,
              pool_seed_base: int = 7000, pool_count: int = 4) -> np.ndarray:
    """An H x W x C image cut at a seeded offset from a small pool of 1/f fields.

    Large mixed workloads (hundreds of images up to 2048 on a side) would spend
    minutes in FFTs if every image were drawn fresh; a seeded crop of one of
    ``pool_count`` seeded 1/f fields of side ``pool_side`` keeps the 1/f
    statistics at every scale below the field size."""
    if H > pool_side or W > pool_side:
        return image(H, W, C, dtype, seed)
    rng = np.random.default_rng(seed)
    chans = []
    for c in range(C):
        field = _pool_field(pool_side, pool_seed_base + int(rng.integers(pool_count)) * 16 + c, dtype)
        y0 = int(rng.integers(0, pool_side - H + 1))
        x0 = int(rng.integers(0, pool_side - W + 1))
        chans.append(field[y0:y0 + H, x0:x0 + W])
    if C == 1:
        return np.ascontiguousarray(chans[0])
    return np.ascontiguousarray(np.stack(chans, axis=-1))


_POOL: dict = {}


def _pool_field(side: int, seed: int, dtype: str) -> np.ndarray:
    key = (side, seed, dtype)
    if key not in _POOL:
        _POOL[key] = to_dtype(one_over_f(side, side, seed), dtype)
    return _POOL[key]


def batch_specs(n: int = 256, seed: int = 3, side_lo: int = 64, side_hi: int = 2048,
                C: int = 3, sigma_lo: float = 1.0, sigma_hi: float = 30.0, K: int = 4):
    """Mixed batch: H, W iid uniform integers in [side_lo, side_hi], sigma
    log-uniform in [sigma_lo, sigma_hi], fixed C and K.  Image i is drawn with
    seed 1000 * seed + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        H = int(rng.integers(side_lo, side_hi + 1))
        W = int(rng.integers(side_lo, side_hi + 1))
        sigma = float(math.exp(rng.uniform(math.log(sigma_lo), math.log(sigma_hi))))
        out.append(dict(H=H, W=W, C=C, sigma=sigma, K=K, seed=1000 * seed + i))
    return out


def request_stream(n: int, qps: float, seed: int = 5, side_lo: int = 128, side_hi: int = 4096,
                   sigma_lo: float = 0.5, sigma_hi: float = 50.0):
    """Poisson arrivals at rate qps; per request H, W iid uniform in
    [side_lo, side_hi], C in {1, 3}, dtype in {u8, f32}, sigma log-uniform in
    [sigma_lo, sigma_hi], K in {3, 5} (each binary choice with probability 1/2)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / qps))
        out.append(dict(
            t_arrive=t,
            H=int(rng.integers(side_lo, side_hi + 1)),
            W=int(rng.integers(side_lo, side_hi + 1)),
            C=int(rng.choice([1, 3])),
            dtype=str(rng.choice(["u8", "f32"])),
            sigma=float(math.exp(rng.uniform(math.log(sigma_lo), math.log(sigma_hi)))),
            K=int(rng.choice([3, 5])),
            seed=5000 + i,
        ))
    return out
