"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no FFT arithmetic.  It produces:

* counter-based uniform values in [-1, 1): the SplitMix64 generator of
  Steele, Lea and Flood (OOPSLA 2014).  Element ``i`` of stream ``seed`` is the
  (i+1)-th output of SplitMix64 started from state ``seed * 2**40``, i.e.
  mix64(seed * 2**40 + (i + 1) * 0x9E3779B97F4A7C15).  FP64 values are
  2 * (z >> 11) * 2**-53 - 1, FP32 values 2 * (z >> 40) * 2**-24 - 1; both are
  exact in their type, so host and device copies are bit-identical.  The
  arithmetic is 64-bit two's complement in torch int64 tensors, so the same
  code runs on the host or on the GPU;
* Gaussian random half spectra with a Kolmogorov-like shell spectrum
  E(k) ~ k^(-5/3) (per-mode amplitude |k|^(-11/6)) in the band
  1 <= |k| <= N/3, drawn with numpy's PCG64;
* the paper's analytic test field (section 4, the field used for the timing
  runs): 8 sin x sin 2y sin 3z + 8 sin 4x sin 5y sin 6z on the (2 pi)^3 box.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def _s64(v: int) -> int:
    """Two's complement reading of a 64-bit pattern as a signed integer."""
    v &= (1 << 64) - 1
    return v - (1 << 64) if v >> 63 else v


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix64(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _s64(_M1)
    z = (z ^ _srl(z, 27)) * _s64(_M2)
    return z ^ _srl(z, 31)


def splitmix_bits(seed: int, start: int, count: int,
                  device="cpu") -> torch.Tensor:
    """Raw 64-bit outputs (as int64 bit patterns) for indices [start, start+count)."""
    idx = torch.arange(start + 1, start + 1 + count, dtype=torch.int64,
                       device=device)
    z = idx * _s64(_GAMMA) + _s64(seed << 40)
    return _mix64(z)


def uniform(shape, seed: int, dtype=torch.float64, device="cpu",
            offset: int = 0, chunk: int = 1 << 26) -> torch.Tensor:
    """Seeded uniform values in [-1, 1) of ``shape`` (C order linear index).

    ``offset`` shifts the linear index, so a rank's slab of a larger grid can
    be generated with its global indices.  Generated in chunks to bound the
    temporary memory.
    """
    shape = tuple(int(s) for s in shape)
    total = int(np.prod(shape, dtype=np.int64)) if shape else 1
    out = torch.empty(total, dtype=dtype, device=device)
    for s in range(0, total, chunk):
        c = min(chunk, total - s)
        z = splitmix_bits(seed, offset + s, c, device)
        if dtype == torch.float64:
            u = _srl(z, 11).to(torch.float64) * (2.0 ** -53)
        elif dtype == torch.float32:
            u = (_srl(z, 40).to(torch.float64) * (2.0 ** -24))
        else:
            raise ValueError("dtype must be float64 or float32")
        out[s:s + c] = (2.0 * u - 1.0).to(dtype)
    return out.view(shape)


def uniform_complex(shape, seed_re: int, seed_im: int, dtype=torch.float64,
                    device="cpu") -> torch.Tensor:
    """Complex values whose real and imaginary parts are two uniform streams.

    Returned as a real tensor of shape ``shape + (2,)`` (interleaved re, im).
    """
    re = uniform(shape, seed_re, dtype, device)
    im = uniform(shape, seed_im, dtype, device)
    return torch.stack((re, im), dim=-1)


def _signed(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.where(k <= n // 2, k, k - n)


def kolmogorov_half_spectrum(n: int, seed: int) -> np.ndarray:
    """Random half spectrum [N, N, N//2+1] (complex128) with E(k) ~ k^-5/3.

    Gaussian coefficients (g1 + i g2)/sqrt(2) from PCG64(seed), times the
    per-mode amplitude |k|^(-11/6) for 1 <= |k|^2 and 9 |k|^2 <= N^2, zero
    elsewhere.  The mean (k = 0) mode is zero.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kz = np.arange(n // 2 + 1)
    kxy = _signed(n)
    k2 = (kxy[:, None, None] ** 2 + kxy[None, :, None] ** 2
          + kz[None, None, :] ** 2)
    band = (k2 >= 1) & (9 * k2 <= n * n)
    amp = np.zeros(k2.shape, dtype=np.float64)
    amp[band] = k2[band].astype(np.float64) ** (-11.0 / 12.0)
    shape = (n, n, n // 2 + 1)
    g1 = rng.standard_normal(shape)
    g2 = rng.standard_normal(shape)
    return amp * (g1 + 1j * g2) / math.sqrt(2.0)


def paper_test_field(n: int) -> np.ndarray:
    """8 sin x sin 2y sin 3z + 8 sin 4x sin 5y sin 6z at x_j = 2 pi j / N."""
    x = 2.0 * np.pi * np.arange(n) / n
    sx, sy, sz = x[:, None, None], x[None, :, None], x[None, None, :]
    return (8.0 * np.sin(sx) * np.sin(2 * sy) * np.sin(3 * sz)
            + 8.0 * np.sin(4 * sx) * np.sin(5 * sy) * np.sin(6 * sz))


def paper_test_field_torch(n: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    """The same field built with torch on ``device`` (large grids on the GPU):
    [1, N, N, N], the sines evaluated once per axis and combined by
    broadcasting.  Values agree with ``paper_test_field`` to rounding."""
    t = 2.0 * math.pi * torch.arange(n, dtype=torch.float64, device=device) / n
    s = [torch.sin(a * t) for a in (1, 2, 3, 4, 5, 6)]
    out = torch.empty((1, n, n, n), dtype=dtype, device=device)
    for i0 in range(0, n, 64):
        sl = slice(i0, min(n, i0 + 64))
        blk = (8.0 * s[0][sl, None, None] * s[1][None, :, None] * s[2][None, None, :]
               + 8.0 * s[3][sl, None, None] * s[4][None, :, None] * s[5][None, None, :])
        out[0, sl] = blk.to(dtype)
    return out
