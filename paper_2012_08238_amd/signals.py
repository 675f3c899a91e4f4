"""Seeded synthetic test signals (experimental-setup section of the paper).

K frequencies drawn uniformly without replacement from [0, N), each with
magnitude 1 and a phase uniform in [0, 2 pi); the other frequencies are zero
(exactly sparse) or the time signal gets complex white Gaussian noise scaled to
the requested SNR (general sparse; "general sparse" means 20 dB).

The spectrum follows the 1/N forward convention, so the time signal is
x = N * IDFT(xhat) and a unit tone has |x_t| = 1. SNR is measured in time:
SNR_dB = 10 log10(||x_signal||^2 / ||noise||^2), noise variance per sample
split equally between the real and imaginary parts.

This module only makes inputs: it holds none of the sparse-FFT arithmetic and is
shared by the tests, the benchmark and the CPU baseline.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_MASK64 = (1 << 64) - 1


def derive_seed(master: int, i: int) -> int:
    """Per-signal seed: output i of a SplitMix64 stream started at ``master``."""
    state = (master + (i + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


@dataclass
class Signal:
    x: np.ndarray          # complex128[N] time signal (cast to complex64 for the GPU)
    freqs: np.ndarray      # int64[K] ascending tone positions
    tones: np.ndarray      # complex128[K] tone values (unit magnitude)
    snr_db: float | None   # None for exactly sparse


def make_signal(N: int, K: int, snr_db: float | None = None, seed: int = 0,
                freqs=None, tones=None) -> Signal:
    """One seeded test signal. ``freqs``/``tones`` override the random draw
    (used for the paper's printed examples)."""
    rng = np.random.default_rng(seed & _MASK64)
    if freqs is None:
        freqs = np.sort(rng.choice(N, size=K, replace=False)).astype(np.int64)
    else:
        freqs = np.asarray(freqs, dtype=np.int64)
    if tones is None:
        tones = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, size=freqs.shape[0]))
    else:
        tones = np.asarray(tones, dtype=np.complex128)
    xhat = np.zeros(N, dtype=np.complex128)
    xhat[freqs] = tones
    x = np.fft.ifft(xhat) * N
    if snr_db is not None:
        p_sig = float(np.mean(x.real ** 2 + x.imag ** 2))
        var = p_sig * 10.0 ** (-snr_db / 10.0)
        x = x + np.sqrt(var / 2.0) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    return Signal(x=x, freqs=freqs, tones=tones, snr_db=snr_db)


def make_signal_torch(N: int, K: int, snr_db: float | None, seed: int, device):
    """Same recipe generated directly on a torch device as complex64 (used for
    benchmark batches where host generation would dominate set-up time).
    Returns (x complex64 tensor on device, freqs int64 numpy, tones complex128 numpy)."""
    import torch
    rng = np.random.default_rng(seed & _MASK64)
    freqs = np.sort(rng.choice(N, size=K, replace=False)).astype(np.int64)
    tones = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, size=K))
    xhat = torch.zeros(N, dtype=torch.complex128, device=device)
    xhat[torch.from_numpy(freqs).to(device)] = torch.from_numpy(tones).to(device)
    x = torch.fft.ifft(xhat) * N
    if snr_db is not None:
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed & 0x7FFFFFFFFFFFFFFF))
        p_sig = float(torch.mean(x.real ** 2 + x.imag ** 2))
        var = p_sig * 10.0 ** (-snr_db / 10.0)
        nr = torch.randn(N, generator=gen, device=device, dtype=torch.float64)
        ni = torch.randn(N, generator=gen, device=device, dtype=torch.float64)
        x = x + (var / 2.0) ** 0.5 * torch.complex(nr, ni)
    return x.to(torch.complex64).contiguous(), freqs, tones


def impulse(N: int, j: int) -> np.ndarray:
    """x = e_j (probe that reveals exactly which samples a bucketization reads)."""
    x = np.zeros(N, dtype=np.complex128)
    x[j] = 1.0
    return x


def uneven_batch_specs(n: int = 256, seed: int = 4, log2n=(16, 22), k=(10, 500), snr=(-10.0, 40.0)):
    """(N, K, SNR dB) of an uneven batch: N = 2^e with e uniform over the integers
    of ``log2n``, K uniform over the integers of ``k``, SNR uniform over ``snr``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        e = int(rng.integers(log2n[0], log2n[1] + 1))
        out.append((1 << e, int(rng.integers(k[0], k[1] + 1)), float(rng.uniform(snr[0], snr[1]))))
    return out


def poisson_arrivals(rate: float, n: int, seed: int = 2000) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
