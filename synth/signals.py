"""Synthetic stand-ins for the paper's datasets (Section 5.2, Table 2).

The paper's recordings (MIT-BIH, EEG, seismic traces, wind/solar/load power,
temperature, irradiance, wind speed) are not available, so every workload is
generated here from a fixed seed.  Each generator returns float64 samples; the
callers cast to float32, the sample type the codec compresses (Section 3.2).

Recipe (constants marked "reading" are choices where the workload description
is silent):
  * EEG-like, fs = 256 Hz: four sinusoids with frequency U(1, 40) Hz, amplitude
    U(10, 50), phase U(0, 2*pi) (reading), plus 1/f noise: white Gaussian noise
    shaped by 1/sqrt(f) in the frequency domain with the DC bin zeroed
    (reading), rescaled to standard deviation 5.
  * Seismic-like, fs = 500 Hz: a Ricker wavelet with peak frequency U(10, 60) Hz
    per stream (reading), support +-0.2 s (reading), convolved with a
    Bernoulli(0.01) * N(0, 1) reflectivity series.
  * Power-grid, fs = 3840 Hz (64 samples per 60 Hz cycle, reading): per-unit
    amplitude (reading) 60 Hz fundamental plus 3rd/5th/7th harmonics at
    10/5/2 %, modulated by a daily load ramp 1 + 0.2*sin(2*pi*n/L + phi) whose
    period is compressed to the stream length L (reading).
  * Meteorological: 15 + AR(1)(phi = 0.999, sigma_e = 0.1) + 5*cos(2*pi*n/1440)
    (constants 15, 0.1, 5 and the 1440-sample diurnal period are readings).
  * Multichannel EEG: 64 independent EEG-like sources mixed by a 64x64 matrix
    with N(0, 1/64) entries (reading).
"""
from __future__ import annotations

import numpy as np

ROOT_SEED = 2605_01086
DOMAINS = ("eeg", "seismic", "power", "meteo")

# SeedSequence spawn keys: (purpose, config, stream).  Purpose 0 = evaluation
# streams, purpose 1 = codebook-training streams, so the two never share draws.
_PURPOSE_EVAL = 0
_PURPOSE_TRAIN = 1


def stream_rng(config: int, stream: int) -> np.random.Generator:
    """Generator for evaluation stream `stream` of workload `config`."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(_PURPOSE_EVAL, int(config), int(stream)))
    return np.random.Generator(np.random.PCG64(ss))


def training_rng(config: int, domain: int) -> np.random.Generator:
    """Generator for the codebook-training signal of `domain` in `config`."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(_PURPOSE_TRAIN, int(config), int(domain)))
    return np.random.Generator(np.random.PCG64(ss))


def eeg_like(n: int, rng: np.random.Generator, fs: float = 256.0) -> np.ndarray:
    t = np.arange(n, dtype=np.float64) / fs
    x = np.zeros(n, dtype=np.float64)
    f = rng.uniform(1.0, 40.0, size=4)
    a = rng.uniform(10.0, 50.0, size=4)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=4)
    for i in range(4):
        x += a[i] * np.sin(2.0 * np.pi * f[i] * t + ph[i])
    if n >= 2:
        w = rng.standard_normal(n)
        W = np.fft.rfft(w)
        k = np.arange(W.shape[0], dtype=np.float64)
        k[0] = 1.0
        W = W / np.sqrt(k)
        W[0] = 0.0
        pink = np.fft.irfft(W, n=n)
        sd = pink.std()
        if sd > 0:
            x += pink * (5.0 / sd)
    return x


def _ricker(fp: float, fs: float, half_support_s: float = 0.2) -> np.ndarray:
    t = np.arange(-half_support_s, half_support_s + 0.5 / fs, 1.0 / fs)
    a = (np.pi * fp * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def seismic_like(n: int, rng: np.random.Generator, fs: float = 500.0) -> np.ndarray:
    fp = rng.uniform(10.0, 60.0)
    refl = (rng.random(n) < 0.01) * rng.standard_normal(n)
    w = _ricker(fp, fs)
    return np.convolve(refl, w, mode="same")[:n]


def power_like(n: int, rng: np.random.Generator, fs: float = 3840.0) -> np.ndarray:
    t = np.arange(n, dtype=np.float64) / fs
    phi = rng.uniform(0.0, 2.0 * np.pi)
    ph0 = rng.uniform(0.0, 2.0 * np.pi)
    ramp = 1.0 + 0.2 * np.sin(2.0 * np.pi * np.arange(n) / max(n, 1) + phi)
    w = 2.0 * np.pi * 60.0 * t + ph0
    wave = np.sin(w) + 0.10 * np.sin(3 * w) + 0.05 * np.sin(5 * w) + 0.02 * np.sin(7 * w)
    return ramp * wave


def meteo_like(n: int, rng: np.random.Generator) -> np.ndarray:
    e = rng.standard_normal(n) * 0.1
    ar = np.empty(n, dtype=np.float64)
    # AR(1) via a recursive filter, started from its stationary distribution.
    acc = rng.standard_normal() * 0.1 / np.sqrt(1.0 - 0.999 ** 2)
    # Block recursion keeps this vectorised: y[i] = phi^(i+1) y0 + sum phi^(i-j) e[j].
    blk = 4096
    p = 0.999 ** np.arange(1, blk + 1)
    for s in range(0, n, blk):
        m = min(blk, n - s)
        seg = e[s:s + m]
        # Linear filter inside the block by cumulative scaling (stable for m <= 4096).
        scale = 0.999 ** np.arange(m)
        y = np.cumsum(seg / scale) * scale + acc * p[:m]
        ar[s:s + m] = y
        acc = y[-1]
    phase = rng.uniform(0.0, 2.0 * np.pi)
    return 15.0 + ar + 5.0 * np.cos(2.0 * np.pi * np.arange(n) / 1440.0 + phase)


def multichannel_eeg(n_ch: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """[n_ch, n] EEG-like channels correlated by a random N(0, 1/n_ch) mixing matrix."""
    src = np.stack([eeg_like(n, rng) for _ in range(n_ch)])
    M = rng.standard_normal((n_ch, n_ch)) / np.sqrt(n_ch)
    return M @ src


_GEN = {"eeg": eeg_like, "seismic": seismic_like, "power": power_like, "meteo": meteo_like}


def domain_signal(domain: str, n: int, rng: np.random.Generator) -> np.ndarray:
    return _GEN[domain](int(n), rng)


def batch_lengths(n_streams: int, lo_log2: float, hi_log2: float, rng: np.random.Generator) -> np.ndarray:
    """Stream lengths floor(2**U(lo, hi)), log-uniform."""
    return np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, size=n_streams)).astype(np.int64)
