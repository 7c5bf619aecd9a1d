"""FP64 oracle of the log-Mel front end the paper trains on (Sec. 3).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or run
this module.  It shares no code, tables or helpers with the GPU path.

The paper's features: 128 log-Mel bands from 32 ms windows every 10 ms, the
Mel filterbank spanning 125 Hz to 7500 Hz (and four frames stacked, then
down-sampled by three: a view of these frames).  At 16 kHz a window is 512
samples and the hop 160.

Readings where the paper is silent:
* Frame t covers samples [160 t, 160 t + 512) of a mic's output; only whole
  frames (no padding): max(0, 1 + (T - 512) // 160) frames for T samples.
* Periodic Hann window w[n] = 0.5 - 0.5 cos(2 pi n / 512).
* Power spectrum P[k] = |sum_n w[n] y[n] e^{-2 pi i k n / 512}|^2, k = 0..256.
* Mel scale m(f) = 2595 log10(1 + f / 700); 130 edges equally spaced in mel
  from m(125) to m(7500); band b is the triangle over edges b, b+1, b+2 (in
  Hz), weight at bin frequency k * 16000 / 512: rising, then falling, 1 at
  the centre, 0 outside.
* Log: natural log of (band energy + 1e-6).
"""
from __future__ import annotations

import math

import numpy as np

FS, WIN, HOP, BANDS, F_LO, F_HI, FLOOR = 16000, 512, 160, 128, 125.0, 7500.0, 1e-6


def hz_to_mel(f):
    return 2595.0 * np.log10(1.0 + np.asarray(f, np.float64) / 700.0)


def mel_to_hz(m):
    return 700.0 * (10.0 ** (np.asarray(m, np.float64) / 2595.0) - 1.0)


def filterbank() -> np.ndarray:
    """Weights [128, 257] of the triangular Mel filters."""
    edges = mel_to_hz(np.linspace(hz_to_mel(F_LO), hz_to_mel(F_HI), BANDS + 2))
    f = np.arange(WIN // 2 + 1) * (FS / WIN)
    W = np.zeros((BANDS, WIN // 2 + 1))
    for b in range(BANDS):
        lo, c, hi = edges[b], edges[b + 1], edges[b + 2]
        up = (f - lo) / (c - lo)
        down = (hi - f) / (hi - c)
        W[b] = np.clip(np.minimum(up, down), 0.0, None)
    return W


def n_frames(T: int) -> int:
    return max(0, 1 + (int(T) - WIN) // HOP) if T >= WIN else 0


def power_spectra(y: np.ndarray) -> np.ndarray:
    """[frames, 257] power spectra of the windowed frames of y, in FP64."""
    y = np.asarray(y, np.float64)
    F = n_frames(y.size)
    if F == 0:
        return np.zeros((0, WIN // 2 + 1))
    idx = np.arange(F)[:, None] * HOP + np.arange(WIN)[None, :]
    w = 0.5 - 0.5 * np.cos(2.0 * math.pi * np.arange(WIN) / WIN)
    X = np.fft.rfft(y[idx] * w[None, :], axis=1)
    return X.real ** 2 + X.imag ** 2


def mel_energies(y: np.ndarray) -> np.ndarray:
    """[frames, 128] Mel band energies (before the log)."""
    return power_spectra(y) @ filterbank().T


def logmel(y: np.ndarray) -> np.ndarray:
    """[frames, 128] log-Mel features of one mic's output."""
    return np.log(mel_energies(y) + FLOOR)


def stack(feat: np.ndarray, k: int = 4, step: int = 3) -> np.ndarray:
    """Frames t, t+1, .., t+k-1 side by side, every `step`-th t."""
    F = feat.shape[0]
    if F < k:
        return np.zeros((0, k * feat.shape[1]))
    starts = np.arange(0, F - k + 1, step)
    return np.concatenate([feat[starts + i] for i in range(k)], axis=1)
