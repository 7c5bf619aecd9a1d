"""Pins of the log-Mel oracle (Sec. 3 front end), CPU only."""
import math

import numpy as np
import pytest

from oracle import logmel_oracle as lm


@pytest.mark.parametrize("T,F", [(0, 0), (511, 0), (512, 1), (671, 1), (672, 2), (16000, 97)])
def test_frame_count(T, F):
    # whole frames of 512 samples every 160: 1 + (T - 512) // 160
    assert lm.n_frames(T) == F


def test_power_spectrum_of_an_on_bin_tone():
    # a unit cosine at bin 40 under the periodic Hann window: the transform is
    # 128 at bin 40 and -64 at bins 39 and 41, zero elsewhere
    n = np.arange(512)
    y = np.cos(2 * math.pi * 40 * n / 512)
    P = lm.power_spectra(y)[0]
    assert abs(P[40] - 128.0 ** 2) < 1e-8
    assert abs(P[39] - 64.0 ** 2) < 1e-8 and abs(P[41] - 64.0 ** 2) < 1e-8
    rest = np.delete(P, [39, 40, 41])
    assert np.max(rest) < 1e-16


def test_band_energies_and_features_of_an_on_bin_tone():
    # the tone's power spectrum is fixed in closed form (above), so a band's
    # energy is its weights at bins 39, 40 and 41 times 64^2, 128^2 and 64^2,
    # and its feature the natural log of that energy plus 1e-6; at amplitude
    # 1e-5 the energies are of the order of that floor
    n = np.arange(512)
    W = lm.filterbank()
    for amp in (1.0, 1e-5):
        y = amp * np.cos(2 * math.pi * 40 * n / 512)
        E = amp * amp * (W[:, 39] * 64.0 ** 2 + W[:, 40] * 128.0 ** 2 + W[:, 41] * 64.0 ** 2)
        assert np.count_nonzero(E) >= 2
        assert np.allclose(lm.mel_energies(y)[0], E, rtol=1e-9, atol=1e-15 * amp * amp)
        assert np.allclose(lm.logmel(y)[0], np.log(E + 1e-6), rtol=0.0, atol=1e-9)


def test_power_spectrum_by_the_dft_sum_and_parseval():
    rng = np.random.default_rng(41)
    y = rng.standard_normal(700)
    P = lm.power_spectra(y)[1]                      # the frame at 160
    w = [0.5 - 0.5 * math.cos(2 * math.pi * k / 512) for k in range(512)]
    seg = [w[k] * y[160 + k] for k in range(512)]
    for k in (0, 1, 77, 255, 256):
        re = sum(seg[n] * math.cos(2 * math.pi * k * n / 512) for n in range(512))
        im = sum(seg[n] * math.sin(2 * math.pi * k * n / 512) for n in range(512))
        assert abs(P[k] - (re * re + im * im)) <= 1e-9 * max(P[k], 1.0)
    full = P[0] + P[256] + 2 * np.sum(P[1:256])
    assert abs(full / 512 - sum(v * v for v in seg)) <= 1e-9 * full


def test_filterbank_edges_and_partition_of_unity():
    assert abs(lm.hz_to_mel(1000.0) - 999.986) < 1e-3         # the scale puts 1 kHz at ~1000 mel
    edges = lm.mel_to_hz(np.linspace(lm.hz_to_mel(125.0), lm.hz_to_mel(7500.0), 130))
    assert abs(edges[0] - 125.0) < 1e-9 and abs(edges[-1] - 7500.0) < 1e-9
    W = lm.filterbank()
    assert W.shape == (128, 257) and W.min() >= 0.0 and W.max() <= 1.0
    f = np.arange(257) * 31.25
    inner = (f >= edges[1]) & (f <= edges[128])
    # between the first and the last centre, neighbouring triangles add to one
    assert np.allclose(W[:, inner].sum(axis=0), 1.0, atol=1e-12)
    assert not np.any(W[:, f < 125.0]) and not np.any(W[:, f > 7500.0])


def test_silence_gives_the_floor_and_stacking_is_a_view():
    feat = lm.logmel(np.zeros(2000))
    assert feat.shape == (lm.n_frames(2000), 128) and np.all(feat == math.log(1e-6))
    f = np.arange(10 * 3, dtype=np.float64).reshape(10, 3)
    s = lm.stack(f, 4, 3)
    assert s.shape == (3, 12)
    assert np.array_equal(s[1], np.concatenate([f[3], f[4], f[5], f[6]]))
