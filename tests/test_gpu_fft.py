"""FFT engine (r2c / c2r per size) against numpy.fft in FP64."""
import numpy as np
import pytest

from tests.gpu_util import cuda

SIZES = [512, 1024, 2048, 4096, 8192, 16384, 32768]


@pytest.mark.gpu
@pytest.mark.parametrize("n", SIZES)
def test_rfft_matches_numpy(n):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n)).astype(np.float32)
    got = rsim.rfft(torch.from_numpy(x).cuda(), n).cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    ref = np.fft.rfft(x.astype(np.float64), axis=1)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err < 2e-6, err


@pytest.mark.gpu
@pytest.mark.parametrize("n", SIZES)
def test_irfft_inverts(n):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal((2, n)).astype(np.float32)
    spec = np.fft.rfft(x.astype(np.float64), axis=1)
    s32 = np.stack([spec.real, spec.imag], -1).astype(np.float32)
    got = rsim.irfft(torch.from_numpy(s32).cuda(), n).cpu().numpy()
    err = np.max(np.abs(got - x)) / np.max(np.abs(x))
    assert err < 2e-6, err


@pytest.mark.gpu
@pytest.mark.parametrize("n", [512, 8192, 32768])
def test_special_inputs(n):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    x = np.zeros((3, n), np.float32)
    x[0, 0] = 1.0                                    # impulse -> flat spectrum
    k = n // 8 + 3
    x[1] = np.cos(2 * np.pi * k * np.arange(n) / n)  # cosine -> two bins
    x[2, :] = 1.0                                    # DC only
    got = rsim.rfft(torch.from_numpy(x).cuda(), n).cpu().numpy()
    g = got[..., 0] + 1j * got[..., 1]

    def bound(ref):
        # float32 FFT error: |err|_2 <= c eps log2(n) |X|_2 with a small c.
        return 4.0 * 2.0 ** -24 * np.log2(n) * np.linalg.norm(ref) + 1e-6

    ref0 = np.ones(n // 2 + 1)
    assert np.max(np.abs(g[0] - ref0)) <= bound(ref0)
    ref1 = np.zeros(n // 2 + 1)
    ref1[k] = n / 2
    assert np.max(np.abs(g[1] - ref1)) <= bound(ref1)
    ref2 = np.zeros(n // 2 + 1)
    ref2[0] = n
    assert np.max(np.abs(g[2] - ref2)) <= bound(ref2)
