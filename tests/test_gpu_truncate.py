"""RIR cut-off on the GPU: n_c and L bit-exact against the oracle's float32 rule."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import cuda


def _run(rirs, eta):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    lens = np.array([len(h) for h in rirs], np.int32)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    flat = np.concatenate([np.asarray(h, np.float32) for h in rirs] + [np.zeros(1, np.float32)])
    h = torch.from_numpy(flat).cuda()
    n_c, L = rsim.truncate_rir(h, torch.from_numpy(off).cuda(), torch.from_numpy(lens).cuda(), eta)
    return n_c.cpu().numpy(), L.cpu().numpy()


def _edge_rirs():
    r = np.random.default_rng(0)
    out = [np.zeros(0, np.float32), np.zeros(9, np.float32), np.array([0.3], np.float32)]
    g = np.zeros(2000, np.float32)
    g[-1] = 2.0
    out.append(g)                                           # peak at the last tap
    s = np.zeros(5000, np.float32)
    s[1234] = 0.8
    out.append(s)                                           # single spike
    out.append(np.array([1.0, 0.1, 0.5, 0.1, 0.49], np.float32))   # q == p_th at 10 log10(4) dB
    out.append(np.array([1e-20, 4e-21, 1e-25, 0.0], np.float32))  # subnormal powers
    out.append(np.array([0.1, -0.5, 0.2, 0.5, 0.3, 0.1], np.float32))  # repeated peak
    for L0 in (1, 63, 64, 65, 1023, 1024, 1025, 3000, 16000):   # ragged against the chunking
        out.append((r.standard_normal(L0) * np.exp(-np.arange(L0) / (L0 / 5 + 1))).astype(np.float32))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("eta", [0.0, 5.0, 10.0, 20.0, 30.0, 10 * math.log10(4.0), math.inf])
def test_cut_bit_exact(eta):
    rng = synth.rng_for(2, 5)
    rirs = _edge_rirs()
    for _ in range(300):
        t60 = rng.uniform(0.1, 1.0)
        rirs.append(synth.rir(rng, int(math.ceil(t60 * 16000)), t60, int(rng.integers(20, 401))))
    n_c, L = _run(rirs, eta)
    for k, h in enumerate(rirs):
        ref_nc, ref_L, _ = oracle.cut_rir(h, eta)
        assert (int(n_c[k]), int(L[k])) == (ref_nc, ref_L), (k, len(h))


@pytest.mark.gpu
def test_cut_nonfinite_keeps_rir_and_flags():
    from paper_1712_03439_amd import rsim

    rsim.device_status()  # clear
    rirs = [np.array([0.5, np.nan, 0.1], np.float32), np.array([0.5, 3e19, 0.1], np.float32),
            np.array([1.0, 0.0, 0.001], np.float32)]
    n_c, L = _run(rirs, 20.0)
    assert list(L[:2]) == [3, 3] and list(n_c[:2]) == [2, 2]
    assert (int(n_c[2]), int(L[2])) == oracle.cut_rir(rirs[2], 20.0)[:2]
    assert rsim.device_status() & rsim.DEV_NONFINITE
    assert rsim.device_status() == 0  # read clears


def _long_rirs():
    """RIRs past the 32 chunk maxima the cut kernel keeps (more than 32768
    taps), where the last tap at or above the threshold is searched from the
    tail: decaying noise, the last such tap in the first chunk (a lone spike
    at the start, every other tap far below), the final tap, and a tie with
    the peak at the far end."""
    r = np.random.default_rng(31)
    out = []
    for L0 in (32768, 32769, 40000, 65537):
        out.append((r.standard_normal(L0) * np.exp(-np.arange(L0) / (L0 / 6))).astype(np.float32))
        early = (r.standard_normal(L0) * 1e-4).astype(np.float32)
        early[5] = 1.0
        out.append(early)                                   # the cut lands in the first chunk
        last = (r.standard_normal(L0) * 1e-3).astype(np.float32)
        last[-1] = 0.5
        out.append(last)                                    # the final tap is the peak
        tie = (r.standard_normal(L0) * 1e-2).astype(np.float32)
        tie[7], tie[L0 - 2] = 0.75, -0.75                   # equal powers, the later one kept
        out.append(tie)
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("eta", [0.0, 10.0, 20.0, 30.0, math.inf])
def test_cut_bit_exact_past_the_chunk_maxima(eta):
    rirs = _long_rirs()
    n_c, L = _run(rirs, eta)
    for k, h in enumerate(rirs):
        ref_nc, ref_L, _ = oracle.cut_rir(h, eta)
        assert (int(n_c[k]), int(L[k])) == (ref_nc, ref_L), (k, len(h), eta)
    if eta == 20.0:
        # the lone early spike: everything after index 5 is 80 dB down
        assert [int(v) for v in n_c[1::4]] == [5, 5, 5, 5]
        assert [int(v) for v in L[2::4]] == [len(h) for h in rirs[2::4]]
