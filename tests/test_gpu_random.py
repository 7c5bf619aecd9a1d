"""Seeded random batches through the forward (cut + eq. 2) and the adjoint,
every output sample and every gradient entry against the FP64 oracle; the
same kind of batches through the reverberant energies, the front end
(separate and fused), the full-length filtering, and random RIR shapes
through the cut; and three wider batches (up to 16 mics, 8 sources, 60000
samples, 16000 taps) through the forward, the adjoint and the energies.

Each of 24 batches draws its shape from a wide range: 1-27 utterances, 1-8 mics,
0-4 sources per utterance (0: nothing to write), sources of 1 to 12000
samples, RIRs of 0 to 3000 taps, a threshold from {inf, 30, 20, 10, 3} dB,
and one of: the library's own size rule, a forced FFT size per utterance (so
several kernel families run in one call), a forced size with a forced hop, a
caller's processing order, or the epoch as one graph.  Bars as in the
forward and adjoint tests: 1e-5 of the peak per (utterance, mic) and per
gradient tensor; the cut lengths bit-exact."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, cuda, max_rel_err
from tests.test_gpu_backward import _check_full_many, _run
from tests.test_gpu_mix import _check_utterances, _simulate

ETAS = (math.inf, 30.0, 20.0, 10.0, 3.0)
MODES = ("rule", "sizes", "sizes+hop", "order", "graph")


def _random_batch(k):
    rng = synth.rng_for(60, k)
    U = int(rng.integers(1, 28))
    J = int(rng.choice([1, 2, 3, 4, 5, 8]))
    srcs, rirs, snrs = [], [], []
    for _ in range(U):
        I = int(rng.choice([0, 1, 1, 2, 2, 3, 4]))
        n = int(rng.choice([1, 7, 64, 513])) if rng.random() < 0.15 else int(rng.integers(100, 12000))
        kinds = [synth.speech_like, synth.white_noise] + ([synth.pink_noise] if n >= 64 else [])
        srcs.append([kinds[int(rng.integers(len(kinds)))](rng, n) for _ in range(I)])
        row = []
        for _ in range(I):
            taps = []
            for _ in range(J):
                if rng.random() < 0.05:
                    taps.append(np.zeros(0, np.float32))
                    continue
                L0 = int(rng.integers(1, 3000))
                taps.append(synth.rir(rng, L0, float(rng.uniform(0.1, 0.9)), int(rng.integers(0, min(L0, 200)))))
            row.append(taps)
        rirs.append(row)
        snrs.append([0.0] + [float(rng.uniform(0.0, 30.0)) for _ in range(I - 1)])
    return synth.pack(srcs, rirs, snrs, J), rng


def _forced(b, rng, with_hop):
    """A random valid FFT size per utterance (and hop): N at least the longest
    uncut RIR, which bounds every cut length; the hop at most N - L0 + 1."""
    S, J = b.max_src, b.n_mic
    l2 = np.zeros(b.n_utt, np.int32)
    hop = np.zeros(b.n_utt, np.int32)
    for u in range(b.n_utt):
        I = int(b.n_src[u])
        lmax0 = max([int(b.rir_len0[(u * S + i) * J + j]) for i in range(I) for j in range(J)], default=0)
        lo = max(9, math.ceil(math.log2(max(lmax0, 1))))
        l2[u] = int(rng.integers(lo, 16))
        room = (1 << int(l2[u])) - max(lmax0, 1) + 1
        hop[u] = int(rng.integers(max(1, room // 4), room + 1))
    return l2, (hop if with_hop else None)


@pytest.mark.gpu
@pytest.mark.parametrize("k", range(24))
def test_random_batch_forward_and_adjoint(k):
    cuda()
    b, rng = _random_batch(k)
    eta = ETAS[k % len(ETAS)]
    mode = MODES[(k + k // len(ETAS)) % len(MODES)]
    l2, hop = _forced(b, rng, mode == "sizes+hop") if mode.startswith("sizes") else (None, None)
    order = rng.permutation(b.n_utt).astype(np.int32) if mode == "order" else None
    print(f"batch {k}: U={b.n_utt} J={b.n_mic} S={b.max_src} eta={eta} mode={mode}", flush=True)
    db, alpha, y, rl, ol = _simulate(b, eta, fft_log2n=l2, hop=hop, order=order, use_graph=mode == "graph")
    _check_utterances(b, range(b.n_utt), eta, y, rl, ol)
    gx, gh, ga, gys = _run(b, eta, 100 + k, fft_log2n=l2, hop=hop)
    _check_full_many(b, eta, gx, gh, ga, gys, list(range(b.n_utt)))


@pytest.mark.gpu
@pytest.mark.parametrize("k", range(8))
def test_random_batch_energies(k):
    # the reverberant energies of every (source, mic) slot after the cut, at
    # the energy bar of the reverberant-gain tests
    from tests.test_gpu_reverb import _check_energies, _energies

    b, _ = _random_batch(100 + k)
    eta = ETAS[k % len(ETAS)]
    print(f"batch {100 + k}: U={b.n_utt} J={b.n_mic} S={b.max_src} eta={eta}", flush=True)
    _, e, rl = _energies(b, eta)
    _check_energies(b, eta, e, rl)


@pytest.mark.gpu
@pytest.mark.parametrize("k", range(8))
def test_random_batch_features(k):
    # the front end on the mixed outputs and fused into the mix, at the
    # feature bars of the front-end tests against the oracle's features of
    # the unfused kernel's samples.  Sizes are forced per utterance among
    # those with a fused kernel (4096-16384), so that both paths run the same
    # transforms: the fused features must then equal the separate ones bit
    # for bit (with the size rule free, short RIRs can get a smaller N on the
    # separate path, whose samples then differ by rounding)
    from tests.test_gpu_logmel import _compare_fused, _fused

    b, rng = _random_batch(200 + k)
    eta = ETAS[k % len(ETAS)]
    l2 = rng.integers(12, 15, b.n_utt).astype(np.int32)
    print(f"batch {200 + k}: U={b.n_utt} J={b.n_mic} S={b.max_src} eta={eta}", flush=True)
    ref, feat_f, off, cap, ol, rl = _fused(b, eta, fft_log2n=l2, use_graph=bool(k % 2))
    assert _compare_fused(b, ref, feat_f, off, cap, ol, rl)


def _random_rir(rng):
    """A RIR of a random shape: decaying noise, spikes, silence, plateaus of
    equal taps, huge or tiny scales (subnormal powers), lengths around the
    cut kernel's chunking and past its 32768-tap chunk maxima."""
    L0 = int(rng.choice([0, 1, 2, 63, 64, 65, 1023, 1024, 1025, 32768, 32769])) if rng.random() < 0.2 \
        else int(rng.integers(1, 40000))
    kind = int(rng.integers(5))
    n = np.arange(L0)
    if kind == 0:
        h = rng.standard_normal(L0) * np.exp(-n / max(1.0, float(rng.uniform(1, L0 + 1))))
    elif kind == 1:
        h = np.zeros(L0)
        for _ in range(int(rng.integers(1, 6))):
            if L0:
                h[int(rng.integers(L0))] = float(rng.choice([-1.0, 1.0])) * float(rng.uniform(0.1, 2.0))
    elif kind == 2:
        h = np.full(L0, float(rng.uniform(-1, 1)))                  # every tap equal
    elif kind == 3:
        h = rng.standard_normal(L0) * 10.0 ** float(rng.uniform(-25, -19))   # subnormal powers
    else:
        h = rng.standard_normal(L0) * 10.0 ** float(rng.uniform(10, 18))     # powers near the float32 top
    return h.astype(np.float32)


@pytest.mark.gpu
@pytest.mark.parametrize("k", range(4))
def test_random_rirs_cut_bit_exact(k):
    # 300 random RIR shapes per call and thresholds anywhere in 0-60 dB (not
    # only round values): n_c and L bit-exact against the oracle's rule
    from tests.test_gpu_truncate import _run as cut

    rng = synth.rng_for(300, k)
    rirs = [_random_rir(rng) for _ in range(300)]
    for eta in [float(rng.uniform(0.0, 60.0)) for _ in range(3)] + [0.0, math.inf]:
        n_c, L = cut(rirs, eta)
        for r, h in enumerate(rirs):
            nc_ref, L_ref, _ = oracle.cut_rir(h, eta)
            assert (int(n_c[r]), int(L[r])) == (nc_ref, L_ref), (k, eta, r, len(h))


@pytest.mark.gpu
@pytest.mark.parametrize("k", range(6))
def test_random_batch_full_length_filtering(k):
    # eqs. 4-5 on random batches, every utterance at its own transform size
    # (grouped into one call per size), against the oracle's mix
    from tests.test_gpu_fft_filter import _check, _run as ffilter

    b, _ = _random_batch(400 + k)
    eta = ETAS[k % len(ETAS)]
    print(f"batch {400 + k}: U={b.n_utt} J={b.n_mic} S={b.max_src} eta={eta}", flush=True)
    y, rl, ol, alpha = ffilter(b, eta, chunk=int(1 + k % 4))
    _check(b, eta, y, rl, ol, alpha, range(b.n_utt))


@pytest.mark.gpu
@pytest.mark.parametrize("k", range(6))
def test_random_batch_kernel_variants_same_bits(k):
    # forced sizes per utterance over every family and a random kernel variant
    # per family, three times: each choice gives the bits of the default
    # variants (every variant computes each sample with the same operations)
    torch = cuda()
    from paper_1712_03439_amd import autotune, rsim

    b, rng = _random_batch(600 + k)
    eta = ETAS[k % len(ETAS)]
    l2 = _forced(b, rng, bool(k % 2))
    f, m = autotune.model_costs()

    def run(var):
        db = rsim.DeviceBatch(b, fft_log2n=l2[0], hop=l2[1])
        alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
        y = rsim.simulate(db, alpha, eta, tune=rsim.tune_table(f, m, False, var), use_graph=bool(var[0] % 2))
        torch.cuda.synchronize()
        return y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()

    y0, rl0, ol0 = run([0] * 6)
    for _ in range(3):
        var = [int(rng.choice(autotune.VARIANTS[fam])) for fam in range(6)]
        y, rl, ol = run(var)
        assert np.array_equal(rl, rl0) and np.array_equal(ol, ol0)
        for u in range(b.n_utt):
            off, st, T = int(b.out_off[u]), int(b.out_stride[u]), int(ol0[u])
            for j in range(b.n_mic):
                s = slice(off + j * st, off + j * st + T)
                assert np.array_equal(y[s].view(np.uint32), y0[s].view(np.uint32)), (var, u, j)


def _wide_batch(k):
    """Wider shapes: up to 40 utterances, 16 mics and 8 sources, sources of
    up to 60000 samples and RIRs of up to 16000 taps."""
    rng = synth.rng_for(61, k)
    U = int(rng.integers(1, 41))
    J = int(rng.integers(1, 17))
    srcs, rirs, snrs = [], [], []
    for _ in range(U):
        I = int(rng.integers(0, 9))
        n = int(rng.integers(1, 60000))
        srcs.append([(synth.white_noise if rng.random() < 0.5 else synth.speech_like)(rng, n) for _ in range(I)])
        rirs.append([[synth.rir(rng, int(rng.integers(0, 16001)), float(rng.uniform(0.1, 1.0)),
                                int(rng.integers(0, 300))) for _ in range(J)] for _ in range(I)])
        snrs.append([0.0] + [float(rng.uniform(0, 30)) for _ in range(I - 1)])
    return synth.pack(srcs, rirs, snrs, J)


@pytest.mark.gpu
@pytest.mark.parametrize("k", [0, 12, 18])
def test_wide_random_batch_forward_adjoint_energies(k):
    # up to 15 mics and 8 sources: the forward and the adjoint in full and the
    # reverberant energies, all against the oracle
    from tests.test_gpu_reverb import _check_energies, _energies

    b = _wide_batch(k)
    eta = ETAS[k % len(ETAS)]
    print(f"wide batch {k}: U={b.n_utt} J={b.n_mic} S={b.max_src} eta={eta}", flush=True)
    db, alpha, y, rl, ol = _simulate(b, eta, use_graph=bool(k % 2))
    _check_utterances(b, range(b.n_utt), eta, y, rl, ol)
    gx, gh, ga, gys = _run(b, eta, 900 + k)
    _check_full_many(b, eta, gx, gh, ga, gys, list(range(b.n_utt)))
    _, e, rl2 = _energies(b, eta)
    _check_energies(b, eta, e, rl2)


@pytest.mark.gpu
def test_random_ola_shapes():
    # rsim_ola_convolve on 40 random (signal, RIR, FFT size, hop) shapes,
    # the hop anywhere from 1 to its largest value N - L + 1
    torch = cuda()
    from paper_1712_03439_amd import rsim

    rng = synth.rng_for(700, 0)
    for k in range(40):
        l2 = int(rng.integers(9, 16))
        N = 1 << l2
        nh = int(rng.integers(1, N + 1))
        nx = int(rng.integers(1, 5 * N))
        hop = int(rng.integers(1, N - nh + 2)) if rng.random() < 0.5 else 0
        x = rng.standard_normal(nx).astype(np.float32)
        h = (rng.standard_normal(nh) * np.exp(-np.arange(nh) / (nh / 3 + 1))).astype(np.float32)
        y = rsim.ola_convolve(torch.from_numpy(x).cuda(), torch.from_numpy(h).cuda(), N, hop).cpu().numpy()
        ref = oracle.convolve(x, h)
        assert y.shape == ref.shape, (k, nx, nh, N, hop)
        assert max_rel_err(y, ref) <= TOL, (k, nx, nh, N, hop, max_rel_err(y, ref))
