"""Reverberant-at-mic gains on the GPU (rsim_reverb_energy) against the FP64
oracle.

Bar: |E_gpu - E_ref| <= 1e-5 E_ref for every (source, mic) slot, the bar of
the mix's outputs applied to the energy itself.  The energy is
sum_l r_hh[l] r_xx[l] with r_xx accumulated by float32 transforms, so the
error scales with float32 rounding times sum_l |r_hh[l]| r_xx[0], a few tens
of times E for noise-like RIRs; measured on the batched workload it stays
below 6e-7 E (20 times inside the bar).  The gains then agree to 1e-5
relative and give the requested SNR to 1e-4 dB."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import TOL, cuda, max_rel_err


def _energies(b, eta):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    db = rsim.DeviceBatch(b)
    rsim.truncate_batch(db, eta)
    e = rsim.reverb_energy(db)
    torch.cuda.synchronize()
    return db, e.cpu().numpy(), db.rir_len.cpu().numpy()


def _check_energies(b, eta, e, rl):
    S, J = b.max_src, b.n_mic
    for u in range(b.n_utt):
        xs, hs = b.sources(u), b.rirs(u)
        for i in range(S):
            for j in range(J):
                r = (u * S + i) * J + j
                if i >= len(xs):
                    assert e[r] == 0.0, (u, i, j)
                    continue
                L = int(rl[r])
                assert L == oracle.cut_rir(hs[i][j], eta)[1]
                h = np.asarray(hs[i][j], np.float64)[:L]
                x = np.asarray(xs[i], np.float64)
                ref = oracle.reverb_energy(x, h)
                assert abs(e[r] - ref) <= TOL * ref + 1e-30, (u, i, j, e[r], ref)


@pytest.mark.gpu
def test_energies_of_a_batch():
    b = synth.make_config2(n_utt=24, epoch=7)
    _, e, rl = _energies(b, 20.0)
    _check_energies(b, 20.0, e, rl)


@pytest.mark.gpu
def test_energies_at_every_transform_size():
    # longest kept RIR 1 .. 16384 taps: transforms of 512 .. 32768 points
    rng = synth.rng_for(61, 0)
    srcs, rirs, snrs = [], [], []
    for L in (1, 7, 255, 256, 257, 1000, 4096, 4097, 8192, 8193, 12000, 16384):
        I = 1 + len(srcs) % 3
        n = int(rng.integers(200, 30000))
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(I - 1)])
        rirs.append([[synth.rir(rng, L if j == 0 else max(1, L // (j + 2)), 0.5, 0) for j in range(3)]
                     for _ in range(I)])
        snrs.append([0.0] + [float(v) for v in rng.uniform(0, 30, I - 1)])
    b = synth.pack(srcs, rirs, snrs, 3)
    _, e, rl = _energies(b, math.inf)
    _check_energies(b, math.inf, e, rl)


@pytest.mark.gpu
def test_gains_give_the_requested_snr_and_drive_the_mix():
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=8, epoch=8)
    db, e, rl = _energies(b, 20.0)
    S, J = b.max_src, b.n_mic
    alpha = rsim.batch_gains_reverb(db, b.snr_db, e)
    y = rsim.mix(db, torch.from_numpy(alpha).cuda())
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    ol = db.out_len.cpu().numpy()
    for u in range(b.n_utt):
        xs, hs = b.sources(u), b.rirs(u)
        I = len(xs)
        cut = [[np.asarray(hs[i][j], np.float32)[: int(rl[(u * S + i) * J + j])] for j in range(J)]
               for i in range(I)]
        E = np.array([[oracle.reverb_energy(xs[i], cut[i][j]) for j in range(J)] for i in range(I)])
        ref_a = oracle.snr_gains_reverb(E, b.snrs(u))
        got_a = alpha[u * S * J:(u * S + I) * J].reshape(I, J).astype(np.float64)
        assert np.allclose(got_a, ref_a, rtol=1e-5, atol=0), u
        for i in range(1, I):
            for j in range(J):
                snr = 10 * math.log10(E[0, j] / (got_a[i, j] ** 2 * E[i, j]))
                assert abs(snr - b.snrs(u)[i]) <= 1e-4, (u, i, j)
        # the mix with these gains (the oracle mixes with the same float32 gains)
        ref = oracle.mix(xs, cut, got_a)
        off, st = int(b.out_off[u]), int(b.out_stride[u])
        T = ref.shape[1]
        assert int(ol[u]) == T
        for j in range(J):
            assert max_rel_err(y[off + j * st: off + j * st + T], ref[j]) <= TOL, (u, j)


@pytest.mark.gpu
def test_kept_rir_longer_than_the_largest_transform_is_flagged():
    torch = cuda()
    from paper_1712_03439_amd import rsim

    rng = synth.rng_for(62, 0)
    b = synth.pack([[synth.speech_like(rng, 5000)], [synth.speech_like(rng, 3000)]],
                   [[[synth.rir(rng, 20000, 0.9, 10)]], [[synth.rir(rng, 500, 0.2, 10)]]], [[0.0], [0.0]], 1)
    rsim.device_status()
    _, e, rl = _energies(b, math.inf)
    assert math.isnan(e[0]) and rsim.device_status() & rsim.DEV_BADPLAN
    ref = oracle.reverb_energy(b.sources(1)[0], b.rirs(1)[0][0])
    assert abs(e[b.max_src] - ref) <= 1e-4 * ref


@pytest.mark.gpu
def test_energies_of_more_slots_than_the_cost_cache_holds():
    # 9000 utterances x 4 source slots = 36000 slots, more than the LDS cost
    # cache of a workgroup holds (the balanced ranges are then computed from
    # the descriptors twice); short sources, few taps, some empty slots
    rng = synth.rng_for(63, 0)
    srcs, rirs, snrs = [], [], []
    for u in range(9000):
        I = 4 if u == 4321 else 1 + (u % 7 == 0)
        n = int(rng.integers(50, 300))
        srcs.append([synth.white_noise(rng, n) for _ in range(I)])
        rirs.append([[synth.rir(rng, int(rng.integers(1, 40)), 0.2, 0)] for _ in range(I)])
        snrs.append([0.0] * I)
    b = synth.pack(srcs, rirs, snrs, 1)
    assert b.n_utt * b.max_src > 35000
    _, e, rl = _energies(b, math.inf)
    _check_energies(b, math.inf, e, rl)
