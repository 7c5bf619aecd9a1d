"""rsim_simulate_static (the entry point for callers that cannot allocate: its
workspace is the library's static scratch) against rsim_simulate on the same
batches.  Both compute every output sample with the same operations, so the
outputs, cut lengths and output lengths must be bit-identical; two
utterances of each batch are also checked against the FP64 oracle (bar:
1e-5 of the peak per utterance and mic)."""
import math

import numpy as np
import pytest

import synth
from tests.gpu_util import cuda
from tests.test_gpu_mix import _check_utterances


def _reference(b, eta, tune=None, fft_log2n=None):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    db = rsim.DeviceBatch(b, fft_log2n=fft_log2n)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    y = rsim.simulate(db, alpha, eta, tune=tune)
    torch.cuda.synchronize()
    return db, alpha, y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()


def _static(db, alpha, eta, tune=None):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    db.rir_len.fill_(-1)
    db.out_len.fill_(-1)
    y = torch.full((max(db.y_len, 1),), float("nan"), device=db.device)
    rsim.simulate_static(db, alpha, eta, y, tune=tune)
    return y


def _same(b, y_ref, rl_ref, ol_ref, y, rl, ol):
    assert np.array_equal(rl_ref, rl) and np.array_equal(ol_ref, ol)
    for u in range(b.n_utt):
        off, st, T = int(b.out_off[u]), int(b.out_stride[u]), int(ol[u])
        for j in range(b.n_mic):
            s = slice(off + j * st, off + j * st + T)
            assert np.array_equal(y_ref[s], y[s]), (u, j)


@pytest.mark.gpu
def test_static_entry_matches_simulate_on_two_calls_in_a_row():
    # a 48-utterance batch, then a smaller one: the second call reuses the
    # scratch the first left behind
    torch = cuda()
    big = synth.make_config2(n_utt=48, epoch=21)
    small = synth.make_config2(n_utt=6, epoch=22)
    refs = [_reference(b, 20.0) for b in (big, small)]
    outs = []
    for (db, alpha, *_r) in refs:
        y = _static(db, alpha, 20.0)
        torch.cuda.synchronize()
        outs.append((y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()))
    for b, (db, alpha, y_ref, rl_ref, ol_ref), (y, rl, ol) in zip((big, small), refs, outs):
        _same(b, y_ref, rl_ref, ol_ref, y, rl, ol)
        _check_utterances(b, (0, b.n_utt - 1), 20.0, y, rl, ol)


def _wide(n_utt, seed):
    # 4 sources and 8 mics per utterance: one work item's slot of RIR spectra
    # at N = 32768 is 36 spectra of 16384 bins (4.7 MB)
    rng = synth.rng_for(24, seed)
    srcs, rirs = [], []
    for u in range(n_utt):
        n = int(rng.integers(500, 3000))
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(3)])
        rirs.append([[synth.rir(rng, int(rng.integers(5, 200)), 0.1, 0) for _ in range(8)] for _ in range(4)])
    return synth.pack(srcs, rirs, [[0.0, 5.0, 10.0, 20.0]] * n_utt, 8)


@pytest.mark.gpu
def test_static_entry_with_fewer_workgroups_than_slots_wanted():
    # more utterances than the block split's threshold, at N = 32768 with 8
    # mics: the persistent grid's scratch slots would need several times the
    # static array, so fewer workgroups run; a smaller batch follows
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b1 = _wide(1100, 0)
    b2 = _wide(40, 1)
    l2a, l2b = np.full(b1.n_utt, 15, np.int32), np.full(b2.n_utt, 15, np.int32)
    db1, a1, y1_ref, rl1_ref, ol1_ref = _reference(b1, math.inf, fft_log2n=l2a)
    assert db1.workspace_bytes() > 2 * rsim.STATIC_SCRATCH_BYTES
    db2, a2, y2_ref, rl2_ref, ol2_ref = _reference(b2, 30.0, fft_log2n=l2b)
    y1 = _static(db1, a1, math.inf)
    y2 = _static(db2, a2, 30.0)
    torch.cuda.synchronize()
    _same(b1, y1_ref, rl1_ref, ol1_ref, y1.cpu().numpy(), db1.rir_len.cpu().numpy(), db1.out_len.cpu().numpy())
    _same(b2, y2_ref, rl2_ref, ol2_ref, y2.cpu().numpy(), db2.rir_len.cpu().numpy(), db2.out_len.cpu().numpy())
    _check_utterances(b1, (0, 1099), math.inf, y1.cpu().numpy(), db1.rir_len.cpu().numpy(), db1.out_len.cpu().numpy())
    _check_utterances(b2, (0,), 30.0, y2.cpu().numpy(), db2.rir_len.cpu().numpy(), db2.out_len.cpu().numpy())


@pytest.mark.gpu
def test_static_entry_on_a_run_of_random_batches():
    # eight seeded random batches in a row (1-27 utterances, 1-8 mics, 0-4
    # sources, forced sizes per utterance in half of them): each call's
    # scratch layout differs from the previous one's, and every call must
    # give the bits of rsim_simulate
    torch = cuda()
    from tests.test_gpu_random import ETAS, _forced, _random_batch

    for k in range(8):
        b, rng = _random_batch(500 + k)
        eta = ETAS[k % len(ETAS)]
        l2 = _forced(b, rng, False)[0] if k % 2 else None
        db, alpha, y_ref, rl_ref, ol_ref = _reference(b, eta, fft_log2n=l2)
        y = _static(db, alpha, eta)
        torch.cuda.synchronize()
        _same(b, y_ref, rl_ref, ol_ref, y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy())


@pytest.mark.gpu
def test_static_entry_captured_in_a_graph():
    # the callers the entry is for include code under graph capture: the call
    # is captured into a torch CUDA graph and replayed three times, the
    # inputs changed in place by eager work between the replays; every
    # replay gives the bits of rsim_simulate on the inputs of that moment
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=10, epoch=50)
    l2 = np.where(np.arange(b.n_utt) % 2 == 0, 13, 14).astype(np.int32)   # two families
    db = rsim.DeviceBatch(b, fft_log2n=l2)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    y = torch.zeros(max(db.y_len, 1), device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rsim.simulate_static(db, alpha, 20.0, y, stream=s)   # first use on the device before capture
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rsim.simulate_static(db, alpha, 20.0, y, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.no_grad():
            db.x.mul_(0.5 + rep)
            db.h.neg_()
        torch.cuda.synchronize()
        y.zero_()
        g.replay()
        torch.cuda.synchronize()
        got, rl, ol = y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()
        ref = rsim.simulate(db, alpha, 20.0, y=torch.zeros_like(y))
        torch.cuda.synchronize()
        assert np.array_equal(rl, db.rir_len.cpu().numpy()) and np.array_equal(ol, db.out_len.cpu().numpy())
        assert np.array_equal(got.view(np.uint32), ref.cpu().numpy().view(np.uint32)), rep
    assert rsim.device_status() == 0


@pytest.mark.gpu
def test_static_entry_rejects_a_batch_that_does_not_fit():
    # 64 sources x 64 mics forced to N = 32768: one workgroup's slot of RIR
    # spectra alone is larger than the static array; nothing is launched
    torch = cuda()
    from paper_1712_03439_amd import rsim

    rng = synth.rng_for(23, 0)
    srcs = [[synth.white_noise(rng, 200) for _ in range(64)]]
    rirs = [[[synth.rir(rng, 8, 0.1, 0) for _ in range(64)] for _ in range(64)]]
    b = synth.pack(srcs, rirs, [[0.0] * 64], 64)
    db = rsim.DeviceBatch(b, fft_log2n=np.array([15], np.int32))
    alpha = torch.ones(64 * 64, device="cuda")
    with pytest.raises(rsim.RsimError) as e:
        _static(db, alpha, 20.0)
    assert e.value.code == rsim.RSIM_EWORKSPACE
    torch.cuda.synchronize()
    assert int(db.rir_len.min()) == -1 and int(db.out_len.min()) == -1  # untouched
