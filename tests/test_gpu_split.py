"""The forward's block split (batches with fewer work items than compute
units: each utterance's blocks are divided into ranges run by different
workgroups, their RIR spectra formed by a pass of their own, and the samples
where two ranges overlap summed by a pass after the kernel).

The split changes no floating-point operation of an output sample (the
overlap sum adds the same two operands), so a batch run split must give the
same bits as the same utterances run in a batch large enough not to split;
and every output is checked against the FP64 oracle (bar: 1e-5 of the peak
per utterance and mic)."""
import math

import numpy as np
import pytest

import synth
from tests.gpu_util import cuda
from tests.test_gpu_mix import _check_utterances, _large_subset, _simulate


def _many(n_utt, seed, l2, n_mic=3):
    rng = synth.rng_for(70, seed)
    srcs, rirs, snrs = [], [], []
    for u in range(n_utt):
        I = 1 + u % 2
        n = int(rng.integers(3000, 12000))
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(I - 1)])
        L0 = int(rng.integers(20, 900))
        rirs.append([[synth.rir(rng, L0, 0.2, int(rng.integers(0, 20))) for _ in range(n_mic)] for _ in range(I)])
        snrs.append([0.0] + [float(v) for v in rng.uniform(0, 20, I - 1)])
    return synth.pack(srcs, rirs, snrs, n_mic)


def _same_bits(big, pick, y_big, ol_big, small, y_small, ol_small):
    for k, u in enumerate(pick):
        assert int(ol_small[k]) == int(ol_big[u])
        T = int(ol_big[u])
        for j in range(big.n_mic):
            a = y_big[int(big.out_off[u]) + j * int(big.out_stride[u]):][:T]
            b = y_small[int(small.out_off[k]) + j * int(small.out_stride[k]):][:T]
            assert np.array_equal(a, b), (u, j)


@pytest.mark.gpu
def test_split_gives_the_bits_of_the_unsplit_kernel():
    # 1200 utterances (more work items than the split's threshold: one work
    # item per utterance) against 5 of them alone (split into block ranges)
    big = _many(1200, 0, 11)
    pick = [0, 7, 301, 777, 1199]
    small = synth.subset(big, pick)
    l2 = 11
    _, _, y_big, rl_big, ol_big = _simulate(big, 20.0, fft_log2n=np.full(big.n_utt, l2, np.int32))
    _, _, y_small, rl_small, ol_small = _simulate(small, 20.0, fft_log2n=np.full(small.n_utt, l2, np.int32))
    _same_bits(big, pick, y_big, ol_big, small, y_small, ol_small)
    _check_utterances(small, range(small.n_utt), 20.0, y_small, rl_small, ol_small)


@pytest.mark.gpu
def test_split_with_several_mic_groups_per_work_item():
    # 400 utterances with 5 mics: more utterances than compute units, so a
    # work item runs all three mic groups (the block's source spectra cached
    # in its slot for the later groups), and fewer than four items per
    # compute unit, so the blocks are split as well; against the same
    # utterances in a 1200-utterance batch (not split)
    big = _many(1200, 1, 11, n_mic=5)
    pick = list(range(0, 1200, 3))[:400]
    small = synth.subset(big, pick)
    _, _, y_big, rl_big, ol_big = _simulate(big, 20.0, fft_log2n=np.full(big.n_utt, 11, np.int32))
    _, _, y_small, rl_small, ol_small = _simulate(small, 20.0, fft_log2n=np.full(small.n_utt, 11, np.int32))
    _same_bits(big, pick, y_big, ol_big, small, y_small, ol_small)
    _check_utterances(small, (0, 199, 399), 20.0, y_small, rl_small, ol_small)


@pytest.mark.gpu
@pytest.mark.parametrize("graph", [False, True])
def test_one_long_utterance_split_every_family(graph):
    # one 20 s utterance with 4 sources and 8 mics at every transform size it
    # fits (the 32768-point family included), eager and as a graph
    b = _large_subset(1, 5)
    for l2 in (13, 14, 15):
        db, alpha, y, rl, ol = _simulate(b, math.inf if l2 == 15 else 20.0, fft_log2n=np.array([l2], np.int32),
                                         use_graph=graph)
        _check_utterances(b, [0], math.inf if l2 == 15 else 20.0, y, rl, ol)


@pytest.mark.gpu
def test_split_with_a_hop_below_the_rir_keeps_one_range():
    # a forced hop shorter than the kept RIR: every output sample gets the
    # tails of several blocks, so the utterance is not split
    rng = synth.rng_for(71, 0)
    srcs = [[synth.speech_like(rng, 30000), synth.white_noise(rng, 30000)]]
    rirs = [[[synth.rir(rng, 3000, 0.4, 10)] * 2, [synth.rir(rng, 2500, 0.4, 5)] * 2]]
    b = synth.pack(srcs, rirs, [[0.0, 6.0]], 2)
    db, alpha, y, rl, ol = _simulate(b, math.inf, fft_log2n=np.array([13], np.int32), hop=np.array([1000], np.int32))
    _check_utterances(b, [0], math.inf, y, rl, ol)
