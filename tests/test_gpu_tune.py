"""Kernel variants and the measuring tuner on the GPU.

Every variant of the filter-and-mix kernel computes each output sample with the
same operations in the same order, so their outputs are bit-identical; one of
them is checked against the FP64 oracle (bar: 1e-5 of the peak per
utterance and mic).  The tuner's table must drive a correct mix."""
import numpy as np
import pytest

import synth
from tests.gpu_util import cuda
from tests.test_gpu_mix import _check_utterances


def _batch(n_utt, J, seed, len_s=(0.2, 1.5), taps=(300, 3000)):
    rng = synth.rng_for(60, seed)
    srcs, rirs, snrs = [], [], []
    for u in range(n_utt):
        I = 1 + int(rng.integers(0, 4))
        n = int(rng.uniform(*len_s) * 16000)
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(I - 1)])
        L0 = int(rng.integers(*taps))
        rirs.append([[synth.rir(rng, L0, 0.3, int(rng.integers(20, 200))) for _ in range(J)] for _ in range(I)])
        snrs.append([0.0] + [float(v) for v in rng.uniform(0, 30, I - 1)])
    return synth.pack(srcs, rirs, snrs, J)


def _run(b, l2, variant_code, eta=20.0):
    torch = cuda()
    from paper_1712_03439_amd import autotune, rsim

    f, m = autotune.model_costs()
    var = [0] * 6
    var[autotune.FAMILY[l2]] = variant_code
    tune = rsim.tune_table(f, m, True, var)
    db = rsim.DeviceBatch(b, fft_log2n=np.full(b.n_utt, l2, np.int32))
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    y = rsim.simulate(db, alpha, eta, tune=tune)
    torch.cuda.synchronize()
    return y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()


def _same_outputs(b, ya, yb, out_len):
    for u in range(b.n_utt):
        off, st, T = int(b.out_off[u]), int(b.out_stride[u]), int(out_len[u])
        for j in range(b.n_mic):
            s = slice(off + j * st, off + j * st + T)
            if not np.array_equal(ya[s], yb[s]):
                return (u, j)
    return None


@pytest.mark.gpu
@pytest.mark.parametrize("n_utt", [5, 300])
def test_every_kernel_variant_gives_the_same_bits(n_utt):
    # 3 mics (two-mic passes leave one over); 5 utterances split into mic-group
    # work items, 300 (more than the compute units) do not
    b = _batch(n_utt, 3, n_utt)
    from paper_1712_03439_amd import autotune

    for l2 in (12, 13, 14):
        ref, rl, ol = _run(b, l2, 2)
        for code in autotune.VARIANTS[autotune.FAMILY[l2]]:
            if code == 2:
                continue
            y, rl2, ol2 = _run(b, l2, code)
            assert np.array_equal(rl, rl2) and np.array_equal(ol, ol2)
            assert _same_outputs(b, ref, y, ol) is None, (l2, code, _same_outputs(b, ref, y, ol))
        _check_utterances(b, (0, n_utt // 2, n_utt - 1), 20.0, ref, rl, ol)


@pytest.mark.gpu
def test_variant_one_mic_per_pass_against_the_oracle():
    b = _batch(6, 4, 7)
    for l2 in (13, 14):
        y, rl, ol = _run(b, l2, 1)
        _check_utterances(b, range(b.n_utt), 20.0, y, rl, ol)


@pytest.mark.gpu
def test_tuner_table_drives_a_correct_mix():
    torch = cuda()
    from paper_1712_03439_amd import autotune, rsim

    b = synth.make_config2(n_utt=96, epoch=3)
    db = rsim.DeviceBatch(b)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    rsim.truncate_batch(db, 20.0)
    tune, entry = autotune.tune(db, alpha, min_probe=16, reps=2)
    assert all(0 <= v <= 4 for v in entry["variant"]) and entry["variant"][5] in (0, 4)
    assert all(c >= 0 and np.isfinite(c) for c in entry["cost_fft"] + entry["cost_mac"])
    sizes = {int(m): r for m, r in entry["measured"]["sizes"].items()}
    shapes = autotune.batch_shapes(db)
    assert 15 in sizes and sizes[15]["utterances"] == len(shapes)
    # the one-size rule under the fitted table: if its size was timed on the
    # whole batch, no other size timed on the whole batch ran faster
    hs = [(nx, I, J, L) for _, nx, I, J, L in shapes]
    m_star = autotune.batch_log2n(hs, entry["cost_fft"], entry["cost_mac"])
    # with one size per batch the sizes below it are disabled, the rest kept
    if entry["one_size"]:
        assert entry["sizes_from"] == m_star
        for m in autotune.LOG2N:
            assert (entry["cost_fft"][m - 9] > 0) == (m >= m_star)
    whole = {m: r["ms"][str(entry["variant"][autotune.FAMILY[m]])] for m, r in sizes.items()
             if r["utterances"] == len(shapes)}
    if m_star in whole:
        assert whole[m_star] <= min(whole.values()) * (1 + 1e-9), (m_star, whole)
    # the tuned table (sizes and variants) gives correct outputs
    y = rsim.simulate(db, alpha, 20.0, tune=tune)
    torch.cuda.synchronize()
    y, rl, ol = y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()
    _check_utterances(b, range(0, b.n_utt, 4), 20.0, y, rl, ol)
