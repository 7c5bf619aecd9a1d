"""Overlap-add filtering and eq. (2) mixing on the GPU against the FP64 oracle.

Bar: per (utterance, mic), max |y_gpu - y_ref| <= 1e-5 * max |y_ref|; the cut
lengths are bit-exact; out_len = Nx + max L - 1."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import oracle_pool
from tests.gpu_util import TOL, cuda, max_rel_err


def _ola(x, h, n, hop=0):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    y = rsim.ola_convolve(torch.from_numpy(np.asarray(x, np.float32)).cuda(),
                          torch.from_numpy(np.asarray(h, np.float32)).cuda(), n, hop)
    return y.cpu().numpy()


@pytest.mark.gpu
def test_tiny_config_full():
    # 1 s speech-like source, 4096-tap RIR (direct path at 40), FFT 8192, hop 4096.
    b = synth.make_config0()
    x = b.sources(0)[0]
    h = b.rirs(0)[0][0]
    y = _ola(x, h, 8192, 4096)
    ref = oracle.convolve(x, h)
    assert y.shape == (20095,) and ref.shape == (20095,)
    assert max_rel_err(y, ref) <= TOL


@pytest.mark.gpu
@pytest.mark.parametrize("nx,nh,n,hop", [
    (1, 1, 512, 0), (5, 3, 512, 0), (700, 100, 512, 0), (10000, 257, 512, 256),
    (3000, 1000, 2048, 0), (3001, 999, 2048, 100),      # hop far below the tail: many overlaps
    (20000, 4096, 8192, 0), (16000, 4096, 8192, 4097), (50000, 5000, 16384, 0),
    (40000, 12000, 32768, 0), (12345, 777, 4096, 0), (9999, 1, 1024, 0), (100, 500, 1024, 0),
])
def test_ola_shapes(nx, nh, n, hop):
    rng = np.random.default_rng(nx * 7 + nh)
    x = rng.standard_normal(nx).astype(np.float32)
    h = (rng.standard_normal(nh) * np.exp(-np.arange(nh) / (nh / 4 + 1))).astype(np.float32)
    y = _ola(x, h, n, hop)
    ref = oracle.convolve(x, h)
    assert y.shape == ref.shape
    assert max_rel_err(y, ref) <= TOL


@pytest.mark.gpu
def test_ola_delta_rir_is_a_delay():
    x = np.random.default_rng(3).standard_normal(30000).astype(np.float32)
    h = np.zeros(3000, np.float32)
    h[1234] = 1.0
    y = _ola(x, h, 8192)
    assert np.max(np.abs(y[1234:1234 + 30000] - x)) <= 1e-5 * np.max(np.abs(x))
    assert np.max(np.abs(y[:1234])) <= 1e-5 * np.max(np.abs(x))


def _simulate(b, eta, fft_log2n=None, hop=None, order=None, tune=None, use_graph=False):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    db = rsim.DeviceBatch(b, order=order, fft_log2n=fft_log2n, hop=hop)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    stream = torch.cuda.Stream() if use_graph else None
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            y = rsim.simulate(db, alpha, eta, tune=tune, use_graph=True)
    else:
        y = rsim.simulate(db, alpha, eta, tune=tune)
    torch.cuda.synchronize()
    return db, alpha.cpu().numpy(), y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()


def _oracle_case(b, u, eta, rir_len):
    """The oracle's inputs for utterance u: cut RIRs (lengths checked
    bit-exact against the GPU's), gains and output length."""
    J, S = b.n_mic, b.max_src
    xs = b.sources(u)
    hs = b.rirs(u)
    I = len(xs)
    cut = []
    for i in range(I):
        row = []
        for j in range(J):
            n_c, L, _ = oracle.cut_rir(hs[i][j], eta)
            assert int(rir_len[(u * S + i) * J + j]) == L, (u, i, j)
            row.append(np.asarray(hs[i][j], np.float32)[:L])
        cut.append(row)
    alpha = oracle.snr_gains([oracle.dry_power(x) for x in xs], b.snrs(u), J)
    T = oracle.out_length(len(xs[0]) if I else 0, [[len(c) for c in row] for row in cut])
    return xs, cut, alpha, T


def _check_utterances(b, utts, eta, y, rir_len, out_len):
    """Every output sample of the listed utterances against the oracle's mix
    (eq. 2), one (utterance, mic) per worker process: max |y - ref| <= TOL * max |ref|."""
    cases = {u: _oracle_case(b, u, eta, rir_len) for u in utts}
    for u, (xs, cut, alpha, T) in cases.items():
        assert int(out_len[u]) == T, (u, int(out_len[u]), T)

    pairs = [(u, j) for u in utts for j in range(b.n_mic) if cases[u][3] > 0]
    tasks = [(cases[u][0], [cases[u][1][i][j] for i in range(len(cases[u][0]))], cases[u][2][:, j], cases[u][3])
             for u, j in pairs]
    worst = 0.0
    for (u, j), ref in zip(pairs, oracle_pool.pmap(oracle_pool.mix_mic, tasks)):
        off, st, T = int(b.out_off[u]), int(b.out_stride[u]), cases[u][3]
        e = max_rel_err(y[off + j * st: off + j * st + T], ref)
        worst = max(worst, e)
        assert e <= TOL, (u, j, e)
    return worst


def _check_utterance(b, u, eta, y, rir_len, out_len):
    _check_utterances(b, [u], eta, y, rir_len, out_len)


@pytest.mark.gpu
def test_one_room_config_full():
    b = synth.make_config1()
    db, alpha, y, rl, ol = _simulate(b, 20.0)
    _check_utterance(b, 0, 20.0, y, rl, ol)


@pytest.mark.gpu
@pytest.mark.parametrize("eta", [20.0, math.inf])
def test_batched_subset(eta):
    b = synth.make_config2(n_utt=48)
    db, alpha, y, rl, ol = _simulate(b, eta)
    _check_utterances(b, range(b.n_utt), eta, y, rl, ol)


@pytest.mark.gpu
def test_batched_subset_graph_and_order():
    b = synth.make_config2(n_utt=24, epoch=3)
    order = np.argsort(-(b.src_len.astype(np.int64) * (b.n_src + b.n_mic)), kind="stable").astype(np.int32)
    db, alpha, y, rl, ol = _simulate(b, 20.0, order=order, use_graph=True)
    _check_utterances(b, range(b.n_utt), 20.0, y, rl, ol)


@pytest.mark.gpu
@pytest.mark.parametrize("l2", [9, 10, 11, 12, 13, 14, 15])
def test_forced_fft_sizes(l2):
    # every plan, four mics (two mic groups), sources that span several blocks
    rng = synth.rng_for(9, l2)
    srcs, rirs = [], []
    for u in range(3):
        n = int(rng.integers(3000, 30000))
        srcs.append([synth.speech_like(rng, n), synth.white_noise(rng, n)])
        L0 = int(rng.integers(50, min(2 ** l2 // 2, 6000)))
        rirs.append([[synth.rir(rng, L0, 0.4, 30) for _ in range(4)] for _ in range(2)])
    b = synth.pack(srcs, rirs, [[0.0, 12.0]] * 3, 4)
    db, alpha, y, rl, ol = _simulate(b, math.inf, fft_log2n=np.full(3, l2, np.int32))
    _check_utterances(b, range(3), math.inf, y, rl, ol)


@pytest.mark.gpu
def test_ragged_and_degenerate_utterances():
    rng = synth.rng_for(11, 0)
    srcs = [
        [synth.speech_like(rng, 1)],                                  # one sample
        [synth.speech_like(rng, 5000), synth.white_noise(rng, 5000)],
        [synth.speech_like(rng, 7000)],
        [synth.speech_like(rng, 333), synth.pink_noise(rng, 333), synth.white_noise(rng, 333)],
    ]
    z = np.zeros(0, np.float32)
    rirs = [
        [[synth.rir(rng, 100, 0.2, 5), synth.rir(rng, 1, 0.2, 0)]],
        [[synth.rir(rng, 900, 0.3, 20), z], [z, synth.rir(rng, 2000, 0.3, 40)]],   # empty RIRs
        [[z, z]],                                                     # nothing to convolve
        [[synth.rir(rng, 64, 0.1, 3)] * 2, [synth.rir(rng, 10, 0.1, 1)] * 2, [synth.rir(rng, 7, 0.1, 0)] * 2],
    ]
    b = synth.pack(srcs, rirs, [[0.0], [0.0, 5.0], [0.0], [0.0, 3.0, 9.0]], 2)
    db, alpha, y, rl, ol = _simulate(b, 20.0)
    _check_utterances(b, range(b.n_utt), 20.0, y, rl, ol)
    assert int(ol[2]) == 0


@pytest.mark.gpu
def test_a_batch_without_any_sample_is_accepted_everywhere():
    # three utterances without sources: x, h and y are empty, so their device
    # pointers are NULL; every entry point accepts the batch, writes zero
    # output lengths and flags nothing
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.pack([[], [], []], [[], [], []], [[0.0]] * 3, 2)
    db = rsim.DeviceBatch(b)
    assert db.x.numel() == 0 and db.h.numel() == 0 and b.y_len == 0
    rsim.device_status()
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    rsim.truncate_batch(db, 20.0)
    y = rsim.simulate(db, alpha, 20.0)
    rsim.mix(db, alpha, y=y)
    gx, gh, ga = rsim.mix_backward(db, alpha, torch.zeros(1, device="cuda"))
    e = rsim.reverb_energy(db)
    rsim.logmel(db, y)
    rsim.simulate_logmel(db, alpha, 20.0)
    rsim.fft_filter(db, alpha)
    rsim.simulate_static(db, alpha, 20.0, torch.zeros(1, device="cuda"))
    torch.cuda.synchronize()
    assert rsim.device_status() == 0
    assert not db.out_len.any() and not db.rir_len.any()
    assert gx.numel() == 0 and gh.numel() == 0 and not ga.any() and not e.any()


@pytest.mark.gpu
def test_bad_descriptor_is_skipped_and_flagged():
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=4, epoch=7)
    b.src_off = b.src_off.copy()
    b.src_off[1 * b.max_src] = 10 ** 12          # utterance 1 points outside x
    rsim.device_status()
    db, alpha, y, rl, ol = _simulate(b, 20.0)
    assert rsim.device_status() & rsim.DEV_BADDESC
    assert int(ol[1]) == 0
    for u in (0, 2, 3):
        _check_utterance(b, u, 20.0, y, rl, ol)


@pytest.mark.gpu
def test_status_read_on_the_calls_stream():
    # a bad descriptor mixed on a side stream: the status read with that
    # stream waits for the call and sees the flag, and the read clears it
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=3, epoch=8)
    b.src_off = b.src_off.copy()
    b.src_off[2 * b.max_src] = 10 ** 12          # utterance 2 points outside x
    rsim.device_status()
    db = rsim.DeviceBatch(b)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rsim.simulate(db, alpha, 20.0, stream=side)
    assert rsim.device_status(side) & rsim.DEV_BADDESC
    assert rsim.device_status(side) == 0
    assert int(db.out_len[2].item()) == 0


@pytest.mark.gpu
def test_a_given_stream_carries_the_calls_own_work():
    # calls given a side stream and no stream context: the binding's own
    # work (the adjoint's zero-filled gradients, the outputs and workspaces it
    # allocates) goes to that stream with the kernels, so the results equal
    # those of the same calls on the current stream, bit for bit
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=24, epoch=3)
    db = rsim.DeviceBatch(b)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    rsim.truncate_batch(db, 20.0)
    g = torch.sin(torch.arange(max(db.y_len, 1), device="cuda", dtype=torch.float32) * 0.01)
    x = torch.from_numpy(synth.white_noise(synth.rng_for(16, 0), 20000)).cuda()
    h = torch.from_numpy(synth.rir(synth.rng_for(16, 1), 3000, 0.4, 25)).cuda()
    outs = []
    for side in (None, torch.cuda.Stream()):
        torch.cuda.synchronize()
        y = rsim.mix(db, alpha, stream=side)
        grads = rsim.mix_backward(db, alpha, g, stream=side)
        c = rsim.ola_convolve(x, h, 8192, stream=side)
        (side if side is not None else torch.cuda.current_stream()).synchronize()
        ol = db.out_len.cpu().numpy()
        yv = y.cpu().numpy()
        parts = [yv[int(b.out_off[u]) + j * int(b.out_stride[u]):][:int(ol[u])]
                 for u in range(b.n_utt) for j in range(b.n_mic)]
        outs.append([np.concatenate(parts)] + [t.cpu().numpy() for t in grads] + [c.cpu().numpy()])
    for a, c in zip(*outs):
        assert np.array_equal(a.view(np.uint32), c.view(np.uint32))


@pytest.mark.gpu
def test_graph_and_eager_calls_agree_across_families():
    # One utterance per FFT-size family, so every call runs several family
    # kernels side by side; eager and graph calls on the null stream and on a
    # side stream, interleaved, must all give the same bits.
    torch = cuda()
    from paper_1712_03439_amd import rsim

    rng = synth.rng_for(13, 0)
    sizes = [9, 11, 12, 13, 14, 15, 14, 13]
    srcs, rirs = [], []
    for l2 in sizes:
        n = int(rng.integers(2000, 40000))
        srcs.append([synth.speech_like(rng, n), synth.white_noise(rng, n)])
        L0 = int(rng.integers(20, min(2 ** l2 // 2, 5000)))
        rirs.append([[synth.rir(rng, L0, 0.3, 10) for _ in range(2)] for _ in range(2)])
    b = synth.pack(srcs, rirs, [[0.0, 6.0]] * len(sizes), 2)
    db = rsim.DeviceBatch(b, fft_log2n=np.asarray(sizes, np.int32))
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    rsim.truncate_batch(db, 20.0)
    side = torch.cuda.Stream()
    outs = []
    for k, (graph, on_side) in enumerate([(False, False), (True, False), (True, True), (False, True),
                                           (True, False), (False, False)]):
        y = torch.full((max(db.y_len, 1),), float("nan"), device="cuda")
        if on_side:
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                rsim.mix(db, alpha, y=y, use_graph=graph)
            torch.cuda.current_stream().wait_stream(side)
        else:
            rsim.mix(db, alpha, y=y, use_graph=graph)
        torch.cuda.synchronize()
        outs.append(y.cpu().numpy())
    rl, ol = db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()
    _check_utterances(b, range(b.n_utt), 20.0, outs[0], rl, ol)
    for u in range(b.n_utt):
        off, st, T = int(b.out_off[u]), int(b.out_stride[u]), int(ol[u])
        for j in range(b.n_mic):
            ref = outs[0][off + j * st: off + j * st + T]
            for k in range(1, len(outs)):
                assert np.array_equal(outs[k][off + j * st: off + j * st + T], ref), (k, u, j)
    # the descriptor states the forced sizes (binding default): launching
    # every family instead gives the same bits; a size left out of the stated
    # set skips its utterance with BADPLAN and leaves the others as they were
    assert db.fft_sizes == sum(1 << m for m in set(sizes))
    rsim.device_status()
    for bits, skip in ((0, None), (db.fft_sizes & ~(1 << 15), sizes.index(15))):
        db.fft_sizes = bits
        y = torch.full((max(db.y_len, 1),), float("nan"), device="cuda")
        rsim.mix(db, alpha, y=y)
        torch.cuda.synchronize()
        y = y.cpu().numpy()
        assert bool(rsim.device_status() & rsim.DEV_BADPLAN) == (skip is not None)
        ol2 = db.out_len.cpu().numpy()
        for u in range(b.n_utt):
            off, st, T = int(b.out_off[u]), int(b.out_stride[u]), int(ol[u])
            if u == skip:
                assert ol2[u] == 0 and np.all(np.isnan(y[off: off + b.n_mic * st]))
                continue
            for j in range(b.n_mic):
                assert np.array_equal(y[off + j * st: off + j * st + T], outs[0][off + j * st: off + j * st + T]), (bits, u, j)


@pytest.mark.gpu
def test_one_fft_size_for_the_batch():
    # one N for every utterance (the smallest summed cost), eager and as a graph
    torch = cuda()
    from paper_1712_03439_amd import autotune, rsim

    b = synth.make_config2(n_utt=24, epoch=5)
    f, m = autotune.model_costs()
    tune = rsim.tune_table(f, m, one_size=True)
    for graph in (False, True):
        db, alpha, y, rl, ol = _simulate(b, 20.0, tune=tune, use_graph=graph)
        _check_utterances(b, range(b.n_utt), 20.0, y, rl, ol)


def _large_subset(n_utt, eta_seed):
    # the large workload's shapes: 1-20 s, up to 4 sources, 8 mics, T60 up to
    # 1.0 s (L0 = ceil(T60 fs) <= 16000); utterance 0 is the extreme case
    # (20 s, 4 sources, 16000-tap RIRs)
    rng = synth.rng_for(4, 500 + eta_seed)
    srcs, rirs, snrs = [], [], []
    for u in range(n_utt):
        n = 20 * synth.FS if u == 0 else int(rng.uniform(1.0, 20.0) * synth.FS)
        I = 4 if u == 0 else int(1 + rng.integers(0, 4))
        t60 = 1.0 if u == 0 else float(rng.uniform(0.1, 1.0))
        L0 = min(int(math.ceil(t60 * synth.FS)), 16000)
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(I - 1)])
        rirs.append([[synth.rir(rng, L0, t60, int(rng.integers(20, 401))) for _ in range(8)] for _ in range(I)])
        snrs.append([0.0] + [float(v) for v in rng.uniform(0, 30, I - 1)])
    return synth.pack(srcs, rirs, snrs, 8)


@pytest.mark.gpu
@pytest.mark.parametrize("eta", [math.inf, 30.0, 20.0, 10.0])
def test_large_workload_subset_full(eta):
    # twelve utterances of the large workload, every output sample of every
    # mic against the oracle, including the extreme one (20 s, 4 sources,
    # 8 mics, 16000-tap RIRs)
    b = _large_subset(12, int(eta) if math.isfinite(eta) else 99)
    db, alpha, y, rl, ol = _simulate(b, eta)
    worst = _check_utterances(b, range(b.n_utt), eta, y, rl, ol)
    print(f"large workload eta={eta}: max error {worst:.2e} of the peak")


@pytest.mark.gpu
def test_large_workload_sizes_per_utterance():
    # the large workload without a cut takes a size per utterance (16384 for
    # the shorter RIRs, 32768 for the longest): several kernel families in one
    # graph, and concurrently on the side streams eagerly; both give the same
    # bits, checked in full against the oracle
    from paper_1712_03439_amd import autotune, rsim

    b = _large_subset(16, 77)
    f, m = autotune.model_costs()
    tune = rsim.tune_table(f, m, one_size=False)
    db, alpha, y, rl, ol = _simulate(b, math.inf, tune=tune, use_graph=True)
    _, _, y_eager, rl_e, ol_e = _simulate(b, math.inf, tune=tune, use_graph=False)
    assert np.array_equal(rl, rl_e) and np.array_equal(ol, ol_e)
    L = rl.reshape(b.n_utt, -1).max(axis=1)
    shapes = [(int(b.src_len[u]), int(b.n_src[u]), b.n_mic, int(L[u])) for u in range(b.n_utt)]
    sizes = {autotune.utterance_log2n(*sh, f, m) for sh in shapes}
    assert len(sizes) >= 2, sizes
    for u in range(b.n_utt):
        off, st, T = int(b.out_off[u]), int(b.out_stride[u]), int(ol[u])
        for j in range(b.n_mic):
            assert np.array_equal(y[off + j * st: off + j * st + T], y_eager[off + j * st: off + j * st + T]), (u, j)
    _check_utterances(b, range(b.n_utt), math.inf, y, rl, ol)


@pytest.mark.gpu
def test_batched_workload_full_size():
    # the whole 2048-utterance epoch in the benchmark's launch configuration:
    # LPT order, the tuner's table measured on the cut batch (FFT size and
    # kernel variants), one graph for cut + mix; 64 utterances (the longest,
    # the most sources, the longest RIR, every 33rd) compared in full, every
    # cut length bit-exact
    torch = cuda()
    from paper_1712_03439_amd import autotune, rsim

    b = synth.make_config2(epoch=2)
    order = np.argsort(-(b.src_len.astype(np.int64) * (b.n_src + b.n_mic)), kind="stable").astype(np.int32)
    db = rsim.DeviceBatch(b, order=order)
    alpha_t = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        rsim.truncate_batch(db, 20.0, stream=stream)
    stream.synchronize()
    tune, _ = autotune.tune(db, alpha_t, stream=stream, reps=1)
    with torch.cuda.stream(stream):
        y = rsim.simulate(db, alpha_t, 20.0, tune=tune, use_graph=True, stream=stream)
    torch.cuda.synchronize()
    y, rl, ol = y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()
    longest = int(np.argmax(b.src_len))
    most_src = int(np.argmax(b.n_src))
    longest_rir = int(np.argmax(b.rir_len0)) // (b.max_src * b.n_mic)
    utts = sorted({0, longest, most_src, longest_rir} | set(range(1, b.n_utt, 33)))
    assert len(utts) >= 64
    _check_utterances(b, utts, 20.0, y, rl, ol)
    for r in range(len(b.rir_len0)):
        h = b.h[b.rir_off[r]: b.rir_off[r] + b.rir_len0[r]]
        assert int(rl[r]) == oracle.cut_rir(h, 20.0)[1], r


@pytest.mark.gpu
@pytest.mark.parametrize("l2", [11, 13, 14, 15])
def test_single_source_many_mics(l2):
    # one source and several mic groups: every later group reuses the one
    # source spectrum of the block
    rng = synth.rng_for(14, l2)
    srcs, rirs = [], []
    for u in range(3):
        n = int(rng.integers(3000, 40000))
        srcs.append([synth.speech_like(rng, n)])
        L0 = int(rng.integers(50, min(2 ** l2 // 2, 5000)))
        rirs.append([[synth.rir(rng, L0, 0.3, 10) for _ in range(6)]])
    b = synth.pack(srcs, rirs, [[0.0]] * 3, 6)
    db, alpha, y, rl, ol = _simulate(b, math.inf, fft_log2n=np.full(3, l2, np.int32))
    _check_utterances(b, range(3), math.inf, y, rl, ol)


@pytest.mark.gpu
def test_many_utterances_several_mic_groups():
    # more utterances than compute units with 5 mics: one work item per
    # utterance, the source spectra cached for the later mic groups (one and
    # several sources); with few utterances each mic group is its own item
    rng = synth.rng_for(15, 0)
    srcs, rirs = [], []
    for u in range(300):
        I = 1 + u % 3
        n = int(rng.integers(1000, 5000))
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(I - 1)])
        L0 = int(rng.integers(30, 900))
        rirs.append([[synth.rir(rng, L0, 0.2, int(rng.integers(0, 30))) for _ in range(5)] for _ in range(I)])
    b = synth.pack(srcs, rirs, [[0.0] + [3.0] * (len(s) - 1) for s in srcs], 5)
    db, alpha, y, rl, ol = _simulate(b, 20.0)
    _check_utterances(b, (0, 1, 2, 150, 299), 20.0, y, rl, ol)
    small = synth.subset(b, [0, 1, 2, 3])
    db, alpha, y, rl, ol = _simulate(small, 20.0)
    _check_utterances(small, range(4), 20.0, y, rl, ol)


@pytest.mark.gpu
def test_differentiation_workload_forward():
    # 64 utterances of 4 s, 3 sources, 4 mics, 8192-tap RIRs, no cut, N = 16384:
    # fewer utterances than compute units, so each mic pair is its own work item
    b = synth.make_config3()
    db, alpha, y, rl, ol = _simulate(b, math.inf, fft_log2n=np.full(b.n_utt, 14, np.int32))
    _check_utterances(b, range(0, 64, 7), math.inf, y, rl, ol)


@pytest.mark.gpu
def test_one_utterance_of_2_to_the_24_samples_in_full():
    # about 17.5 minutes of audio in one utterance (2^24 + 12345 samples, two
    # sources, three mics, RIRs of up to 3000 taps): its blocks split over
    # many workgroups, every output sample against the oracle
    rng = synth.rng_for(17, 24)
    n = (1 << 24) + 12345
    srcs = [[synth.speech_like(rng, n), synth.white_noise(rng, n)]]
    rirs = [[[synth.rir(rng, int(rng.integers(1000, 3001)), 0.5, int(rng.integers(0, 100))) for _ in range(3)]
             for _ in range(2)]]
    b = synth.pack(srcs, rirs, [[0.0, 6.0]], 3)
    db, alpha, y, rl, ol = _simulate(b, 20.0)
    assert int(ol[0]) > (1 << 24)
    _check_utterances(b, [0], 20.0, y, rl, ol)


@pytest.mark.gpu
def test_calls_from_several_host_threads():
    # four host threads, each with its own batch and stream, call the library
    # at once, five times each; every batch mixes two FFT-size families, so
    # each eager call forks its family kernels onto the library's shared side
    # streams.  Every call gives the bits of the same call made alone.
    import threading

    torch = cuda()
    from paper_1712_03439_amd import rsim

    jobs = []
    for k in range(4):
        b = synth.make_config2(n_utt=12 + 5 * k, epoch=40 + k)
        l2 = np.where(np.arange(b.n_utt) % 2 == 0, 13, 14).astype(np.int32)
        db = rsim.DeviceBatch(b, fft_log2n=l2)
        alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
        y = torch.zeros(max(db.y_len, 1), device="cuda")
        rsim.simulate(db, alpha, 20.0, y=y)
        torch.cuda.synchronize()
        jobs.append((db, alpha, y.cpu().numpy()))
    errors = []

    def work(k):
        db, alpha, ref = jobs[k]
        s = torch.cuda.Stream()
        try:
            for _ in range(5):
                with torch.cuda.stream(s):
                    y = torch.zeros(max(db.y_len, 1), device="cuda")
                    rsim.simulate(db, alpha, 20.0, y=y, stream=s)
                s.synchronize()
                if not np.array_equal(y.cpu().numpy().view(np.uint32), ref.view(np.uint32)):
                    errors.append(k)
        except Exception as e:  # reported below
            errors.append((k, repr(e)))

    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    assert rsim.device_status() == 0
