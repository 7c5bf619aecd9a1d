"""The adjoint of eq. (2) on the GPU (rsim_mix_backward) against the FP64 oracle.

Bar: per gradient tensor of an utterance, max |gpu - ref| <= 1e-5 * max |ref|;
grad_h is zero beyond each cut length.  Every gradient entry is a sum of
products (a correlation, or for dalpha one long dot product), and float32
sums are accurate relative to the size of their terms, not of their result.
A tensor of few entries can cancel far below its terms (a one-sample source:
dx is one dot product of a gradient with a 2580-tap RIR, seen at 4e-4 of its
terms' root-sum-square); only when the bar above fails is the peak replaced
by that root-sum-square, the largest over the tensor's entries, when it is
the larger (float64 on the host, no GPU value involved)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import oracle_pool
from tests.gpu_util import TOL, cuda, max_rel_err


def _setup(b, eta, fft_log2n=None, hop=None):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    db = rsim.DeviceBatch(b, fft_log2n=fft_log2n, hop=hop)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    rsim.truncate_batch(db, eta)
    return db, alpha


def _oracle_problem(b, u, eta):
    xs = b.sources(u)
    hs = b.rirs(u)
    I, J = len(xs), b.n_mic
    cut = [[np.asarray(hs[i][j], np.float32)[: oracle.cut_rir(hs[i][j], eta)[1]] for j in range(J)]
           for i in range(I)]
    alpha = oracle.snr_gains([oracle.dry_power(x) for x in xs], b.snrs(u), J)
    T = oracle.out_length(len(xs[0]) if I else 0, [[len(c) for c in row] for row in cut])
    return xs, cut, alpha, T


def _grad_y(b, seed):
    """Seeded per-utterance output gradients, long enough for the uncut RIRs."""
    rng = synth.rng_for(50, seed)
    per = []
    for u in range(b.n_utt):
        xs = b.sources(u)
        if not xs:
            per.append(np.zeros((b.n_mic, 0)))
            continue
        T = len(xs[0]) + max(len(h) for row in b.rirs(u) for h in row) - 1
        gu = rng.standard_normal((b.n_mic, T)).astype(np.float32)
        per.append(gu)
    return per


def _pack_grad(b, per, T_of):
    g = np.zeros(max(b.y_len, 1), np.float32)
    out = []
    for u in range(b.n_utt):
        T = T_of[u]
        gu = per[u][:, :T]
        off, st = int(b.out_off[u]), int(b.out_stride[u])
        for j in range(b.n_mic):
            g[off + j * st: off + j * st + T] = gu[j]
        out.append(gu)
    return g, out


def _sq_corr(a, b, n_out):
    """sum_m a[m + k]^2 b[m]^2 for the lags k < n_out (float64): the sum of
    squares of the products that one correlation entry adds up."""
    from scipy.signal import fftconvolve

    a2 = np.asarray(a, np.float64) ** 2
    b2 = np.asarray(b, np.float64) ** 2
    if not a2.size or not b2.size or n_out <= 0:
        return np.zeros(max(n_out, 0))
    c = fftconvolve(a2, b2[::-1])[b2.size - 1: b2.size - 1 + n_out]
    return np.pad(np.maximum(c, 0.0), (0, n_out - c.size))


def _term_scales(x, cut, alpha, g):
    """Root-sum-square of the terms of the largest entry of dx_i, of dh_i
    (over its mics) and of each dalpha_ij: dx_i[n] sums a g_j[n + m] h_ij[m]
    over j and m, dh_ij[m] sums a g_j[n + m] x_i[n] over n, dalpha_ij sums
    g_j[n] (h_ij * x_i)[n] over n."""
    from scipy.signal import fftconvolve

    J = len(cut)
    sx = np.zeros(len(x))
    sh = 0.0
    sa = np.zeros(J)
    for j in range(J):
        a2 = float(alpha[j]) ** 2
        sx += a2 * _sq_corr(g[j], cut[j], len(x))
        if len(cut[j]):
            sh = max(sh, float(np.max(a2 * _sq_corr(g[j], x, len(cut[j])))))
            c = fftconvolve(np.asarray(x, np.float64), np.asarray(cut[j], np.float64))
            n = min(c.size, len(g[j]))
            sa[j] = math.sqrt(float(np.sum((np.asarray(g[j][:n], np.float64) * c[:n]) ** 2)))
    return (math.sqrt(float(np.max(sx))) if sx.size else 0.0), math.sqrt(sh), sa


def _err_over(err, peak, floor):
    return err / max(peak, floor, 1e-30)


def _check_full(b, eta, gx, gh, ga, gys, u):
    _check_full_many(b, eta, gx, gh, ga, gys, [u])


def _check_full_many(b, eta, gx, gh, ga, gys, utts):
    """Every entry of dx, dh and dalpha of the listed utterances against the
    oracle's adjoint, one (utterance, source) per worker process (the
    adjoint's terms of one source do not involve the others)."""
    cases = {u: _oracle_problem(b, u, eta) for u in utts}
    for u in utts:
        assert gys[u].shape[1] == cases[u][3]
    keys = [(u, i) for u in utts for i in range(len(cases[u][0]))]
    tasks = [(cases[u][0][i], cases[u][1][i], cases[u][2][i], gys[u]) for u, i in keys]
    refs = dict(zip(keys, oracle_pool.pmap(oracle_pool.backward_source, tasks)))
    worst = 0.0
    J, S = b.n_mic, b.max_src
    for u in utts:
        xs, cut, alpha, T = cases[u]
        I = len(xs)
        dx = [refs[(u, i)][0] for i in range(I)]
        dh = [refs[(u, i)][1] for i in range(I)]
        da = np.array([refs[(u, i)][2] for i in range(I)]).reshape(I, J)
        scales = {}

        def scale(i):  # computed only for a tensor that fails the bar of its peak
            if i not in scales:
                scales[i] = _term_scales(xs[i], cut[i], alpha[i], gys[u])
            return scales[i]

        for i in range(I):
            so, nx = int(b.src_off[u * S + i]), int(b.src_len[u])
            e = max_rel_err(gx[so: so + nx], dx[i])
            if e > TOL:
                err = float(np.max(np.abs(gx[so: so + nx] - dx[i])))
                e = _err_over(err, float(np.max(np.abs(dx[i]))), scale(i)[0])
            worst = max(worst, e)
            assert e <= TOL, ("dx", u, i, e)
        peak_h = max((float(np.max(np.abs(dh[i][j]))) for i in range(I) for j in range(J) if dh[i][j].size),
                     default=0.0)
        errs_h = []
        for i in range(I):
            for j in range(J):
                r = (u * S + i) * J + j
                ro, L0 = int(b.rir_off[r]), int(b.rir_len0[r])
                ref_h = np.zeros(L0)
                ref_h[: dh[i][j].size] = dh[i][j]
                errs_h.append((i, j, float(np.max(np.abs(gh[ro: ro + L0] - ref_h))) if L0 else 0.0))
        floor_h = 0.0
        if any(err > TOL * max(peak_h, 1e-30) for _, _, err in errs_h):
            floor_h = max(scale(i)[1] for i in range(I))
        for i, j, err in errs_h:
            e = _err_over(err, peak_h, floor_h)
            worst = max(worst, e)
            assert e <= TOL, ("dh", u, i, j, err, peak_h, floor_h)
        got_a = np.array([[ga[(u * S + i) * J + j] for j in range(J)] for i in range(I)])
        e = max_rel_err(got_a, da)
        if e > TOL:
            floor_a = max(float(np.max(scale(i)[2])) for i in range(I))
            e = _err_over(float(np.max(np.abs(got_a - da))), float(np.max(np.abs(da))), floor_a)
        worst = max(worst, e)
        assert e <= TOL, ("dalpha", u, e)
    return worst


def _run(b, eta, seed, fft_log2n=None, hop=None):
    torch = cuda()
    from paper_1712_03439_amd import rsim

    db, alpha = _setup(b, eta, fft_log2n, hop)
    rsim.mix(db, alpha)  # its schedule writes out_len
    torch.cuda.synchronize()
    T_of = db.out_len.cpu().numpy()
    per = _grad_y(b, seed)
    g, gys = _pack_grad(b, per, T_of)
    gx, gh, ga = rsim.mix_backward(db, alpha, torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    return gx.cpu().numpy(), gh.cpu().numpy(), ga.cpu().numpy(), gys


@pytest.mark.gpu
def test_fd_subcase_shapes():
    # 256-sample sources, 64-tap RIRs, I = 3, J = 4, N = 512 with hop 64: four
    # blocks, so the block split of both correlations is exercised.
    rng = synth.rng_for(3, 99)
    xs = [synth.speech_like(rng, 256), synth.white_noise(rng, 256), synth.pink_noise(rng, 256)]
    hs = [[synth.rir(rng, 64, 0.5, int(rng.integers(0, 20))) for _ in range(4)] for _ in range(3)]
    b = synth.pack([xs], [hs], [[0.0, 5.0, 15.0]], 4)
    gx, gh, ga, gys = _run(b, math.inf, 1, fft_log2n=np.array([9], np.int32), hop=np.array([64], np.int32))
    _check_full(b, math.inf, gx, gh, ga, gys, 0)


@pytest.mark.gpu
@pytest.mark.parametrize("l2", [9, 11, 12, 13, 14, 15])
def test_backward_ragged_batch(l2):
    rng = synth.rng_for(51, l2)
    srcs, rirs, snrs = [], [], []
    for u in range(3):
        I = 1 + u
        n = int(rng.integers(500, 12000))
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(I - 1)])
        L0 = int(rng.integers(10, min(2 ** l2 // 2, 3000)))
        rirs.append([[synth.rir(rng, L0, 0.3, int(rng.integers(0, 30))) for _ in range(3)] for _ in range(I)])
        snrs.append([0.0] + [float(v) for v in rng.uniform(0, 20, I - 1)])
    b = synth.pack(srcs, rirs, snrs, 3)
    gx, gh, ga, gys = _run(b, 20.0, l2, fft_log2n=np.full(3, l2, np.int32))
    _check_full_many(b, 20.0, gx, gh, ga, gys, range(b.n_utt))


@pytest.mark.gpu
def test_backward_cost_model_sizes_and_degenerate():
    rng = synth.rng_for(52, 0)
    z = np.zeros(0, np.float32)
    srcs = [[synth.speech_like(rng, 3000), synth.pink_noise(rng, 3000)],
            [synth.speech_like(rng, 1)],
            [synth.speech_like(rng, 800)],
            [synth.speech_like(rng, 20000), synth.white_noise(rng, 20000)]]
    rirs = [[[synth.rir(rng, 500, 0.2, 5), z], [synth.rir(rng, 300, 0.2, 9), synth.rir(rng, 900, 0.2, 2)]],
            [[synth.rir(rng, 40, 0.1, 1), synth.rir(rng, 3, 0.1, 0)]],
            [[z, z]],                                 # no tap at all: zero gradients
            [[synth.rir(rng, 5000, 0.4, 100)] * 2, [synth.rir(rng, 2500, 0.4, 50)] * 2]]
    b = synth.pack(srcs, rirs, [[0.0, 3.0], [0.0], [0.0], [0.0, 12.0]], 2)
    gx, gh, ga, gys = _run(b, 20.0, 7)
    _check_full_many(b, 20.0, gx, gh, ga, gys, (0, 1, 3))
    so = int(b.src_off[2 * b.max_src])
    assert not np.any(gx[so: so + 800])
    for j in range(2):
        r = (2 * b.max_src) * 2 + j
        assert ga[r] == 0.0


@pytest.mark.gpu
def test_differentiation_config_full():
    # 64 utterances of 4 s, I = 3, J = 4, 8192-tap RIRs, no cut, N = 16384
    # (hop 8193, 8 blocks): every entry of dx, dh and dalpha of three
    # utterances against the oracle's adjoint
    b = synth.make_config3()
    gx, gh, ga, gys = _run(b, math.inf, 3, fft_log2n=np.full(b.n_utt, 14, np.int32))
    worst = _check_full_many(b, math.inf, gx, gh, ga, gys, [0, 37, 63])
    print(f"differentiation workload: max gradient error {worst:.2e} of the peak")


@pytest.mark.gpu
def test_autograd_directional_derivative():
    # y is linear in x, in h and in alpha: for the loss <w, y> the directional
    # derivative along d equals (loss(p + d) - loss(p - d)) / 2 exactly up to
    # float32 rounding of the forward.
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=6, epoch=1)
    db, alpha = _setup(b, 20.0)
    x = db.x.clone().requires_grad_(True)
    h = db.h.clone().requires_grad_(True)
    a = alpha.clone().requires_grad_(True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    y = rsim.mix_autograd(db, x, h, a)
    w = torch.rand(y.shape, device="cuda", generator=gen)
    loss = torch.sum(w * y)
    loss.backward()
    for k, (p, g) in enumerate(((x, x.grad), (h, h.grad), (a, a.grad))):
        d = torch.randn(p.shape, device="cuda", generator=gen)
        with torch.no_grad():
            args_p = [t.detach() for t in (x, h, a)]
            args_m = [t.detach() for t in (x, h, a)]
            args_p[k] = args_p[k] + d
            args_m[k] = args_m[k] - d
            lp = torch.sum((w * rsim.mix_autograd(db, *args_p)).double())
            lm = torch.sum((w * rsim.mix_autograd(db, *args_m)).double())
            fd = float((lp - lm) / 2)
            an = float(torch.sum(g.double() * d.double()))
        assert abs(fd - an) <= 1e-3 * max(abs(an), 1e-6), (k, fd, an)


@pytest.mark.gpu
def test_backward_many_utterances_one_part_each():
    # more utterances than compute units: every utterance is one work item
    rng = synth.rng_for(53, 0)
    srcs, rirs, snrs = [], [], []
    for u in range(300):
        I = 1 + u % 3
        n = int(rng.integers(1500, 6000))
        srcs.append([synth.speech_like(rng, n)] + [synth.white_noise(rng, n) for _ in range(I - 1)])
        L0 = int(rng.integers(50, 1200))
        rirs.append([[synth.rir(rng, L0, 0.2, int(rng.integers(0, 40))) for _ in range(2)] for _ in range(I)])
        snrs.append([0.0] + [float(v) for v in rng.uniform(0, 20, I - 1)])
    b = synth.pack(srcs, rirs, snrs, 2)
    gx, gh, ga, gys = _run(b, 20.0, 11)
    _check_full_many(b, 20.0, gx, gh, ga, gys, (0, 1, 2, 149, 299))


@pytest.mark.gpu
def test_backward_split_with_two_sizes_of_one_family():
    # N = 1024 and 2048 run in one kernel family; with fewer utterances than
    # compute units each is split into parts, whose correlation and RIR
    # spectra live in per-family buffers laid out for the larger size
    rng = synth.rng_for(54, 0)
    srcs, rirs, snrs = [], [], []
    for u in range(4):
        I = 1 + u % 3
        n = int(rng.integers(3000, 9000))
        srcs.append([synth.speech_like(rng, n)] + [synth.pink_noise(rng, n) for _ in range(I - 1)])
        L0 = int(rng.integers(50, 400))
        rirs.append([[synth.rir(rng, L0, 0.2, int(rng.integers(0, 30))) for _ in range(2)] for _ in range(I)])
        snrs.append([0.0] + [float(v) for v in rng.uniform(0, 20, I - 1)])
    b = synth.pack(srcs, rirs, snrs, 2)
    gx, gh, ga, gys = _run(b, 20.0, 12, fft_log2n=np.array([10, 11, 10, 11], np.int32))
    _check_full_many(b, 20.0, gx, gh, ga, gys, range(b.n_utt))


@pytest.mark.gpu
def test_autograd_keeps_the_forward_cut_lengths():
    # a cut at another threshold between the forward and the backward (the
    # next epoch on the same descriptor) must not change this graph's adjoint
    torch = cuda()
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=5, epoch=4)
    db, alpha = _setup(b, 20.0)
    rl20 = db.rir_len.clone()
    x = db.x.clone().requires_grad_(True)
    h = db.h.clone().requires_grad_(True)
    y = rsim.mix_autograd(db, x, h, alpha)
    w = torch.rand(y.shape, device="cuda", generator=torch.Generator(device="cuda").manual_seed(9))
    rsim.truncate_batch(db, 10.0)
    assert not torch.equal(db.rir_len, rl20)
    torch.sum(w * y).backward()
    gy = (w * torch.ones_like(y)).contiguous()
    gx, gh, _ = rsim.mix_backward(db, alpha, gy, rir_len=rl20, out_len=torch.empty_like(db.out_len))
    torch.cuda.synchronize()
    assert torch.equal(x.grad, gx) and torch.equal(h.grad, gh)


@pytest.mark.gpu
def test_backward_one_utterance_of_2_to_the_22_samples():
    # about 4.4 minutes of audio in one utterance (2^22 + 777 samples, two
    # sources, two mics, RIRs of up to 2000 taps), split into parts: every
    # entry of dx, dh and dalpha against the oracle
    rng = synth.rng_for(55, 22)
    n = (1 << 22) + 777
    srcs = [[synth.speech_like(rng, n), synth.white_noise(rng, n)]]
    rirs = [[[synth.rir(rng, int(rng.integers(500, 2001)), 0.4, int(rng.integers(0, 60))) for _ in range(2)]
             for _ in range(2)]]
    b = synth.pack(srcs, rirs, [[0.0, 8.0]], 2)
    gx, gh, ga, gys = _run(b, 20.0, 22)
    _check_full_many(b, 20.0, gx, gh, ga, gys, [0])
