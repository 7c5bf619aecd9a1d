"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: the convolution is checked against
a brute-force double loop, the cut against eq. (8) evaluated literally over
every m, the gains against the SNR they must reproduce, and the adjoint
against the dot-product identity and central finite differences.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import rsim_oracle as O


def _rng(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- convolution

def brute_conv(x, h):
    """Eq. (2)'s h * x by the textbook double loop over (n, k)."""
    nx, L = len(x), len(h)
    y = [0.0] * (nx + L - 1)
    for n in range(nx):
        for k in range(L):
            y[n + k] += float(h[k]) * float(x[n])
    return np.array(y)


@pytest.mark.parametrize("seed", range(6))
def test_convolve_matches_double_loop(seed):
    r = _rng(seed)
    nx = int(r.integers(1, 65))
    L = int(r.integers(1, 17))
    x = r.standard_normal(nx).astype(np.float32)
    h = r.standard_normal(L).astype(np.float32)
    got = oracle.convolve(x, h)
    ref = brute_conv(x, h)
    assert got.shape == (nx + L - 1,)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_convolve_is_not_correlation():
    # An asymmetric RIR distinguishes h * x from the correlation of h and x.
    x = np.array([1.0, 0.0, 0.0, 0.0], np.float32)
    h = np.array([1.0, 2.0, 3.0], np.float32)
    np.testing.assert_array_equal(oracle.convolve(x, h), [1, 2, 3, 0, 0, 0])


@pytest.mark.parametrize("d", [0, 1, 7, 40])
def test_delta_rir_delays_exactly(d):
    x = _rng(d).standard_normal(300).astype(np.float32)
    h = np.zeros(d + 5, np.float32)
    h[d] = 1.0
    y = oracle.convolve(x, h)
    assert y.size == 300 + d + 5 - 1
    np.testing.assert_array_equal(y[d:d + 300], x.astype(np.float64))
    assert not np.any(y[:d]) and not np.any(y[d + 300:])


def test_output_length_of_tiny_config():
    # 1 s at 16 kHz and a 4096-tap RIR give Nx + M - 1 = 20095 samples.
    x = np.ones(16000, np.float32)
    h = np.zeros(4096, np.float32)
    h[40] = 1.0
    assert oracle.convolve(x, h).size == 20095
    y = oracle.mix([x], [[h]], np.ones((1, 1)))
    assert y.shape == (1, 20095)


def test_mix_linearity():
    r = _rng(11)
    I, J, nx = 3, 2, 200
    xs = [r.standard_normal(nx) for _ in range(I)]
    xs2 = [r.standard_normal(nx) for _ in range(I)]
    hs = [[r.standard_normal(int(r.integers(5, 40))) for _ in range(J)] for _ in range(I)]
    hs2 = [[r.standard_normal(len(hs[i][j])) for j in range(J)] for i in range(I)]
    a = r.uniform(0.1, 2.0, (I, J))
    a2 = r.uniform(0.1, 2.0, (I, J))
    c1, c2 = 0.7, -1.3
    # linear in x
    lhs = O.mix([c1 * p + c2 * q for p, q in zip(xs, xs2)], hs, a)
    rhs = c1 * O.mix(xs, hs, a) + c2 * O.mix(xs2, hs, a)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    # linear in h
    hmix = [[c1 * hs[i][j] + c2 * hs2[i][j] for j in range(J)] for i in range(I)]
    np.testing.assert_allclose(O.mix(xs, hmix, a), c1 * O.mix(xs, hs, a) + c2 * O.mix(xs, hs2, a),
                               atol=1e-12)
    # linear in alpha
    np.testing.assert_allclose(O.mix(xs, hs, c1 * a + c2 * a2),
                               c1 * O.mix(xs, hs, a) + c2 * O.mix(xs, hs, a2), atol=1e-12)


def test_mix_sums_sources_per_mic_and_pads():
    # Two sources, two mics, different RIR lengths: every mic has length
    # Nx + max L - 1 and mic j sees only its own RIRs h_ij.
    x0 = np.array([1.0, 2.0], np.float32)
    x1 = np.array([0.5, -1.0], np.float32)
    h = [[np.array([1.0], np.float32), np.array([0.0, 1.0], np.float32)],
         [np.array([2.0, 0.0, 1.0], np.float32), np.array([1.0], np.float32)]]
    a = np.array([[1.0, 1.0], [3.0, 0.5]])
    y = O.mix([x0, x1], h, a)
    assert y.shape == (2, 4)
    # mic 0: x0 * [1] + 3 * (x1 * [2, 0, 1])
    np.testing.assert_allclose(y[0], [1 + 3 * 1.0, 2 + 3 * -2.0, 3 * 0.5, 3 * -1.0])
    # mic 1: x0 * [0, 1] + 0.5 * (x1 * [1])
    np.testing.assert_allclose(y[1], [0.25, 1 - 0.5, 2, 0])


def test_mix_at_matches_mix():
    r = _rng(5)
    I, J, nx = 2, 3, 123
    xs = [r.standard_normal(nx) for _ in range(I)]
    hs = [[r.standard_normal(int(r.integers(1, 30))) for _ in range(J)] for _ in range(I)]
    a = r.uniform(0.1, 2, (I, J))
    y = O.mix(xs, hs, a)
    idx = [0, 1, 50, y.shape[1] - 2, y.shape[1] - 1]
    for j in range(J):
        np.testing.assert_allclose(O.mix_at(xs, hs, a, j, idx), y[j, idx], atol=1e-12)


# ----------------------------------------------------------------- RIR cut-off

def brute_cut(h, eta):
    """Eq. (8) read literally: the smallest m with max_{n>m} h^2[n] < p_th
    (the max over an empty set counts as below), in float32."""
    h = np.asarray(h, np.float32)
    q = [np.float32(v * v) for v in h]
    P = max(q)
    s = np.float32(0.0) if math.isinf(eta) else np.float32(10.0 ** (-eta / 10.0))
    p_th = np.float32(P * s)
    for m in range(len(h)):
        tail = q[m + 1:]
        if not tail or max(tail) < p_th:
            return m, min(m + 2, len(h))
    raise AssertionError("unreachable")


@pytest.mark.parametrize("seed", range(20))
@pytest.mark.parametrize("eta", [0.0, 5.0, 10.0, 20.0, 30.0, math.inf])
def test_cut_matches_eq8_brute_force(seed, eta):
    r = _rng(seed)
    L0 = int(r.integers(1, 60))
    h = (r.standard_normal(L0) * np.exp(-np.arange(L0) / r.uniform(2, 20))).astype(np.float32)
    n_c, L, flag = oracle.cut_rir(h, eta)
    assert (n_c, L) == brute_cut(h, eta)
    assert not flag


@pytest.mark.parametrize("d", [0, 3, 17])
def test_cut_single_spike(d):
    h = np.zeros(40, np.float32)
    h[d] = 0.8
    assert oracle.cut_rir(h, 20.0)[:2] == (d, d + 2)


def test_cut_no_cut_and_zero_and_last_tap():
    h = np.linspace(1, 0, 25).astype(np.float32)
    assert oracle.cut_rir(h, math.inf)[:2] == (24, 25)        # eta = inf keeps all
    assert oracle.cut_rir(np.zeros(9, np.float32), 20.0)[:2] == (8, 9)  # P = 0 keeps all
    g = np.zeros(12, np.float32)
    g[-1] = 2.0
    assert oracle.cut_rir(g, 10.0)[:2] == (11, 12)            # peak at the last tap
    assert oracle.cut_rir(np.zeros(0, np.float32), 20.0) == (-1, 0, False)


def test_cut_eta_zero_keeps_through_last_peak():
    h = np.array([0.1, -0.5, 0.2, 0.5, 0.3, 0.1], np.float32)
    # p_th = P: the last sample with h^2 == P is index 3.
    assert oracle.cut_rir(h, 0.0)[:2] == (3, 5)


def test_cut_threshold_equality_is_kept():
    # eta = 10 log10(4) gives s = fl32(0.25) = 0.25 exactly, P = 1 -> p_th = 0.25,
    # and h = 0.5 gives q = 0.25 == p_th exactly: eq. (8)'s strict '<' keeps it.
    eta = 10.0 * math.log10(4.0)
    assert float(oracle.cut_scale(eta)) == 0.25
    h = np.array([1.0, 0.1, 0.5, 0.1, 0.49], np.float32)
    assert oracle.cut_rir(h, eta)[:2] == (2, 4)


def test_cut_subnormal_power():
    # q values are subnormal float32 numbers; nothing may be flushed to zero.
    h = np.array([1e-20, 4e-21, 1e-25, 0.0], np.float32)
    q = h * h
    assert q[0] > 0 and q[0] < np.finfo(np.float32).tiny
    n_c, L, _ = oracle.cut_rir(h, 10.0)
    assert (n_c, L) == brute_cut(h, 10.0)
    assert n_c == 1                      # 1.6e-41 >= fl32(1e-40 * 0.1)


def test_cut_nonfinite_keeps_all_and_flags():
    h = np.array([0.5, np.nan, 0.1], np.float32)
    assert oracle.cut_rir(h, 20.0) == (2, 3, True)
    h = np.array([0.5, 3e19, 0.1], np.float32)  # h^2 overflows float32
    assert oracle.cut_rir(h, 20.0) == (2, 3, True)


def test_cut_scale_rejects_bad_eta():
    with pytest.raises(ValueError):
        oracle.cut_scale(-1.0)
    with pytest.raises(ValueError):
        oracle.cut_scale(float("nan"))


def test_cut_monotone_in_eta():
    r = _rng(3)
    h = (r.standard_normal(500) * np.exp(-np.arange(500) / 80)).astype(np.float32)
    Ls = [oracle.cut_rir(h, e)[1] for e in (0.0, 5.0, 10.0, 20.0, 30.0, 60.0, math.inf)]
    assert Ls == sorted(Ls) and Ls[-1] == 500


# ----------------------------------------------------------------------- gains

def test_snr_gains_reproduce_requested_snr():
    r = _rng(7)
    for _ in range(20):
        I = int(r.integers(1, 5))
        xs = [r.standard_normal(1000) * r.uniform(0.01, 3) for _ in range(I)]
        snr = [0.0] + list(r.uniform(0, 30, I - 1))
        p = [oracle.dry_power(x) for x in xs]
        a = oracle.snr_gains(p, snr, 2)
        assert np.all(a[0] == 1.0)
        for i in range(1, I):
            for j in range(2):
                scaled = a[i, j] * xs[i]
                got = 10 * math.log10(np.mean(xs[0] ** 2) / np.mean(scaled ** 2))
                assert abs(got - snr[i]) < 1e-9


def test_snr_gains_silent_noise():
    a = oracle.snr_gains([1.0, 0.0], [0.0, 10.0], 3)
    assert np.all(a[1] == 0.0) and np.all(a[0] == 1.0)


# -------------------------------------------------------------------- backward

def _random_problem(seed, I=3, J=4, nx=256, L=64):
    r = _rng(seed)
    xs = [r.standard_normal(nx) for _ in range(I)]
    hs = [[r.standard_normal(int(r.integers(L // 2, L + 1))) for _ in range(J)] for _ in range(I)]
    a = r.uniform(0.2, 1.5, (I, J))
    return r, xs, hs, a


def test_adjoint_dot_product_identities():
    r, xs, hs, a = _random_problem(1)
    y = O.mix(xs, hs, a)
    g = r.standard_normal(y.shape)
    dx, dh, da = O.mix_backward(xs, hs, a, g)
    lhs = float(np.sum(y * g))
    # y is linear in x, in h and in alpha separately.
    assert abs(sum(float(np.dot(xs[i], dx[i])) for i in range(3)) - lhs) < 1e-9 * abs(lhs)
    assert abs(sum(float(np.dot(hs[i][j], dh[i][j])) for i in range(3) for j in range(4)) - lhs) \
        < 1e-9 * abs(lhs)
    assert abs(float(np.sum(a * da)) - lhs) < 1e-9 * abs(lhs)


def test_gradients_match_central_differences():
    # Loss = sum_j sum_n w_j[n] y_j[n]^2 (256-sample sources, 64-tap RIRs, I=3, J=4).
    r, xs, hs, a = _random_problem(2)
    T = O.mix(xs, hs, a).shape[1]
    w = r.uniform(0, 1, (4, T))

    def loss(xs_, hs_, a_):
        y = O.mix(xs_, hs_, a_)
        return float(np.sum(w * y * y))

    y = O.mix(xs, hs, a)
    dx, dh, da = O.mix_backward(xs, hs, a, 2.0 * w * y)
    # The loss is quadratic in each argument, so a central difference is exact
    # up to rounding for any step; a step of 1e-3 keeps cancellation small.
    eps = 1e-3
    for (i, n) in [(0, 0), (1, 100), (2, 255)]:
        xp = [v.copy() for v in xs]
        xm = [v.copy() for v in xs]
        xp[i][n] += eps
        xm[i][n] -= eps
        fd = (loss(xp, hs, a) - loss(xm, hs, a)) / (2 * eps)
        assert abs(fd - dx[i][n]) <= 1e-6 * max(1.0, abs(fd))
    for (i, j, k) in [(0, 0, 0), (1, 3, 10), (2, 2, len(hs[2][2]) - 1)]:
        hp = [[v.copy() for v in row] for row in hs]
        hm = [[v.copy() for v in row] for row in hs]
        hp[i][j][k] += eps
        hm[i][j][k] -= eps
        fd = (loss(xs, hp, a) - loss(xs, hm, a)) / (2 * eps)
        assert abs(fd - dh[i][j][k]) <= 1e-6 * max(1.0, abs(fd))
    for (i, j) in [(0, 0), (2, 3)]:
        ap = a.copy()
        am = a.copy()
        ap[i, j] += eps
        am[i, j] -= eps
        fd = (loss(xs, hs, ap) - loss(xs, hs, am)) / (2 * eps)
        assert abs(fd - da[i, j]) <= 1e-6 * max(1.0, abs(fd))


def test_simulate_cuts_then_mixes():
    r = _rng(9)
    x = [r.standard_normal(50)]
    h = np.zeros(30, np.float32)
    h[2] = 1.0
    h[20] = 0.05          # 26 dB below the peak: cut at 20 dB, kept at 30 dB
    y20, nc, L, _ = O.simulate(x, [[h]], [0.0], 20.0)
    assert L[0][0] == 4 and y20.shape == (1, 53)
    y30, nc, L, _ = O.simulate(x, [[h]], [0.0], 30.0)
    assert L[0][0] == 22 and y30.shape == (1, 71)


def test_empty_rir_contributes_nothing():
    x = np.arange(5, dtype=np.float32)
    assert oracle.convolve(x, np.zeros(0, np.float32)).size == 0
    y = O.mix([x], [[np.zeros(0, np.float32), np.array([2.0], np.float32)]], np.ones((1, 2)))
    assert y.shape == (2, 5)
    assert not np.any(y[0]) and np.allclose(y[1], 2 * x)
    assert O.mix([x], [[np.zeros(0, np.float32)]], np.ones((1, 1))).shape == (1, 0)


def test_sampled_adjoint_agrees_with_central_differences():
    # mix_backward_at evaluates each gradient entry as its own direct sum; pin it
    # by central differences of the quadratic loss, like the full adjoint.
    r, xs, hs, a = _random_problem(4, I=2, J=3, nx=90, L=20)
    T = O.mix(xs, hs, a).shape[1]
    w = r.uniform(0, 1, (3, T))
    y = O.mix(xs, hs, a)
    g = 2.0 * w * y

    def loss(xs_, hs_, a_):
        yy = O.mix(xs_, hs_, a_)
        return float(np.sum(w * yy * yy))

    eps = 1e-3
    x_idx, h_idx = [0, 45, 89], [0, 7, len(hs[1][2]) - 1]
    dx, dh, da = O.mix_backward_at(xs, hs, a, g, 1, 2, x_idx, h_idx)
    for t, n in enumerate(x_idx):
        xp = [v.copy() for v in xs]
        xm = [v.copy() for v in xs]
        xp[1][n] += eps
        xm[1][n] -= eps
        fd = (loss(xp, hs, a) - loss(xm, hs, a)) / (2 * eps)
        assert abs(fd - dx[t]) <= 1e-6 * max(1.0, abs(fd))
    for t, k in enumerate(h_idx):
        hp = [[v.copy() for v in row] for row in hs]
        hm = [[v.copy() for v in row] for row in hs]
        hp[1][2][k] += eps
        hm[1][2][k] -= eps
        fd = (loss(xs, hp, a) - loss(xs, hm, a)) / (2 * eps)
        assert abs(fd - dh[t]) <= 1e-6 * max(1.0, abs(fd))
    ap, am = a.copy(), a.copy()
    ap[1, 2] += eps
    am[1, 2] -= eps
    fd = (loss(xs, hs, ap) - loss(xs, hs, am)) / (2 * eps)
    assert abs(fd - da) <= 1e-6 * max(1.0, abs(fd))
    # a tap index beyond the RIR has no gradient
    assert O.mix_backward_at(xs, hs, a, g, 1, 2, [], [len(hs[1][2]) + 3])[1][0] == 0.0


# --------------------------------------------------- reverberant-at-mic gains
def test_reverb_energy_of_a_scaled_delay():
    # h = a delta[n - d]: (h * x)[n] = a x[n - d], so E = a^2 sum x^2
    rng = np.random.default_rng(31)
    x = rng.standard_normal(3000).astype(np.float32)
    h = np.zeros(700, np.float32)
    h[321] = np.float32(0.375)
    e = oracle.reverb_energy(x, h)
    ref = 0.375 ** 2 * float(np.sum(x.astype(np.float64) ** 2))
    assert abs(e - ref) <= 1e-12 * ref


def test_reverb_energy_by_parseval_and_by_autocorrelation():
    # Parseval on a transform long enough for the whole convolution, and the
    # identity E = sum_l r_hh[l] r_xx[l] with both autocorrelations from
    # numpy.correlate: three routes to the same number
    rng = np.random.default_rng(32)
    for nx, L in ((1, 1), (50, 7), (4000, 900), (2500, 2600)):
        x = rng.standard_normal(nx)
        h = rng.standard_normal(L) * np.exp(-np.arange(L) / (L / 3 + 1))
        e = oracle.reverb_energy(x, h)
        n = 1 << int(np.ceil(np.log2(nx + L - 1)))
        pars = float(np.sum(np.abs(np.fft.fft(x, n) * np.fft.fft(h, n)) ** 2) / n)
        rxx = np.correlate(x, x, "full")[nx - 1:]
        rhh = np.correlate(h, h, "full")[L - 1:]
        m = min(L, nx)
        auto = float(rhh[0] * rxx[0] + 2.0 * np.dot(rhh[1:m], rxx[1:m]))
        assert abs(pars - e) <= 1e-9 * e and abs(auto - e) <= 1e-9 * e


def test_reverb_gains_give_the_snr_at_every_mic():
    rng = np.random.default_rng(33)
    E = rng.uniform(0.1, 50.0, (4, 3))
    snr = [0.0, 3.5, 12.0, 27.25]
    a = oracle.snr_gains_reverb(E, snr)
    assert np.all(a[0] == 1.0)
    for i in range(1, 4):
        for j in range(3):
            assert abs(10 * math.log10(E[0, j] / (a[i, j] ** 2 * E[i, j])) - snr[i]) <= 1e-9
    E[2, 1] = 0.0
    E[0, 2] = 0.0
    a = oracle.snr_gains_reverb(E, snr)
    assert a[2, 1] == 0.0 and np.all(a[1:, 2] == 0.0)
