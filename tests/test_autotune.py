"""The tuner's fit (host logic, no GPU): from timed sizes and kernel variants to
the cost table that the schedule's size rule (eq. 6 and the paragraph after
it) evaluates."""
import numpy as np

from paper_1712_03439_amd import autotune

MF, MM = autotune.model_costs()


def _shapes(seed, n=200, lmax_hi=5000):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(16000, 240000)), int(rng.integers(1, 5)), 2, int(rng.integers(300, lmax_hi)))
            for _ in range(n)]


def _model_sum(shapes, m):
    cs = [autotune.utt_cost(nx, I, J, L, m, MF, MM) for nx, I, J, L in shapes]
    return None if any(c is None for c in cs) else float(sum(cs))


def _measured(shapes, k_true, penalty):
    """Times of a fictitious GPU: size m runs k_true[m] ms per 1e6 model units
    with the best variant; variant v costs penalty[v] times that."""
    sizes = {}
    for m, k in k_true.items():
        ms = _model_sum(shapes, m)
        if ms is None:
            continue
        vs = autotune.VARIANTS[autotune.FAMILY[m]]
        sizes[m] = {"utterances": len(shapes), "model": ms, "ms": {v: k * ms / 1e6 * penalty[v] for v in vs}}
    return {"sizes": sizes}


def test_fit_picks_the_size_that_ran_fastest():
    shapes = _shapes(1)
    # the built-in model prefers 16384 for this batch; the fictitious GPU runs
    # 8192 well and 16384 badly, so the measured optimum moves
    assert autotune.batch_log2n(shapes, MF, MM) == 14
    k_true = {13: 1.0, 14: 1.6, 15: 1.3}
    entry = autotune.fit(_measured(shapes, k_true, {1: 1.0, 2: 1.0, 3: 1.0, 4: 1.0}))
    t = {m: k_true[m] * _model_sum(shapes, m) for m in k_true}
    assert autotune.batch_log2n(shapes, entry["cost_fft"], entry["cost_mac"]) == min(t, key=t.get)
    # the fitted summed cost reproduces each measured time (ns)
    for m in k_true:
        s = sum(autotune.utt_cost(nx, I, J, L, m, entry["cost_fft"], entry["cost_mac"]) for nx, I, J, L in shapes)
        assert abs(s / 1e6 - t[m] / 1e6) <= 1e-9 * t[m]


def test_fit_variant_choice_and_default_on_ties():
    shapes = _shapes(2)
    k_true = {13: 1.0, 14: 1.0, 15: 1.0}
    e = autotune.fit(_measured(shapes, k_true, {1: 1.2, 2: 1.1, 3: 0.9, 4: 1.3}))
    assert e["variant"][3] == 3 and e["variant"][4] == 3  # 8192 and 16384 families
    assert e["variant"][5] == 4                            # 32768 has one variant
    assert e["variant"][0] == 0 and e["variant"][1] == 0   # not measured: default
    e = autotune.fit(_measured(shapes, k_true, {1: 1.0, 2: 1.0, 3: 1.0, 4: 1.0}))
    assert e["variant"][3] == autotune.DEFAULT_VARIANT
    # within the timing noise the default stays
    e = autotune.fit(_measured(shapes, k_true, {1: 1.2, 2: 1.01, 3: 1.0, 4: 1.3}))
    assert e["variant"][4] == autotune.DEFAULT_VARIANT
    e = autotune.fit(_measured(shapes, k_true, {1: 1.2, 2: 1.05, 3: 1.0, 4: 1.3}))
    assert e["variant"][4] == 3
    # the chosen variant's time sets the size's scale
    e = autotune.fit(_measured(shapes, {14: 2.0}, {1: 1.5, 2: 1.0, 3: 3.0, 4: 3.0}))
    k = e["cost_fft"][14 - 9] / MF[14 - 9]
    assert abs(k - 2.0) < 1e-9


def test_fit_family_with_two_sizes_scores_relative_times():
    # 1024 and 2048 share a kernel family: a variant 5% worse at both beats one
    # 20% better at one and 50% worse at the other
    shapes = [(64000, 2, 2, 200)] * 50
    meas = {"sizes": {}}
    for m, pen in ((10, {1: 1.05, 2: 1.0, 3: 0.8, 4: 2.0}), (11, {1: 1.05, 2: 1.5, 3: 1.6, 4: 2.0})):
        ms = _model_sum(shapes, m)
        meas["sizes"][m] = {"utterances": 50, "model": ms, "ms": {v: p * ms / 1e6 for v, p in pen.items()}}
    e = autotune.fit(meas)
    assert e["variant"][1] == 1


def test_unmeasured_sizes_take_the_nearest_scale():
    shapes = _shapes(3, lmax_hi=1500)
    meas = _measured(shapes, {12: 3.0, 14: 1.0}, {1: 1.0, 2: 1.0, 3: 1.0, 4: 1.0})
    e = autotune.fit(meas)
    k = [e["cost_fft"][m - 9] / MF[m - 9] for m in range(9, 16)]
    assert np.allclose(k, [3.0, 3.0, 3.0, 3.0, 1.0, 1.0, 1.0])  # 13: tie between 12 and 14 -> 14
    assert np.allclose([e["cost_mac"][m - 9] / MM[m - 9] for m in range(9, 16)], k)


def test_fit_round_trips_through_its_stored_form():
    shapes = _shapes(4)
    e = autotune.fit(_measured(shapes, {13: 1.2, 14: 1.0, 15: 1.1}, {1: 1.1, 2: 1.0, 3: 1.05, 4: 1.2}))
    e2 = autotune.fit(e["measured"])
    assert e2["variant"] == e["variant"]
    assert np.allclose(e2["cost_fft"], e["cost_fft"]) and np.allclose(e2["cost_mac"], e["cost_mac"])
    t = autotune.entry_to_tune(e)
    assert list(t.variant) == e["variant"] and t.one_size == 1
    assert np.allclose(list(t.cost_fft), e["cost_fft"], rtol=1e-6)


def test_sub_batch_rows_and_order():
    # DeviceBatch.select on host tensors: descriptor rows of the chosen
    # utterances, the parent's order restricted to them
    import synth
    from paper_1712_03439_amd import rsim

    b = synth.make_config2(n_utt=12, epoch=2)
    order = np.array([5, 3, 11, 0, 1, 2, 4, 6, 7, 8, 9, 10], np.int32)
    db = rsim.DeviceBatch(b, device="cpu", order=order)
    idx = [0, 3, 4, 11]
    sub = db.select(idx)
    S, J = b.max_src, b.n_mic
    assert sub.U == 4 and sub.x is db.x and sub.y_len == db.y_len
    assert np.array_equal(sub.n_src.numpy(), b.n_src[idx])
    assert np.array_equal(sub.out_off.numpy(), b.out_off[idx])
    rows = [(u * S + i) * J + j for u in idx for i in range(S) for j in range(J)]
    assert np.array_equal(sub.rir_off.numpy(), b.rir_off[rows])
    assert np.array_equal(sub.rir_len.numpy(), db.rir_len.numpy()[rows])
    assert np.array_equal(sub.src_off.numpy(), b.src_off.reshape(-1)[[u * S + i for u in idx for i in range(S)]])
    # parent order 5, 3, 11, 0, ...: of idx, 3 comes first, then 11, 0, 4
    assert [idx[k] for k in sub.order.numpy()] == [3, 11, 0, 4]
    assert sub.max_rir_len0 == int(b.rir_len0[rows].max())


def test_policy_keeps_one_size_within_the_noise():
    assert autotune.choose_policy(10.0, 10.0) is True
    assert autotune.choose_policy(10.0, 9.9) is True     # 1 % faster: noise
    assert autotune.choose_policy(10.0, 9.5) is False    # 5 % faster: per utterance
    assert autotune.choose_policy(10.0, 11.0) is True


def test_pruning_keeps_the_batch_size_and_every_larger_one():
    f, c = autotune.model_costs()
    shapes = [(16000 * 3, 2, 2, 3000), (16000 * 9, 3, 2, 5000), (16000, 1, 2, 700)]
    entry = {"cost_fft": list(f), "cost_mac": list(c), "one_size": True}
    m = autotune.batch_log2n(shapes, f, c)
    assert m > 9
    assert autotune.keep_sizes_from_batch_size(entry, shapes) == m
    assert entry["sizes_from"] == m
    for k in autotune.LOG2N:
        assert (entry["cost_fft"][k - 9] > 0) == (k >= m) and (entry["cost_mac"][k - 9] > 0) == (k >= m)
    # the pruned table picks the same size, and every utterance still has one
    assert autotune.batch_log2n(shapes, entry["cost_fft"], entry["cost_mac"]) == m
    for nx, I, J, L in shapes + [(50, 1, 2, 20)]:
        assert autotune.utterance_log2n(nx, I, J, L, entry["cost_fft"], entry["cost_mac"]) >= m
    # a size per utterance keeps every size
    e2 = {"cost_fft": list(f), "cost_mac": list(c), "one_size": False}
    assert autotune.keep_sizes_from_batch_size(e2, shapes) == 0 and e2["cost_fft"] == list(f)
