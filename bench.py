#!/usr/bin/env python3
"""Benchmark of the room-simulator hot path on one MI355X.

One step = one epoch of the batched workload: 2048 utterances of 1-15 s at
16 kHz, each with a target and 0-3 noise sources, 2 microphones, RIRs of
ceil(T60 fs) taps with T60 ~ U(0.1, 0.9) s drawn fresh for every epoch, cut at
eta = 20 dB below the peak power, SNRs ~ U(0, 30) dB.  A step runs the RIR
cut-off and the batched overlap-add filter-and-mix (one HIP graph, built
anew for the epoch).  Inputs (sources, that epoch's RIRs and gains) are resident
in HBM before the timed region starts.

Prints one JSON line with the throughput in simulated audio-seconds per second,
the roofline of the dominant kernel (the filter-and-mix kernel, HBM-bound by
the published peaks), the plain per-utterance GPU path and the FP64 oracle on
the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks: HBM3E bandwidth and the FP32 vector rate.  The FP32
# figure counts packed FP32 instructions (two lanes' worth per instruction);
# the library emits none, so the unpacked rate, 256 CUs x 64 lanes x 2 FLOP
# per FMA x 2.4 GHz = 78.6 TFLOP/s, is the practical ceiling of its
# arithmetic and is reported beside the published one.
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_TFLOPS = 78.6
COUNTERS = os.path.join(ROOT, "profiles", "mix_kernel_batched2048_hbm_counters.json")


def _code_only(text: str) -> str:
    """C/C++ source without its comments and blank lines (string and character
    literals are kept as they are), so that a change of comments alone does
    not make counters stale."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def source_digest() -> str:
    """Digest of the kernel sources' code (comments left out); counters taken
    on other code are stale."""
    import hashlib

    h = hashlib.sha256()
    for rel in ("paper_1712_03439_amd/csrc/rsim.hip", "paper_1712_03439_amd/csrc/fft_engine.hpp",
                "paper_1712_03439_amd/csrc/kernels.hpp", "include/rsim.h"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


# rsim_tune.variant code -> (mic accumulators, waves per SIMD) of the kernel
VARIANT_TEMPLATE = {1: (1, 2), 2: (2, 1), 3: (2, 2), 4: (1, 4)}


def mix_kernel_name(log2n: int, variant) -> str:
    """Symbol of the filter-and-mix kernel that runs size 2^log2n."""
    from paper_1712_03439_amd import autotune

    f = autotune.FAMILY[log2n]
    code = (variant[f] if variant is not None and variant[f] else autotune.DEFAULT_VARIANT) if f < 5 else 4
    jg, w = VARIANT_TEMPLATE[code]
    return f"void rsim::mix_kernel<{32 << f}, {jg}, {w}, false>(rsim::MixArgs)"


def counter_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernels have changed since it was taken or it
    covers another kernel."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256") != source_digest() or c.get("kernel") != kernel:
        return None
    return int(c["fetch_bytes_per_launch"] + c["write_bytes_per_launch"])


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def lpt_order(b) -> np.ndarray:
    """Longest work first: utterance length times (sources + mics)."""
    cost = b.src_len.astype(np.int64) * (b.n_src.astype(np.int64) + b.n_mic)
    return np.argsort(-cost, kind="stable").astype(np.int32)


def host_plan(nx, I, J, lmax, tune_fft, tune_mac, l2=0):
    """N, hop and block count of an utterance under the schedule's rule (the
    batch's one size l2, else the utterance's own choice), for FLOP accounting."""
    from paper_1712_03439_amd import autotune

    if not l2:
        l2 = autotune.utterance_log2n(nx, I, J, lmax, tune_fft, tune_mac)
    N = 1 << l2
    B = N - lmax + 1
    return N, B, (nx + B - 1) // B


def host_info() -> dict:
    """The host's core count and CPU model (the oracle's hardware)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"os_cpu_count": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


class ParityCases:
    """GPU outputs of seeded utterances of every workload, kept on the host
    so that the FP64 oracle (in the cpu_baseline leg) can give each
    workload's max error relative to the peak (per utterance and mic, the
    tests' bar)."""

    def __init__(self):
        self.forward = []   # (label, sources, rirs, snrs, eta, gpu cut lengths [I][J], gpu outputs [J][T])
        self.adjoint = []   # (label, sources, cut rirs, alpha, g [J][T], gx [I][nx], gh [I][J][L0], ga [I][J])

    def add_forward(self, label, b, u, eta, y, rl, ol):
        S, J = b.max_src, b.n_mic
        I = int(b.n_src[u])
        off, st, T = int(b.out_off[u]), int(b.out_stride[u]), int(ol[u])
        outs = [np.array(y[off + j * st: off + j * st + T]) for j in range(J)]
        lens = [[int(rl[(u * S + i) * J + j]) for j in range(J)] for i in range(I)]
        self.forward.append((label, b.sources(u), b.rirs(u), list(b.snrs(u)), eta, lens, outs))


def _forward_error(case):
    import oracle

    label, xs, hs, snrs, eta, lens, outs = case
    ref, _, Ls, _ = oracle.simulate(xs, hs, snrs, eta)
    if Ls != lens:
        return label, float("inf")
    err = 0.0
    for j, got in enumerate(outs):
        if got.size != ref.shape[1]:
            return label, float("inf")
        peak = float(np.max(np.abs(ref[j]))) if got.size else 0.0
        if peak > 0.0:
            err = max(err, float(np.max(np.abs(got.astype(np.float64) - ref[j]))) / peak)
    return label, err


def _adjoint_error(case):
    import oracle

    label, xs, cut, alpha, g, gx, gh, ga = case
    dx, dh, da = oracle.mix_backward(xs, cut, alpha, g)
    err = 0.0
    for i in range(len(xs)):
        err = max(err, float(np.max(np.abs(gx[i] - dx[i]))) / float(np.max(np.abs(dx[i]))))
    peak_h = max(float(np.max(np.abs(r))) for row in dh for r in row if r.size)
    for i, row in enumerate(dh):
        for j, r in enumerate(row):
            got = np.asarray(gh[i][j], np.float64)
            ref = np.zeros(got.size)
            ref[: r.size] = r
            err = max(err, float(np.max(np.abs(got - ref))) / peak_h)
    err = max(err, float(np.max(np.abs(np.asarray(ga) - da))) / float(np.max(np.abs(da))))
    return label, err


def oracle_errors(cases: ParityCases, workers: int) -> dict:
    """Max error of each workload's GPU outputs relative to the oracle's
    peak, over its seeded utterances (one utterance per worker process);
    inf for a cut length or output length that differs."""
    import multiprocessing as mp

    out = {}
    with mp.get_context("spawn").Pool(workers, initializer=_one_thread) as pool:
        res = pool.map(_forward_error, cases.forward, chunksize=1) + pool.map(_adjoint_error, cases.adjoint,
                                                                               chunksize=1)
    for label, e in res:
        out[label] = max(out.get(label, 0.0), e)
    return {k: float(f"{v:.3g}") for k, v in out.items()}


def _one_thread():
    """Worker set-up: one compute thread per oracle process (the pool fills
    the cores; numpy's BLAS would otherwise start a thread pool in each)."""
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except ImportError:
        pass


def oracle_utterance(args):
    import oracle

    sources, rirs, snrs, eta = args
    oracle.simulate(sources, rirs, snrs, eta)
    return 0


def cpu_baseline(base, eta, n_utt, max_workers=16, cases: "ParityCases" = None):
    """The FP64 oracle (cut + gains + direct convolution + mix) on a seeded
    sample of utterances, one process per host core (at most 16); then, with
    `cases`, the oracle's max error of every workload's GPU outputs (untimed)."""
    import multiprocessing as mp

    rng = np.random.default_rng(1234)
    idx = rng.choice(base.n_utt, size=min(n_utt, base.n_utt), replace=False)
    tasks = [(base.sources(int(u)), base.rirs(int(u)), list(base.snrs(int(u))), eta) for u in idx]
    audio = float(np.sum(base.src_len[idx].astype(np.float64))) / 16000.0
    cores = max(1, min(max_workers, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_one_thread) as pool:
        pool.map(oracle_utterance, tasks[:cores])          # warm the workers
        t0 = time.perf_counter()
        pool.map(oracle_utterance, tasks, chunksize=1)
        dt = time.perf_counter() - t0
    res = {"value": audio / dt, "unit": "audio-s/s", "cores": cores, "kind": "oracle",
           "sample": f"{len(idx)} seeded utterances of the batched workload ({audio:.0f} audio-s), "
                     f"FP64 direct convolution, {dt:.1f} s wall",
           "host": host_info()}
    if cases is not None:
        t0 = time.perf_counter()
        res["max_rel_error"] = oracle_errors(cases, cores)
        res["error_seconds"] = round(time.perf_counter() - t0, 1)
    return res


def differentiation(torch, rsim, synth, dev, reps: int = 10, cases: "ParityCases" = None):
    """Forward and adjoint of the mix on the differentiation workload: 64
    utterances of 4 s, 3 sources, 4 mics, 8192-tap RIRs, no cut, N = 16384
    (hop 8193, 8 blocks), loss sum_j sum_n w_j[n] y_j[n]^2 so g = 2 w y.  The
    forward's kernel variant is chosen by the tuner on this batch (with 64
    utterances, splitting the mics over more work items can fill more CUs)."""
    from paper_1712_03439_amd import autotune

    b = synth.make_config3()
    U, S, J = b.n_utt, b.max_src, b.n_mic
    db = rsim.DeviceBatch(b, device=dev, fft_log2n=np.full(U, 14, np.int32))
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).to(dev)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        rsim.truncate_batch(db, math.inf, stream=stream)
    tune, entry = autotune.tune(db, alpha, policy=False, stream=stream)
    with torch.cuda.stream(stream):
        y = torch.zeros(max(db.y_len, 1), dtype=torch.float32, device=dev)
        ws_f = db.workspace(tune)
        ws_b = db.workspace(None, backward=True)
        rsim.mix(db, alpha, y=y, ws=ws_f, tune=tune, stream=stream)
        w = torch.from_numpy(synth.loss_weights(3, max(db.y_len, 1))).to(dev)
        g = 2.0 * w * y
        for _ in range(2):
            rsim.mix(db, alpha, y=y, ws=ws_f, tune=tune, stream=stream)
            rsim.mix_backward(db, alpha, g, ws=ws_b, stream=stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        for _ in range(reps):
            rsim.mix(db, alpha, y=y, ws=ws_f, tune=tune, stream=stream)
        ev[1].record(stream)
        for _ in range(reps):
            rsim.mix_backward(db, alpha, g, ws=ws_b, stream=stream)
        ev[2].record(stream)
    torch.cuda.synchronize()
    t_f = ev[0].elapsed_time(ev[1]) / reps
    t_b = ev[1].elapsed_time(ev[2]) / reps
    if cases is not None:
        # forward outputs of three utterances and the adjoint of one, for the oracle
        yh, rl, ol = y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()
        for u in (0, 31, 63):
            cases.add_forward("differentiation_forward", b, u, math.inf, yh, rl, ol)
        gx, gh, ga = rsim.mix_backward(db, alpha, g, ws=ws_b, stream=stream)
        torch.cuda.synchronize()
        gx, gh, ga, gn = gx.cpu().numpy(), gh.cpu().numpy(), ga.cpu().numpy(), g.cpu().numpy()
        u = 17
        I, T, nx = int(b.n_src[u]), int(ol[u]), int(b.src_len[u])
        xs, hs = b.sources(u), b.rirs(u)
        cut = [[np.asarray(hs[i][j], np.float32)[: int(rl[(u * S + i) * J + j])] for j in range(J)] for i in range(I)]
        a = alpha.cpu().numpy()[u * S * J:(u * S + I) * J].reshape(I, J).astype(np.float64)
        off, st = int(b.out_off[u]), int(b.out_stride[u])
        gu = np.stack([gn[off + j * st: off + j * st + T] for j in range(J)])
        gxu = [gx[int(b.src_off[u * S + i]): int(b.src_off[u * S + i]) + nx] for i in range(I)]
        ghu = [[gh[int(b.rir_off[(u * S + i) * J + j]): int(b.rir_off[(u * S + i) * J + j])
                   + int(b.rir_len0[(u * S + i) * J + j])] for j in range(J)] for i in range(I)]
        gau = ga[u * S * J:(u * S + I) * J].reshape(I, J)
        cases.adjoint.append(("differentiation_adjoint", xs, cut, a, gu, gxu, ghu, gau))
    # algorithmic work of the adjoint: per block J gradient spectra, I source
    # spectra, I inverse transforms (dx) and 2 I J spectral products; per
    # utterance I J RIR spectra and I J inverse transforms (r)
    N = 16384
    c = 2.5 * N * math.log2(N)
    mac = 8 * (N / 2 + 1)
    flops, byts = 0.0, 0
    L = db.rir_len.cpu().numpy().astype(np.int64).reshape(U, S * J)
    T = db.out_len.cpu().numpy().astype(np.int64)
    for u in range(U):
        I, nx = int(b.n_src[u]), int(b.src_len[u])
        lmax = int(L[u].max())
        nb = -(-nx // (N - lmax + 1))
        flops += nb * ((2 * I + J) * c + 2 * I * J * mac) + 2 * I * J * c
        byts += 4 * (2 * I * nx + J * int(T[u]) + 2 * int(L[u].sum())) + 8 * I * J
    achieved = flops / (t_b * 1e-3) / 1e12
    return {"workload": "64 utterances of 4 s, 3 sources, 4 mics, 8192-tap RIRs, no cut, N = 16384",
            "forward_variant": entry["variant"],
            "forward_ms": round(t_f, 4), "backward_ms": round(t_b, 4),
            "audio_s_per_s": round(b.audio_seconds / ((t_f + t_b) * 1e-3), 1),
            "backward_roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4)},
            "backward_alu_unpacked": {"achieved": round(achieved, 2), "peak": FP32_UNPACKED_TFLOPS,
                                      "unit": "TFLOP/s", "frac": round(achieved / FP32_UNPACKED_TFLOPS, 4)},
            "backward_hbm": {"achieved": round(byts / (t_b * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(byts / (t_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def rir_generation(torch, rsim, synth, dev, base, db, alpha, y, ws, tune, eta, reps: int = 5, order: int = 8):
    """The image-method RIRs (eq. 1, 17^3 virtual rooms) of every RIR slot of
    the batched workload's epoch (its lengths ceil(T60 fs)), generated on the
    GPU into a packed buffer: one untimed call, then `reps` timed ones; and
    whole epochs with those rooms (generation, cut and mix as one graph)."""
    geom, refl = synth.image_geometry(base)
    used = np.nonzero(base.rir_len0 > 0)[0]
    lens = base.rir_len0[used].astype(np.int32)
    off = base.rir_off[used].astype(np.int64)
    g = torch.from_numpy(geom[used]).to(dev)
    r = torch.from_numpy(refl[used]).to(dev)
    o = torch.from_numpy(off).to(dev)
    ln = torch.from_numpy(lens).to(dev)
    h = torch.empty(int(base.h.size), dtype=torch.float32, device=dev)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    max_len = int(lens.max())
    with torch.cuda.stream(stream):
        rsim.image_rir(g, r, o, ln, h, max_len, order=order, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            rsim.image_rir(g, r, o, ln, h, max_len, order=order, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    if rsim.device_status():
        raise RuntimeError("image-method generation flagged a bad descriptor")
    ms = e0.elapsed_time(e1) / reps
    taps = int(lens.astype(np.int64).sum())
    images = len(lens) * (2 * order + 1) ** 3
    gbs = 4.0 * taps / (ms * 1e-3) / 1e9
    # whole epochs: rooms -> RIRs -> cut -> mix, one graph per epoch
    gall, rall = torch.from_numpy(geom).to(dev), torch.from_numpy(refl).to(dev)
    h_saved = db.h
    db.h = h
    with torch.cuda.stream(stream):
        rsim.simulate_rooms(db, gall, rall, alpha, eta, order=order, y=y, ws=ws, tune=tune, use_graph=True,
                            stream=stream)
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        for _ in range(reps):
            rsim.simulate_rooms(db, gall, rall, alpha, eta, order=order, y=y, ws=ws, tune=tune, use_graph=True,
                                stream=stream)
        e3.record(stream)
    torch.cuda.synchronize()
    db.h = h_saved
    if rsim.device_status():
        raise RuntimeError("an image-method epoch flagged a bad descriptor")
    ms_epoch = e2.elapsed_time(e3) / reps
    return {"workload": f"{len(lens)} RIRs of the batched epoch ({taps} taps, lengths ceil(T60 fs)), "
                        f"{(2 * order + 1) ** 3} images each",
            "ms": round(ms, 4), "rirs_per_s": round(len(lens) / (ms * 1e-3), 1),
            "images_per_s": round(images / (ms * 1e-3), 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4)},
            "epoch_with_rooms": {"ms": round(ms_epoch, 4),
                                 "audio_s_per_s": round(base.audio_seconds / (ms_epoch * 1e-3), 1),
                                 "steps": "image-method RIRs, cut, mix as one graph"}}


def reverb_gains(torch, rsim, dev, base, db, reps: int = 5):
    """Energies of every reverberant source at every mic of the batched epoch
    (the reverberant-at-mic gain rule), after that epoch's cut: one untimed
    call, then `reps` timed ones."""
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        rsim.reverb_energy(db, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            e = rsim.reverb_energy(db, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    if not bool(torch.isfinite(e).all()) or rsim.device_status():
        raise RuntimeError("energy computation flagged a slot")
    # algorithmic work: per source, one transform per half block of N/2
    # samples and its spectral product (an add and a multiply-add per bin),
    # one inverse, one transform of the windowed autocorrelation and one per RIR
    L = db.rir_len.cpu().numpy().astype(np.int64).reshape(base.n_utt, base.max_src, base.n_mic)
    flops, byts = 0.0, 0
    for u in range(base.n_utt):
        nx = int(base.src_len[u])
        for i in range(int(base.n_src[u])):
            lmax = int(L[u, i].max())
            if lmax <= 0 or nx <= 0:
                continue
            m = 14
            while (1 << m) < 2 * lmax:
                m += 1
            N = 1 << m
            nb = -(-nx // (N // 2))
            c = 2.5 * N * m
            flops += nb * (c + 10 * (N / 2 + 1)) + 2 * c + base.n_mic * (c + 4 * (N / 2 + 1))
            byts += 4 * (nx + int(L[u, i].sum()))
    tf = flops / (ms * 1e-3) / 1e12
    return {"workload": "energies of every (source, mic) pair of the batched epoch after its cut",
            "ms": round(ms, 4), "audio_s_per_s": round(base.audio_seconds / (ms * 1e-3), 1),
            "roofline": {"bound": "alu", "achieved": round(tf, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / FP32_PEAK_TFLOPS, 4)},
            "alu_unpacked": {"achieved": round(tf, 2), "peak": FP32_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(tf / FP32_UNPACKED_TFLOPS, 4)},
            "hbm": {"achieved": round(byts / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s"}}


def front_end(torch, rsim, base, db, y, reps: int = 5, alpha=None, eta=20.0, tune=None, mix_ms=None):
    """The log-Mel features (Sec. 3) of every mic output of the batched epoch:
    one untimed call, then `reps` timed ones; then, with alpha, the front end
    fused into the mix (rsim_simulate_logmel: cut, mix and features, no y)
    against the unfused steps (cut + mix, then the separate front end)."""
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        rsim.logmel(db, y, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            rsim.logmel(db, y, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    if rsim.device_status():
        raise RuntimeError("the front end flagged a bad descriptor")
    ms = e0.elapsed_time(e1) / reps
    T = db.out_len.cpu().numpy().astype(np.int64)
    frames = int(rsim.mel_frames(T).sum()) * base.n_mic
    byts = 4 * base.n_mic * int(T.sum()) + frames * 128 * 4
    m = 9
    flops = frames * (2.5 * 512 * m + 4 * 257 + 2 * 2 * 257 + 128 * 8)
    tf = flops / (ms * 1e-3) / 1e12
    gbs = byts / (ms * 1e-3) / 1e9
    out = {"workload": f"128 log-Mel bands of every mic output of the batched epoch ({frames} frames)",
           "ms": round(ms, 4), "frames_per_s": round(frames / (ms * 1e-3), 1),
           "audio_s_per_s": round(base.audio_seconds / (ms * 1e-3), 1),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4)},
           "alu": {"achieved": round(tf, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(tf / FP32_PEAK_TFLOPS, 4)}}
    if alpha is not None:
        # cut + mix + features as one graph with the front end fused into the
        # mix, against cut + mix (one graph) and the separate front end
        off, cap, total = rsim.feature_layout(db)
        feat = torch.empty(max(total, 1), dtype=torch.float32, device=db.device)
        s_ = db.struct()
        import ctypes

        n = int(rsim.lib().rsim_simulate_logmel_workspace_bytes(ctypes.byref(s_), ctypes.byref(tune) if tune else None))
        wsf = torch.empty(max(n, 1), dtype=torch.uint8, device=db.device)
        wsu = db.workspace(tune)
        with torch.cuda.stream(stream):
            rsim.simulate_logmel(db, alpha, eta, feat=feat, ws=wsf, tune=tune, use_graph=True, stream=stream)
            e2, e3, e4 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e2.record(stream)
            for _ in range(reps):
                rsim.simulate_logmel(db, alpha, eta, feat=feat, ws=wsf, tune=tune, use_graph=True, stream=stream)
            e3.record(stream)
            for _ in range(reps):
                rsim.simulate(db, alpha, eta, y=y, ws=wsu, tune=tune, use_graph=True, stream=stream)
                rsim.logmel(db, y, stream=stream)
            e4.record(stream)
        torch.cuda.synchronize()
        if rsim.device_status():
            raise RuntimeError("the fused front end flagged a descriptor")
        fused, unfused = e2.elapsed_time(e3) / reps, e3.elapsed_time(e4) / reps
        byts_f = int(np.sum(base.n_src.astype(np.int64) * base.src_len)) * 4 + frames * 128 * 4
        out["fused"] = {"steps": "cut + mix with the front end fused (features only, no y), one graph",
                        "ms": round(fused, 4), "unfused_ms": round(unfused, 4),
                        "speedup": round(unfused / fused, 3),
                        "audio_s_per_s": round(base.audio_seconds / (fused * 1e-3), 1),
                        "hbm_bytes_algorithmic": byts_f}
    return out


def ladder(torch, rsim, base, db, alpha, y, mix_ms, reps: int = 3):
    """The paper's filtering ladder on the same epoch (Table 1): the
    full-length FFT filtering of eqs. 4-5 (one transform per signal, batched
    global-memory passes) against the overlap-add mix timed above."""
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    l2 = rsim.fft_filter_log2n(db)
    with torch.cuda.stream(stream):
        rsim.fft_filter(db, alpha, y=y, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            rsim.fft_filter(db, alpha, y=y, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    if rsim.device_status():
        raise RuntimeError("full-length filtering flagged an utterance")
    ms = e0.elapsed_time(e1) / reps
    sizes = {f"2^{k}": int(v) for k, v in zip(*np.unique(l2, return_counts=True))}
    return {"workload": "the batched epoch, each utterance at its own transform size", "fft_sizes": sizes,
            "full_length_fft_ms": round(ms, 3), "overlap_add_ms": round(mix_ms, 3),
            "overlap_add_speedup": round(ms / mix_ms, 2)}


def single_utterances(torch, rsim, synth, dev, reps: int = 20, cases: "ParityCases" = None):
    """Per-utterance latency of the two single-utterance workloads (the
    paper's Table 1 measures time per utterance): the tiny case (1 s, one
    4096-tap RIR, N = 8192, hop 4096, through rsim_ola_convolve) and one
    room (8 s, 3 sources at 10 and 20 dB SNR, 2 mics, 12000-tap RIRs cut at
    20 dB, N = 16384, through rsim_simulate, eager).  Each call is timed on
    its own, synchronised, after one untimed call: the host wall time per
    call (the latency a caller sees) and the GPU time between HIP events."""
    out = {}
    b0 = synth.make_config0()
    x = torch.from_numpy(b0.sources(0)[0]).to(dev)
    h = torch.from_numpy(b0.rirs(0)[0][0]).to(dev)
    b1 = synth.make_config1()
    db1 = rsim.DeviceBatch(b1, device=dev, fft_log2n=np.array([14], np.int32))
    a1 = torch.from_numpy(rsim.batch_gains(db1, b1.snr_db)).to(dev)
    y1 = db1.new_output()
    ws1 = db1.workspace()

    def timed(call):
        call()
        torch.cuda.synchronize()
        wall, gpu = [], []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record()
            r = call()
            e1.record()
            torch.cuda.synchronize()
            wall.append((time.perf_counter() - t0) * 1e3)
            gpu.append(e0.elapsed_time(e1))
        return r, float(np.median(wall)), float(np.median(gpu))

    y0, w0, g0 = timed(lambda: rsim.ola_convolve(x, h, 8192, 4096))
    _, w1, g1 = timed(lambda: rsim.simulate(db1, a1, 20.0, y=y1, ws=ws1))
    out["tiny"] = {"workload": "1 utterance of 1 s, 1 source, 1 mic, 4096-tap RIR, no cut, N = 8192, hop 4096 "
                               "(output 20095 samples)",
                   "ms_wall": round(w0, 4), "ms_gpu": round(g0, 4),
                   "audio_s_per_s": round(b0.audio_seconds / (w0 * 1e-3), 1)}
    out["one_room"] = {"workload": "1 utterance of 8 s, 3 sources (10 and 20 dB SNR), 2 mics, 12000-tap RIRs "
                                   "cut at 20 dB, N = 16384",
                       "ms_wall": round(w1, 4), "ms_gpu": round(g1, 4),
                       "audio_s_per_s": round(b1.audio_seconds / (w1 * 1e-3), 1)}
    if cases is not None:
        T = int(y0.numel())
        cases.forward.append(("tiny", b0.sources(0), b0.rirs(0), [0.0], math.inf, [[4096]],
                              [y0.cpu().numpy()[:T]]))
        cases.add_forward("one_room", b1, 0, 20.0, y1.cpu().numpy(), db1.rir_len.cpu().numpy(),
                          db1.out_len.cpu().numpy())
    return out


def gpu_share(torch, rsim, base, db, alpha, y, ws, tune, eta, full_ms, shares: int = 8, reps: int = 10):
    """The one-GPU part of the multi-GPU design: the share of the batched
    epoch one of `shares` GPUs would get when the utterances (in LPT order)
    are dealt round robin, run on this GPU as its own batch (cut + mix, one
    graph), to show what the smaller batch costs in occupancy."""
    order = lpt_order(base)
    idx = np.sort(order[::shares])
    sub = db.select(idx)
    u = torch.as_tensor(idx, device=db.device)
    S, J = db.S, db.J
    rows = ((u[:, None] * S + torch.arange(S, device=db.device)[None, :])[:, :, None] * J
            + torch.arange(J, device=db.device)[None, None, :]).reshape(-1)
    a = alpha[rows].contiguous()
    ws_s = sub.workspace(tune)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        rsim.simulate(sub, a, eta, y=y, ws=ws_s, tune=tune, use_graph=True, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            rsim.simulate(sub, a, eta, y=y, ws=ws_s, tune=tune, use_graph=True, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    audio = float(np.sum(base.src_len[idx].astype(np.float64))) / 16000.0
    return {"workload": f"{len(idx)} of the batched epoch's {base.n_utt} utterances (every {shares}th in "
                        f"LPT order: one GPU's share of {shares})",
            "ms": round(ms, 4), "audio_s_per_s": round(audio / (ms * 1e-3), 1),
            "share_of_epoch_audio": round(audio / base.audio_seconds, 4),
            "time_vs_full_epoch": round(ms / full_ms, 4)}


def large_thresholds(torch, rsim, autotune, synth, dev, etas=(math.inf, 30.0, 20.0, 10.0), reps: int = 3,
                     cases: "ParityCases" = None, full_length: bool = True):
    """The large batched workload (4096 utterances of 1-20 s, up to 4 sources,
    8 mics, T60 U(0.1, 1.0) s, RIRs up to 16000 taps) at each cut threshold:
    per threshold the tuner runs on the cut batch, then cut + mix run as one
    graph `reps` times (after one untimed run); then the full-length FFT
    filtering of eqs. 4-5 on the same cut batch (one untimed and one timed
    call), the comparison of Sec. 2.3 and Table 2 (cost against threshold,
    with and without overlap-add)."""
    t0 = time.perf_counter()
    b = synth.make_config4()
    log(f"large workload: {b.n_utt} utterances, {b.audio_seconds:.0f} audio-s ({time.perf_counter() - t0:.1f} s)")
    db = rsim.DeviceBatch(b, device=dev)  # the device schedule orders the work
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).to(dev)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    y = db.new_output()
    out = {"workload": f"{b.n_utt} utterances of 1-20 s, 1 + U{{0..3}} sources, 8 mics, T60 U(0.1,1.0) s, "
                       f"L0 = ceil(T60 fs) <= 16000", "audio_s": round(b.audio_seconds, 1), "thresholds": {}}
    for eta in etas:
        with torch.cuda.stream(stream):
            rsim.truncate_batch(db, eta, stream=stream)
        stream.synchronize()
        tune, entry = autotune.tune(db, alpha, stream=stream)
        ws = db.workspace(tune)
        with torch.cuda.stream(stream):
            rsim.simulate(db, alpha, eta, y=y, ws=ws, tune=tune, use_graph=True, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                rsim.simulate(db, alpha, eta, y=y, ws=ws, tune=tune, use_graph=True, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        L = db.rir_len.cpu().numpy().astype(np.int64)
        T = db.out_len.cpu().numpy().astype(np.int64)
        I = b.n_src.astype(np.int64)
        J = b.n_mic
        byt = 4 * (np.sum(I * b.src_len) + np.sum(L) + J * np.sum(T)) + (4 * np.sum(b.rir_len0) if eta != math.inf else 0)
        Lr = L.reshape(b.n_utt, b.max_src * J)
        shapes = [(int(b.src_len[u]), int(I[u]), J, int(Lr[u].max())) for u in range(b.n_utt)
                  if int(Lr[u].max()) > 0 and b.src_len[u] > 0]
        tf, tm = autotune.costs(tune)
        l2b = autotune.batch_log2n(shapes, tf, tm) if tune.one_size else 0
        fl, sizes = 0.0, {}
        for nx, Iu, _, lmax in shapes:
            N, B, nb = host_plan(nx, Iu, J, lmax, tf, tm, l2b)
            c = 2.5 * N * math.log2(N)
            fl += nb * ((Iu + J) * c + Iu * J * 8 * (N / 2 + 1)) + Iu * J * c
            sizes[N] = sizes.get(N, 0) + 1
        key = "inf" if eta == math.inf else f"{eta:g}"
        out["thresholds"][key] = {
            "ms": round(ms, 3), "audio_s_per_s": round(b.audio_seconds / (ms * 1e-3), 1),
            "mean_cut_len": round(float(L[L > 0].mean()), 1), "fft_sizes": {str(k): v for k, v in sorted(sizes.items())},
            "variant": entry["variant"], "policy": "one size per batch" if tune.one_size else "size per utterance",
            "policy_ms": {k: round(v, 3) for k, v in entry.get("policy_ms", {}).items()},
            "alu": {"achieved": round(fl / (ms * 1e-3) / 1e12, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(fl / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)},
            "hbm": {"achieved": round(byt / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
        if cases is not None:
            yh, rl, ol = y.cpu().numpy(), db.rir_len.cpu().numpy(), db.out_len.cpu().numpy()
            longest = int(np.argmax(b.src_len.astype(np.int64) * b.n_src))
            for u in sorted({longest} | set(np.random.default_rng(11).choice(b.n_utt, 3, replace=False).tolist())):
                cases.add_forward(f"large_eta_{key}", b, int(u), eta, yh, rl, ol)
        del ws
        if full_length:
            with torch.cuda.stream(stream):
                rsim.fft_filter(db, alpha, y=y, stream=stream)
                e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e2.record(stream)
                rsim.fft_filter(db, alpha, y=y, stream=stream)
                e3.record(stream)
            torch.cuda.synchronize()
            fms = e2.elapsed_time(e3)
            out["thresholds"][key]["full_length_fft_ms"] = round(fms, 2)
            out["thresholds"][key]["full_length_fft_audio_s_per_s"] = round(b.audio_seconds / (fms * 1e-3), 1)
            out["thresholds"][key]["overlap_add_speedup"] = round(fms / ms, 2)
        log(f"large workload, eta {key}: {ms:.2f} ms (cut + mix), {out['thresholds'][key]['audio_s_per_s']:.4g} "
            f"audio-s/s, sizes {out['thresholds'][key]['fft_sizes']}"
            + (f"; full-length FFT {out['thresholds'][key]['full_length_fft_ms']:.1f} ms" if full_length else ""))
    if rsim.device_status():
        raise RuntimeError("the large workload flagged a descriptor or plan")
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eta", type=float, default=20.0)
    ap.add_argument("--n-utt", type=int, default=2048)
    ap.add_argument("--distinct-rooms", type=int, default=0,
                    help="distinct epochs of RIRs to draw (default: warmup + steps)")
    ap.add_argument("--plain-utts", type=int, default=256)
    ap.add_argument("--cpu-utts", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-diff", action="store_true", help="skip the adjoint (differentiation workload) timing")
    ap.add_argument("--no-rirgen", action="store_true", help="skip the image-method RIR generation timing")
    ap.add_argument("--no-reverb", action="store_true", help="skip the reverberant-energy (gain rule) timing")
    ap.add_argument("--no-frontend", action="store_true", help="skip the log-Mel front-end timing")
    ap.add_argument("--no-ladder", action="store_true", help="skip the full-length FFT filtering timing")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large batched workload (4096 utterances, 8 mics) at eta = inf, 30, 20, 10 dB "
                         "(about a minute of host-side generation and 35 GB of GPU memory)")
    ap.add_argument("--no-single", action="store_true", help="skip the single-utterance latencies")
    ap.add_argument("--no-share", action="store_true", help="skip the one-GPU-share timing")
    ap.add_argument("--order", choices=("device", "host"), default="device",
                    help="'device': the schedule orders each family's utterances longest work first "
                         "after the cut; 'host': the order of lpt_order() is passed in")
    ap.add_argument("--tune", default="measure",
                    help="'measure' (time every FFT size and kernel variant on the first epoch's "
                         "batch before the warmup), 'model' (the built-in cost model), 'auto' (this "
                         "device's entry of the stored table) or a table JSON path")
    ap.add_argument("--save-tune", default="", help="with --tune measure: merge the measured entry into this JSON")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the warmup, fill and copy a buffer of this size (a reference "
                         "for the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs the hot path on one GPU; --gpus {args.gpus} is not "
              f"supported (each GPU would take its own share of the utterances; this path runs on one GPU).",
              file=sys.stderr)
        return 2

    import torch

    import synth
    from paper_1712_03439_amd import autotune, rsim

    torch.cuda.set_device(0)
    rsim.init()
    dev = torch.device("cuda:0")
    W, K = args.warmup, args.steps
    E = args.distinct_rooms or (W + K)

    t0 = time.perf_counter()
    base = synth.make_config2(epoch=0, n_utt=args.n_utt)
    log(f"dataset: {base.n_utt} utterances, {base.audio_seconds:.0f} audio-s, "
        f"{base.x.nbytes / 1e9:.2f} GB of sources ({time.perf_counter() - t0:.1f} s)")
    order = lpt_order(base) if args.order == "host" else None
    tune = None if args.tune == "measure" else autotune.load(args.tune)

    x_dev = torch.from_numpy(base.x).to(dev)
    epochs = []
    power = None
    for e in range(E):
        b = base if e == 0 else synth.reroom(base, 2, e, (0.1, 0.9))
        db = rsim.DeviceBatch(b, device=dev, order=order, upload_data=False)
        db.x = x_dev
        db.h = torch.from_numpy(b.h).to(dev)
        if power is None:
            power = rsim.source_power(db).cpu().numpy()
        alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db, power)).to(dev)
        epochs.append((b, db, alpha))
        if e % 5 == 0:
            log(f"rooms for epoch {e} ready ({time.perf_counter() - t0:.1f} s)")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    tune_info = {"source": "built-in cost model" if tune is None else f"stored table ({args.tune})"}
    if args.tune == "measure":
        # The tuner times every FFT size and kernel variant on the first
        # epoch's (cut) batch; its table then drives every epoch's schedule.
        t1 = time.perf_counter()
        _, db0, alpha0 = epochs[0]
        rsim.truncate_batch(db0, args.eta, stream=stream)
        stream.synchronize()
        tune, entry = autotune.tune(db0, alpha0, save=args.save_tune or None, stream=stream)
        tune_info = {"source": "measured on the first epoch's batch", "variant": entry["variant"],
                     "ms": {k: v["ms"] for k, v in entry["measured"]["sizes"].items()},
                     "policy_ms": entry.get("policy_ms"),
                     "sizes_from": entry.get("sizes_from"),
                     "seconds": round(time.perf_counter() - t1, 2)}
        log(f"tuned in {tune_info['seconds']} s: variants {entry['variant']}, "
            + ", ".join(f"N=2^{k}: " + "/".join(f"{t:.3f}" for t in v.values()) + " ms"
                        for k, v in tune_info["ms"].items()))
    tf, tm = autotune.costs(tune)
    y = torch.empty(max(b.y_len for b, _, _ in epochs), dtype=torch.float32, device=dev)
    ws = torch.empty(max(db.workspace_bytes(tune) for _, db, _ in epochs), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    use_graph = not args.no_graph

    def run_epoch(k, ev=None):
        b, db, alpha = epochs[k % E]
        if ev:
            ev[0].record(stream)
        rsim.truncate_batch(db, args.eta, stream=stream)
        if ev:
            ev[1].record(stream)
        rsim.mix(db, alpha, y=y, ws=ws, tune=tune, use_graph=use_graph, stream=stream)
        if ev:
            ev[2].record(stream)

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        a.fill_(1.0)       # writes n * 4 bytes
        c.copy_(a)         # reads and writes n * 4 bytes
        torch.cuda.synchronize()
        del a, c
        log(f"copy probe: fill + copy of {args.copy_probe_mib} MiB")

    with torch.cuda.stream(stream):
        for k in range(W):
            run_epoch(k)
        torch.cuda.synchronize()
        log("warmup done")
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(K):
            run_epoch(W + k, evs[k])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
    st = rsim.device_status()
    if st:
        log(f"device status word {st:#x}")
    trunc_ms = [e[0].elapsed_time(e[1]) for e in evs]
    mix_ms = [e[1].elapsed_time(e[2]) for e in evs]
    audio = base.audio_seconds
    value = K * audio / elapsed
    log(f"timed {K} epochs: {elapsed * 1e3 / K:.3f} ms/epoch, cut {np.mean(trunc_ms):.3f} ms, "
        f"mix {np.mean(mix_ms):.3f} ms, {value:.4g} audio-s/s")

    # Algorithmic bytes and FLOPs of the mix launches of the timed epochs.
    byt, flops, byt_cut = [], [], []
    sizes = {}
    one_size = True if tune is None else bool(tune.one_size)
    for k in range(K):
        b, db, _ = epochs[(W + k) % E]
        L = db.rir_len.cpu().numpy().astype(np.int64)
        T = db.out_len.cpu().numpy().astype(np.int64)
        I = b.n_src.astype(np.int64)
        J = b.n_mic
        byt.append(4 * (np.sum(I * b.src_len) + np.sum(L) + J * np.sum(T)))
        byt_cut.append(4 * np.sum(b.rir_len0.astype(np.int64)))
        f = 0.0
        Lr = L.reshape(b.n_utt, b.max_src * J)
        shapes = [(int(b.src_len[u]), int(I[u]), J, int(Lr[u].max())) for u in range(b.n_utt)
                  if int(Lr[u].max()) > 0 and b.src_len[u] > 0]
        l2b = autotune.batch_log2n(shapes, tf, tm) if one_size else 0
        for nx, Iu, _, lmax in shapes:
            N, B, nb = host_plan(nx, Iu, J, lmax, tf, tm, l2b)
            c = 2.5 * N * math.log2(N)
            f += nb * ((Iu + J) * c + Iu * J * 8 * (N / 2 + 1)) + Iu * J * c
            sizes[N] = sizes.get(N, 0) + 1
        flops.append(f)
    t_mix = float(np.mean(mix_ms)) * 1e-3
    achieved = float(np.mean(byt)) / t_mix / 1e9
    alu = float(np.mean(flops)) / t_mix / 1e12
    # The binding bound of the mix is the one with the longer time at the
    # published peaks (HBM 8 TB/s, FP32 vector 157.3 TFLOP/s).
    t_alu, t_hbm = float(np.mean(flops)) / (FP32_PEAK_TFLOPS * 1e12), float(np.mean(byt)) / (HBM_PEAK_GBS * 1e9)
    dom_n = max(sizes, key=lambda n: sizes[n] * n * math.log2(n))
    kernel = mix_kernel_name(int(math.log2(dom_n)), list(tune.variant) if tune is not None else None)
    traffic = counter_traffic(kernel)
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": round(alu, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(alu / FP32_PEAK_TFLOPS, 4), "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    cases = ParityCases()
    b_last, db_last, _ = epochs[(W + K - 1) % E]
    yh, rlh, olh = y.cpu().numpy(), db_last.rir_len.cpu().numpy(), db_last.out_len.cpu().numpy()
    longest = int(np.argmax(b_last.src_len.astype(np.int64) * b_last.n_src))
    pick = {longest} | set(np.random.default_rng(5).choice(b_last.n_utt, 15, replace=False).tolist())
    for u in sorted(pick):
        cases.add_forward("batched", b_last, int(u), args.eta, yh, rlh, olh)
    del yh
    result = {
        "metric": "simulated audio-sec/sec (FP32, 1 MI355X) batched vs plain; HBM GB/s fraction",
        "value": round(value, 1),
        "unit": "audio-s/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(elapsed * 1e3 / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched: {base.n_utt} utterances of 1-15 s at 16 kHz, 1 target + "
                               f"U{{0..3}} noises, 2 mics, T60 U(0.1,0.9) s, L0 = ceil(T60 fs), cut "
                               f"{args.eta:g} dB, SNR U(0,30) dB, fresh RIRs every epoch",
                   "global_batch": base.n_utt, "audio_s_per_step": round(audio, 1),
                   "eta_db": args.eta, "hip_graph": use_graph,
                   "order": "longest work first, device schedule after the cut" if args.order == "device"
                            else "longest work first by source length x (sources + mics), host",
                   "fft_sizes": {str(k): v // K for k, v in sorted(sizes.items())},
                   "tune": dict(tune_info, policy="one size per batch" if one_size else "size per utterance")},
        "roofline": roof,
        "hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4)},
        "alu": {"achieved": round(alu, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(alu / FP32_PEAK_TFLOPS, 4)},
        "alu_unpacked": {"achieved": round(alu, 2), "peak": FP32_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(alu / FP32_UNPACKED_TFLOPS, 4),
                         "note": "the ceiling of the library's arithmetic: it emits no packed FP32 instructions"},
        "dominant_kernel": kernel,
        "kernel_ms": {"cut": round(float(np.mean(trunc_ms)), 4), "mix": round(float(np.mean(mix_ms)), 4)},
        "cut_hbm": {"achieved": round(float(np.mean(byt_cut)) / (float(np.mean(trunc_ms)) * 1e-3) / 1e9, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(float(np.mean(byt_cut)) / (float(np.mean(trunc_ms)) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "alu_model": "2.5 N log2 N per real FFT + 8 (N/2+1) per spectral MAC; published FP32 vector peak "
                     "157.3 TFLOP/s (packed); unpacked 256 CUs x 64 lanes x 2 FLOP (FMA) x 2.4 GHz = 78.6",
        "bytes_per_step": {"mix": int(np.mean(byt)), "cut": int(np.mean(byt_cut))},
    }

    # the front end reads the last timed epoch's output, still in y
    if not args.no_frontend:
        b_last, db_last, _ = epochs[(W + K - 1) % E]
        _, _, alpha_last = epochs[(W + K - 1) % E]
        result["front_end"] = front_end(torch, rsim, b_last, db_last, y, alpha=alpha_last, eta=args.eta, tune=tune)
        d = result["front_end"]
        log(f"log-Mel front end: {d['ms']:.3f} ms per epoch, {d['frames_per_s']:.4g} frames/s, "
            f"{d['roofline']['frac']:.3f} of the HBM peak; fused into the mix {d['fused']['ms']:.3f} ms per epoch "
            f"against {d['fused']['unfused_ms']:.3f} ms unfused")

    if not args.no_plain:
        # Plain per-utterance path: the same kernels, one utterance per call, no
        # graph, synchronised after every utterance.
        b, db, alpha = epochs[0]
        rng = np.random.default_rng(7)
        sub = np.sort(rng.choice(b.n_utt, size=min(args.plain_utts, b.n_utt), replace=False))
        ws1 = torch.empty(rsim.single_workspace_bytes(db), dtype=torch.uint8, device=dev)
        t_sum, audio_sub = 0.0, 0.0
        with torch.cuda.stream(stream):
            for u in sub:
                torch.cuda.synchronize()
                t0u = time.perf_counter()
                rsim.simulate_one(db, int(u), alpha, args.eta, y, ws1, stream=stream)
                torch.cuda.synchronize()
                t_sum += time.perf_counter() - t0u
                audio_sub += float(b.src_len[u]) / 16000.0
        plain = audio_sub / t_sum
        result["plain_gpu"] = {"value": round(plain, 1), "unit": "audio-s/s",
                               "sample": f"{len(sub)} utterances, one call each, no graph, "
                                         f"synchronised per utterance"}
        result["speedup_vs_plain"] = round(value / plain, 2)
        log(f"plain per-utterance path: {plain:.4g} audio-s/s ({value / plain:.1f}x)")

    if not args.no_share:
        b0_, db0_, alpha0_ = epochs[0]
        result["one_gpu_share"] = gpu_share(torch, rsim, b0_, db0_, alpha0_, y, ws, tune, args.eta,
                                            float(np.mean(mix_ms)) + float(np.mean(trunc_ms)))
        d = result["one_gpu_share"]
        log(f"one GPU's share (1/8 of the epoch): {d['ms']:.3f} ms, {d['audio_s_per_s']:.4g} audio-s/s")

    if not args.no_single:
        result["single_utterance"] = single_utterances(torch, rsim, synth, dev, cases=cases)
        d = result["single_utterance"]
        log(f"single utterances: tiny {d['tiny']['ms_wall']:.3f} ms, one room {d['one_room']['ms_wall']:.3f} ms "
            f"per call (wall)")

    if not args.no_diff:
        result["differentiation"] = differentiation(torch, rsim, synth, dev, cases=cases)
        d = result["differentiation"]
        log(f"differentiation workload: forward {d['forward_ms']:.3f} ms, adjoint {d['backward_ms']:.3f} ms, "
            f"adjoint at {d['backward_roofline']['frac']:.3f} of the FP32 peak")

    if not args.no_rirgen:
        _, db0, alpha0 = epochs[0]
        result["rir_generation"] = rir_generation(torch, rsim, synth, dev, base, db0, alpha0, y, ws, tune, args.eta)
        d = result["rir_generation"]
        log(f"image-method RIRs: {d['ms']:.3f} ms for one epoch's RIRs, {d['rirs_per_s']:.4g} RIRs/s, "
            f"{d['roofline']['frac']:.3f} of the HBM peak; epochs with image-method rooms "
            f"{d['epoch_with_rooms']['ms']:.3f} ms ({d['epoch_with_rooms']['audio_s_per_s']:.4g} audio-s/s)")

    if not args.no_ladder:
        b_last, db_last, alpha_last = epochs[(W + K - 1) % E]
        rsim.truncate_batch(db_last, args.eta)
        result["ladder"] = ladder(torch, rsim, b_last, db_last, alpha_last, y, float(np.mean(mix_ms)))
        d = result["ladder"]
        log(f"full-length FFT filtering: {d['full_length_fft_ms']:.2f} ms per epoch "
            f"(overlap-add {d['overlap_add_ms']:.2f} ms, {d['overlap_add_speedup']:.1f}x)")

    if not args.no_reverb:
        b0, db0, _ = epochs[0]
        rsim.truncate_batch(db0, args.eta)
        result["reverb_gains"] = reverb_gains(torch, rsim, dev, b0, db0)
        d = result["reverb_gains"]
        log(f"reverberant energies: {d['ms']:.3f} ms per epoch, {d['roofline']['frac']:.3f} of the FP32 peak")

    if not args.no_large:
        del y, ws
        epochs.clear()
        torch.cuda.empty_cache()
        result["large"] = large_thresholds(torch, rsim, autotune, synth, dev, cases=cases)

    if not args.no_cpu:
        log("timing the FP64 oracle on the host cores, then its errors of every workload's outputs ...")
        result["cpu_baseline"] = cpu_baseline(base, args.eta, args.cpu_utts, cases=cases)
        log(f"oracle: {result['cpu_baseline']['value']:.4g} audio-s/s on "
            f"{result['cpu_baseline']['cores']} cores; max errors {result['cpu_baseline']['max_rel_error']}")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
