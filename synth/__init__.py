"""Seeded synthetic workloads for the room-simulator hot path.

This module only draws random inputs: speech-like and noise sources, decaying
room impulse responses, SNRs and utterance lengths, and packs them into flat
arrays.  It holds none of the method's arithmetic (no cut, no convolution, no
gain rule), so both the FP64 oracle and the GPU path can consume exactly the
same inputs.

Shapes follow the paper's workload description: 16 kHz sampling and two
microphones (Sec. 2.1, the paragraph after eq. 2); 0-3 noise sources per
utterance; utterances of several seconds and RIRs of a few thousand taps
(Sec. 2.2, the statistics quoted before eq. 3); T60 around 0.5 s (Table 4).
The paper's corpus and room sampler are not available, so everything here is
synthetic; the recipe is documented next to each generator.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

FS = 16000
BASE_SEED = 1712_03439
POOL_LEN = 1 << 23          # 524 s of audio per source pool


def seed_for(config: int, epoch: int = 0) -> int:
    """Seed of (config, epoch): every epoch draws fresh RIRs and SNRs."""
    return BASE_SEED + 1000 * int(config) + int(epoch)


def rng_for(config: int, epoch: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(config, epoch)))


def _rms_normalise(s: np.ndarray, rms: float) -> np.ndarray:
    cur = math.sqrt(float(np.mean(s.astype(np.float64) ** 2))) if s.size else 0.0
    if cur == 0.0:
        return s.astype(np.float32)
    return (s * (rms / cur)).astype(np.float32)


def speech_like(rng: np.random.Generator, n: int, rms: float = 0.1) -> np.ndarray:
    """AR(1) (coefficient 0.95) Gaussian noise times a 4 Hz syllabic envelope."""
    if n <= 0:
        return np.zeros(0, np.float32)
    w = rng.standard_normal(n)
    # AR(1) by a first-order IIR; scipy's lfilter keeps this fast for long n.
    from scipy.signal import lfilter

    s = lfilter([1.0], [1.0, -0.95], w)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    t = np.arange(n, dtype=np.float64)
    env = 0.5 * (1.0 - np.cos(2.0 * math.pi * 4.0 * t / FS + phi))
    return _rms_normalise(s * env, rms)


def white_noise(rng: np.random.Generator, n: int, rms: float = 0.1) -> np.ndarray:
    if n <= 0:
        return np.zeros(0, np.float32)
    return _rms_normalise(rng.standard_normal(n), rms)


def pink_noise(rng: np.random.Generator, n: int, rms: float = 0.1) -> np.ndarray:
    """White noise shaped by 1/sqrt(k) in the rfft domain, DC removed."""
    if n <= 0:
        return np.zeros(0, np.float32)
    from scipy.fft import irfft, next_fast_len, rfft

    m = next_fast_len(n, real=True)
    w = rng.standard_normal(m)
    spec = rfft(w)
    k = np.arange(spec.size, dtype=np.float64)
    shape = np.zeros_like(k)
    shape[1:] = 1.0 / np.sqrt(k[1:])
    return _rms_normalise(irfft(spec * shape, m)[:n], rms)


def rir(rng: np.random.Generator, length: int, t60: float, delay: int,
        sigma0: float = 0.25) -> np.ndarray:
    """Synthetic RIR: unit direct path at `delay`, then Gaussian noise decaying
    by 60 dB over t60 seconds (amplitude 10^(-3 (n-d) / (t60 fs)))."""
    h = np.zeros(length, np.float64)
    if length <= 0:
        return h.astype(np.float32)
    d = min(int(delay), length - 1)
    h[d] = 1.0
    m = length - d - 1
    if m > 0:
        n = np.arange(1, m + 1, dtype=np.float64)
        h[d + 1:] = sigma0 * rng.standard_normal(m) * 10.0 ** (-3.0 * n / (t60 * FS))
    return h.astype(np.float32)


@dataclasses.dataclass
class Batch:
    """A packed batch of utterances.

    Sources of utterance u: x[src_off[u*max_src+i] : +src_len[u]] for i < n_src[u]
    (i = 0 is the target).  RIR (u, i, j): h[rir_off[(u*max_src+i)*J+j] : +rir_len0[...]].
    Output of utterance u, mic j: y[out_off[u] + j*out_stride[u] : +out_stride[u]],
    out_stride[u] = src_len[u] + max_i,j rir_len0 - 1 (room for the uncut length).
    Unused (i >= n_src[u]) slots have length 0 and offset 0.
    """

    n_utt: int
    n_mic: int
    max_src: int
    n_src: np.ndarray      # int32 [U]
    src_len: np.ndarray    # int32 [U]
    src_off: np.ndarray    # int64 [U*max_src]
    rir_off: np.ndarray    # int64 [U*max_src*J]
    rir_len0: np.ndarray   # int32 [U*max_src*J]
    out_off: np.ndarray    # int64 [U]
    out_stride: np.ndarray  # int32 [U]
    x: np.ndarray          # float32 packed sources
    h: np.ndarray          # float32 packed RIRs
    snr_db: np.ndarray     # float64 [U*max_src], entry 0 of each utterance unused
    t60: np.ndarray        # float64 [U*max_src*J]
    y_len: int             # total floats of the packed output

    def sources(self, u: int) -> List[np.ndarray]:
        n = int(self.src_len[u])
        return [self.x[int(self.src_off[u * self.max_src + i]):][:n]
                for i in range(int(self.n_src[u]))]

    def rirs(self, u: int) -> List[List[np.ndarray]]:
        out = []
        for i in range(int(self.n_src[u])):
            row = []
            for j in range(self.n_mic):
                r = (u * self.max_src + i) * self.n_mic + j
                row.append(self.h[int(self.rir_off[r]):][:int(self.rir_len0[r])])
            out.append(row)
        return out

    def snrs(self, u: int) -> np.ndarray:
        return self.snr_db[u * self.max_src:(u + 1) * self.max_src][: int(self.n_src[u])]

    @property
    def audio_seconds(self) -> float:
        return float(np.sum(self.src_len.astype(np.float64))) / FS


def pack(sources: Sequence[Sequence[np.ndarray]], rirs: Sequence[Sequence[Sequence[np.ndarray]]],
         snr_db: Sequence[Sequence[float]], n_mic: int,
         t60: Optional[Sequence[Sequence[Sequence[float]]]] = None) -> Batch:
    """Pack per-utterance lists into a Batch (no arithmetic on the data)."""
    U = len(sources)
    max_src = max(1, max(len(s) for s in sources)) if U else 1
    n_src = np.zeros(U, np.int32)
    src_len = np.zeros(U, np.int32)
    src_off = np.zeros(U * max_src, np.int64)
    rir_off = np.zeros(U * max_src * n_mic, np.int64)
    rir_len0 = np.zeros(U * max_src * n_mic, np.int32)
    out_off = np.zeros(U, np.int64)
    out_stride = np.zeros(U, np.int32)
    snr = np.zeros(U * max_src, np.float64)
    t60a = np.zeros(U * max_src * n_mic, np.float64)
    xs, hs = [], []
    xo = ho = yo = 0
    for u in range(U):
        I = len(sources[u])
        n_src[u] = I
        nx = len(sources[u][0]) if I else 0
        src_len[u] = nx
        for i in range(I):
            assert len(sources[u][i]) == nx, "all sources of an utterance share one length"
            src_off[u * max_src + i] = xo
            xs.append(np.asarray(sources[u][i], np.float32))
            xo += nx
            if i > 0:
                snr[u * max_src + i] = float(snr_db[u][i])
        lmax0 = 0
        for i in range(I):
            for j in range(n_mic):
                r = (u * max_src + i) * n_mic + j
                hh = np.asarray(rirs[u][i][j], np.float32)
                rir_off[r] = ho
                rir_len0[r] = hh.size
                hs.append(hh)
                ho += hh.size
                lmax0 = max(lmax0, hh.size)
                if t60 is not None:
                    t60a[r] = float(t60[u][i][j])
        stride = nx + lmax0 - 1 if (nx > 0 and lmax0 > 0) else 0
        out_off[u] = yo
        out_stride[u] = stride
        yo += n_mic * stride
    x = np.concatenate(xs) if xs else np.zeros(0, np.float32)
    h = np.concatenate(hs) if hs else np.zeros(0, np.float32)
    return Batch(U, n_mic, max_src, n_src, src_len, src_off, rir_off, rir_len0,
                 out_off, out_stride, x.astype(np.float32), h.astype(np.float32),
                 snr, t60a, int(yo))


# ---------------------------------------------------------------------------
# The five workload configurations (sizes from the workload descriptions).
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Config:
    cid: int
    name: str
    description: str


CONFIGS = {
    0: Config(0, "tiny", "1 x 1 s, I=J=1, RIR 4096 (T60 0.3, delay 40), no cut, FFT 8192, hop 4096"),
    1: Config(1, "one_room", "1 x 8 s, target + white + pink noise at 10/20 dB, J=2, RIR 12000 (T60 0.6), cut 20 dB, FFT 16384"),
    2: Config(2, "batched", "2048 utterances 1-15 s, 1 + U{0..3} noises, J=2, T60 U(0.1,0.9), L0=ceil(T60 fs), cut 20 dB, SNR U(0,30)"),
    3: Config(3, "differentiation", "64 x 4 s, I=3, J=4, RIR 8192 (T60 0.5), no cut, FFT 16384"),
    4: Config(4, "large", "4096 utterances 1-20 s, I<=4, J=8, T60 U(0.1,1.0), L0<=16000, cut in {inf,30,20,10} dB"),
}


def _noise(rng, kind: str, n: int) -> np.ndarray:
    return white_noise(rng, n) if kind == "white" else pink_noise(rng, n)


def make_config0(epoch: int = 0) -> Batch:
    rng = rng_for(0, epoch)
    x = speech_like(rng, 16000)
    h = rir(rng, 4096, 0.3, 40)
    return pack([[x]], [[[h]]], [[0.0]], 1, [[[0.3]]])


def make_config1(epoch: int = 0) -> Batch:
    rng = rng_for(1, epoch)
    n = 8 * FS
    xs = [speech_like(rng, n), white_noise(rng, n), pink_noise(rng, n)]
    hs = [[rir(rng, 12000, 0.6, int(rng.integers(20, 401))) for _ in range(2)] for _ in range(3)]
    t60 = [[0.6, 0.6] for _ in range(3)]
    return pack([xs], [hs], [[0.0, 10.0, 20.0]], 2, [t60])


def make_utterances(cid: int, epoch: int, n_utt: int, len_s: tuple, max_noise: int,
                    n_mic: int, t60_range: tuple, max_taps: Optional[int] = None,
                    lengths: Optional[np.ndarray] = None, n_src: Optional[np.ndarray] = None,
                    sources_seed_epoch: int = 0) -> Batch:
    """Random utterances.  Utterance lengths, source counts and source signals
    come from the epoch-0 stream (the dataset), while RIRs, T60s and SNRs come
    from the `epoch` stream (a fresh room every epoch, see `reroom`)."""
    drng = rng_for(cid, sources_seed_epoch)
    if lengths is None:
        lengths = np.round(drng.uniform(len_s[0], len_s[1], n_utt) * FS).astype(np.int64)
    if n_src is None:
        n_src = 1 + drng.integers(0, max_noise + 1, n_utt)
    kinds = drng.integers(0, 2, (n_utt, max_noise + 1))
    # Sources are windows of three long pools (speech-like, white, pink) at
    # random offsets: the same statistics as drawing each one afresh, at a
    # fraction of the cost for thousands of utterances.
    pool_len = max(POOL_LEN, int(np.max(lengths)) + 1)
    pools = [speech_like(drng, pool_len), white_noise(drng, pool_len), pink_noise(drng, pool_len)]
    S = int(max(1, np.max(n_src)))
    total = int(np.sum(lengths * n_src))
    x = np.empty(total, np.float32)
    src_off = np.zeros(n_utt * S, np.int64)
    o = 0
    for u in range(n_utt):
        n = int(lengths[u])
        offs = drng.integers(0, pool_len - n + 1, int(n_src[u]))
        for i in range(int(n_src[u])):
            pool = pools[0] if i == 0 else pools[1 + int(kinds[u, i])]
            x[o:o + n] = pool[offs[i]:offs[i] + n]
            src_off[u * S + i] = o
            o += n
    base = Batch(n_utt, n_mic, S, np.asarray(n_src, np.int32), np.asarray(lengths, np.int32), src_off,
                 np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(n_utt, np.int64),
                 np.zeros(n_utt, np.int32), x, np.zeros(0, np.float32), np.zeros(n_utt * S),
                 np.zeros(0), 0)
    return reroom(base, cid, epoch, t60_range, max_taps)


def reroom(base: Batch, cid: int, epoch: int, t60_range: tuple,
           max_taps: Optional[int] = None) -> Batch:
    """The utterances of `base` in a fresh room for `epoch`: one T60 per
    utterance (every RIR of it has L0 = ceil(T60 fs) taps, capped at
    max_taps), a direct-path delay U{20..400} per RIR, Gaussian noise decaying
    by 60 dB over T60 (the `rir` recipe, drawn for all RIRs at once) and an SNR
    U(0, 30) dB per noise source.  Sources are shared with `base`."""
    rrng = rng_for(cid, 10_000 + epoch)
    U, S, J = base.n_utt, base.max_src, base.n_mic
    n_src = base.n_src.astype(np.int64)
    t60 = rrng.uniform(t60_range[0], t60_range[1], U)
    L0 = np.ceil(t60 * FS).astype(np.int64)
    if max_taps is not None:
        L0 = np.minimum(L0, max_taps)
    slot_u = np.repeat(np.arange(U), S * J)
    slot_i = np.tile(np.repeat(np.arange(S), J), U)
    used = slot_i < n_src[slot_u]
    slot_len = np.where(used, L0[slot_u], 0).astype(np.int64)
    rir_off = np.concatenate([[0], np.cumsum(slot_len)[:-1]]).astype(np.int64)
    ur = np.nonzero(used)[0]
    lens = slot_len[ur]
    delay = np.minimum(rrng.integers(20, 401, ur.size), lens - 1)
    k = np.arange(U * S)
    noise = (k % S >= 1) & (k % S < np.repeat(n_src, S))
    snr = np.zeros(U * S)
    snr[noise] = rrng.uniform(0.0, 30.0, int(np.sum(noise)))
    total = int(np.sum(lens))
    h = rrng.standard_normal(total, dtype=np.float32)
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    # Every RIR of an utterance shares its T60: one decay curve per utterance,
    # shifted to each RIR's direct-path delay.
    env_u = {}
    for k_, r in enumerate(ur):
        u = int(slot_u[r])
        L = int(lens[k_])
        if u not in env_u:
            rate = 3.0 * math.log(10.0) / (t60[u] * FS)
            env_u[u] = (0.25 * np.exp(-rate * np.arange(L, dtype=np.float64))).astype(np.float32)
        s0, d = int(starts[k_]), int(delay[k_])
        seg = h[s0:s0 + L]
        seg[:d] = 0.0
        seg[d] = 1.0
        seg[d + 1:] *= env_u[u][1:L - d]
    nx = base.src_len.astype(np.int64)
    stride = np.where((nx > 0) & (n_src > 0), nx + L0 - 1, 0)
    out_off = np.concatenate([[0], np.cumsum(J * stride)[:-1]]).astype(np.int64)
    return Batch(U, J, S, base.n_src, base.src_len, base.src_off, rir_off, slot_len.astype(np.int32),
                 out_off, stride.astype(np.int32), base.x, h, snr, np.where(used, t60[slot_u], 0.0),
                 int(np.sum(J * stride)))


def make_config2(epoch: int = 0, n_utt: int = 2048) -> Batch:
    return make_utterances(2, epoch, n_utt, (1.0, 15.0), 3, 2, (0.1, 0.9))


def make_config3(epoch: int = 0, n_utt: int = 64, nx: int = 4 * FS, taps: int = 8192) -> Batch:
    rng = rng_for(3, epoch)
    sources, rirs, snrs = [], [], []
    for _ in range(n_utt):
        sources.append([speech_like(rng, nx), white_noise(rng, nx), pink_noise(rng, nx)])
        rirs.append([[rir(rng, taps, 0.5, int(rng.integers(20, 401))) for _ in range(4)]
                     for _ in range(3)])
        snrs.append([0.0] + list(rng.uniform(0.0, 30.0, 2)))
    return pack(sources, rirs, snrs, 4)


def make_config4(epoch: int = 0, n_utt: int = 4096) -> Batch:
    return make_utterances(4, epoch, n_utt, (1.0, 20.0), 3, 8, (0.1, 1.0), max_taps=16000)


def loss_weights(cid: int, n: int) -> np.ndarray:
    """Seeded U(0,1) weights w of the loss sum_j sum_n w_j[n] y_j[n]^2."""
    rng = rng_for(cid, 777)
    return rng.uniform(0.0, 1.0, n).astype(np.float32)


def subset(b: Batch, idx: Sequence[int]) -> Batch:
    """The utterances `idx` of a batch, repacked."""
    return pack([b.sources(u) for u in idx], [b.rirs(u) for u in idx],
                [list(b.snr_db[u * b.max_src:u * b.max_src + int(b.n_src[u])]) for u in idx],
                b.n_mic)


def image_geometry(b: Batch, seed_epoch: int = 0, cid: int = 70):
    """Shoebox rooms for the image method (eq. 1), one per utterance of `b`,
    for every RIR slot of `b`: geom [U*S*J, 9] (room Lx Ly Lz, source xyz,
    mic xyz, metres, float64) and refl [U*S*J] (float64).  Recipe: sides
    U(3, 10) x U(3, 8) x U(2.5, 4) m; reflection coefficient U(0.3, 0.9);
    sources and mics uniform at least 0.5 m inside every wall; mics 10 cm
    apart along a random horizontal direction from a random centre; a source
    at least 0.2 m from every mic (redrawn otherwise).  Unused slots repeat
    the utterance's first valid geometry (they have no taps)."""
    rng = rng_for(cid, seed_epoch)
    U, S, J = b.n_utt, b.max_src, b.n_mic
    geom = np.zeros((U * S * J, 9))
    refl = np.zeros(U * S * J)
    for u in range(U):
        room = np.array([rng.uniform(3.0, 10.0), rng.uniform(3.0, 8.0), rng.uniform(2.5, 4.0)])
        r = rng.uniform(0.3, 0.9)
        span = 0.1 * (J - 1)
        centre = rng.uniform(0.5 + span, room - 0.5 - span)
        phi = rng.uniform(0.0, 2 * np.pi)
        step = 0.1 * np.array([np.cos(phi), np.sin(phi), 0.0])
        mics = [centre + (j - (J - 1) / 2) * step for j in range(J)]
        for i in range(S):
            while True:
                src = rng.uniform(0.5, room - 0.5)
                if min(np.linalg.norm(src - m) for m in mics) >= 0.2:
                    break
            for j in range(J):
                k = (u * S + i) * J + j
                geom[k] = np.concatenate([room, src, mics[j]])
                refl[k] = r
    return geom, refl
