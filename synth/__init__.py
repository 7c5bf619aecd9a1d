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
    from the `epoch` stream (a fresh room every epoch)."""
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
    pools = {"speech": speech_like(drng, pool_len), "white": white_noise(drng, pool_len),
             "pink": pink_noise(drng, pool_len)}
    sources = []
    for u in range(n_utt):
        n = int(lengths[u])
        off = drng.integers(0, pool_len - n + 1, int(n_src[u]))
        s = [pools["speech"][off[0]:off[0] + n]]
        for i in range(1, int(n_src[u])):
            kind = "white" if kinds[u, i] == 0 else "pink"
            s.append(pools[kind][off[i]:off[i] + n])
        sources.append(s)
    return attach_rooms(cid, epoch, sources, n_mic, t60_range, max_taps)


def attach_rooms(cid: int, epoch: int, sources, n_mic: int, t60_range: tuple,
                 max_taps: Optional[int] = None) -> Batch:
    """Draw a fresh room (RIRs, T60s, SNRs) for each utterance of `sources`."""
    rrng = rng_for(cid, 10_000 + epoch)
    rirs, snrs, t60s = [], [], []
    for s in sources:
        I = len(s)
        t60 = rrng.uniform(t60_range[0], t60_range[1])
        L0 = int(math.ceil(t60 * FS))
        if max_taps is not None:
            L0 = min(L0, max_taps)
        rows = []
        for i in range(I):
            rows.append([rir(rrng, L0, t60, int(rrng.integers(20, 401))) for _ in range(n_mic)])
        rirs.append(rows)
        snrs.append([0.0] + list(rrng.uniform(0.0, 30.0, I - 1)))
        t60s.append([[t60] * n_mic for _ in range(I)])
    return pack(sources, rirs, snrs, n_mic, t60s)


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
