"""ctypes binding of librsim.so (include/rsim.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels
behind the C ABI.  PyTorch provides device memory and the current stream.
The library must have been built (``python -m paper_1712_03439_amd.build``);
there is no fallback of any kind when it is missing.

Streams: a call given ``stream`` issues all of its work there, the library's
kernels and this module's own (allocations, fills, small copies), by making
it torch's current stream for the duration of the call; the tensors it
allocates therefore belong to that stream.  Inputs written on another stream
must be ordered before the call by the caller, as for any torch operation.
"""
from __future__ import annotations

import ctypes
import functools
import inspect
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsim.so")

RSIM_OK, RSIM_EINVAL, RSIM_EWORKSPACE, RSIM_EUNSUPPORTED, RSIM_EDEVICE, RSIM_ENOTINIT = range(6)
DEV_NONFINITE, DEV_BADDESC, DEV_BADPLAN = 0x1, 0x2, 0x4

# Every symbol the header declares (checked by the tests).
EXPORTS = (
    "rsim_init", "rsim_strerror", "rsim_version", "rsim_truncate_rir",
    "rsim_ola_workspace_bytes", "rsim_ola_convolve", "rsim_mix_workspace_bytes", "rsim_mix",
    "rsim_simulate", "rsim_mix_backward", "rsim_source_power", "rsim_snr_gains",
    "rsim_device_status", "rsim_rfft", "rsim_irfft", "rsim_image_rir", "rsim_simulate_rooms",
    "rsim_reverb_energy", "rsim_snr_gains_reverb", "rsim_logmel", "rsim_fft_filter_workspace_bytes",
    "rsim_fft_filter", "rsim_simulate_static", "rsim_simulate_logmel_workspace_bytes", "rsim_simulate_logmel",
    "rsim_fft_filter_sizes",
)


class RsimError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = int(code)
        msg = _lib().rsim_strerror(self.code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: rsim status {code} ({msg})")


class RsimBatch(ctypes.Structure):
    _fields_ = [
        ("n_utt", ctypes.c_int32), ("n_mic", ctypes.c_int32), ("max_src", ctypes.c_int32),
        ("max_rir_len0", ctypes.c_int32),
        ("x_len", ctypes.c_int64), ("h_len", ctypes.c_int64), ("y_len", ctypes.c_int64),
        ("n_src", ctypes.c_void_p), ("src_len", ctypes.c_void_p), ("src_off", ctypes.c_void_p),
        ("rir_off", ctypes.c_void_p), ("rir_len0", ctypes.c_void_p), ("rir_len", ctypes.c_void_p),
        ("out_off", ctypes.c_void_p), ("out_stride", ctypes.c_void_p), ("out_len", ctypes.c_void_p),
        ("order", ctypes.c_void_p), ("fft_log2n", ctypes.c_void_p), ("hop", ctypes.c_void_p),
        ("fft_sizes", ctypes.c_int32),
    ]


class RsimTune(ctypes.Structure):
    _fields_ = [("cost_fft", ctypes.c_float * 7), ("cost_mac", ctypes.c_float * 7), ("one_size", ctypes.c_int32),
                ("variant", ctypes.c_int32 * 6)]


_LIB = None
ABI_VERSION = 10200  # rsim_version() of the layouts of RsimBatch and RsimTune and the signatures


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1712_03439_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        bp, tp = ctypes.POINTER(RsimBatch), ctypes.POINTER(RsimTune)
        sig = {
            "rsim_init": ([], i32),
            "rsim_strerror": ([i32], ctypes.c_char_p),
            "rsim_version": ([], i32),
            "rsim_truncate_rir": ([vp, i64, vp, vp, i32, f64, vp, vp, vp], i32),
            "rsim_ola_workspace_bytes": ([i32], sz),
            "rsim_ola_convolve": ([vp, i32, vp, i32, i32, i32, vp, vp, sz, vp], i32),
            "rsim_mix_workspace_bytes": ([bp, tp, i32], sz),
            "rsim_mix": ([bp, vp, vp, vp, vp, vp, sz, tp, i32, vp], i32),
            "rsim_simulate": ([bp, vp, vp, vp, f64, vp, vp, vp, sz, tp, i32, vp], i32),
            "rsim_mix_backward": ([bp, vp, vp, vp, vp, vp, vp, vp, vp, sz, tp, vp], i32),
            "rsim_source_power": ([bp, vp, vp, vp], i32),
            "rsim_snr_gains": ([vp, vp, i32, i32, vp], i32),
            "rsim_device_status": ([vp, vp], i32),
            "rsim_rfft": ([vp, i32, i32, vp, vp], i32),
            "rsim_irfft": ([vp, i32, i32, vp, vp], i32),
            "rsim_image_rir": ([vp, vp, i32, i32, f64, f64, vp, i64, vp, vp, i32, vp], i32),
            "rsim_simulate_rooms": ([bp, vp, vp, vp, vp, i32, f64, f64, vp, f64, vp, vp, vp, sz, tp, i32, vp],
                                    i32),
            "rsim_reverb_energy": ([bp, vp, vp, vp, vp], i32),
            "rsim_snr_gains_reverb": ([vp, vp, i32, i32, vp], i32),
            "rsim_logmel": ([bp, vp, vp, vp, i64, i32, vp], i32),
            "rsim_fft_filter_workspace_bytes": ([bp, i32, i32], sz),
            "rsim_fft_filter": ([bp, vp, vp, vp, vp, i32, i32, vp, sz, vp], i32),
            "rsim_simulate_static": ([bp, vp, vp, vp, f64, vp, vp, tp, vp], i32),
            "rsim_simulate_logmel_workspace_bytes": ([bp, tp], sz),
            "rsim_simulate_logmel": ([bp, vp, vp, vp, f64, vp, vp, vp, i64, vp, sz, tp, i32, vp], i32),
            "rsim_fft_filter_sizes": ([vp, vp, i32, i32, i32, vp], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        # the descriptors mirrored above have the layout of version 1.1
        if lib.rsim_version() // 100 != ABI_VERSION // 100:
            raise ImportError(f"{LIB_PATH} has ABI version {lib.rsim_version()}, this binding needs "
                              f"{ABI_VERSION // 10000}.{ABI_VERSION // 100 % 100}; rebuild it")
        _LIB = lib
    return _LIB


def lib():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


def _check(code: int, where: str) -> None:
    if code != RSIM_OK:
        raise RsimError(code, where)


# ----------------------------------------------------------------- torch glue
def _torch():
    import torch

    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _on_stream(fn):
    """Runs fn with its `stream` argument, when one is given, as torch's
    current stream (see the module docstring)."""
    pos = list(inspect.signature(fn).parameters).index("stream")

    @functools.wraps(fn)
    def wrapped(*args, **kw):
        s = kw.get("stream", args[pos] if len(args) > pos else None)
        if s is None:
            return fn(*args, **kw)
        with _torch().cuda.stream(s):
            return fn(*args, **kw)

    return wrapped


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("rsim: tensors must live in GPU memory")
        if t is not None and not t.is_contiguous():
            raise ValueError("rsim: tensors must be contiguous")


def init() -> None:
    _check(_lib().rsim_init(), "rsim_init")


def device_status(stream=None) -> int:
    """Waits for the work on `stream` (default: the current stream), then
    reads and clears the device status word (RSIM_DEV_* bits)."""
    st = ctypes.c_int32(0)
    _check(_lib().rsim_device_status(_stream(stream), ctypes.byref(st)), "rsim_device_status")
    return int(st.value)


@_on_stream
def truncate_rir(h, off, len0, eta_db: float, n_c=None, length=None, stream=None):
    """RIR tail cut-off (eqs. 7-9) on the GPU.  Returns (n_c, len) int32 tensors."""
    torch = _torch()
    _require_cuda(h, off, len0)
    n = int(len0.numel())
    if n_c is None:
        n_c = torch.empty(n, dtype=torch.int32, device=h.device)
    if length is None:
        length = torch.empty(n, dtype=torch.int32, device=h.device)
    _check(_lib().rsim_truncate_rir(_ptr(h), int(h.numel()), _ptr(off), _ptr(len0), n, float(eta_db),
                                    _ptr(n_c), _ptr(length), _stream(stream)), "rsim_truncate_rir")
    return n_c, length


@_on_stream
def ola_convolve(x, h, fft_n: int, hop: int = 0, stream=None):
    """Overlap-add FFT convolution of one signal with one RIR (eq. 6)."""
    torch = _torch()
    _require_cuda(x, h)
    nx, nh = int(x.numel()), int(h.numel())
    y = torch.empty(max(nx + nh - 1, 0), dtype=torch.float32, device=x.device)
    ws_bytes = int(_lib().rsim_ola_workspace_bytes(int(fft_n)))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=x.device)
    _check(_lib().rsim_ola_convolve(_ptr(x), nx, _ptr(h), nh, int(fft_n), int(hop), _ptr(y), _ptr(ws),
                                    ws_bytes, _stream(stream)), "rsim_ola_convolve")
    return y


@_on_stream
def rfft(x, n: int, stream=None):
    """Forward real FFT of len(x)/n signals of length n (FFT engine test entry)."""
    torch = _torch()
    _require_cuda(x)
    count = int(x.numel()) // n
    spec = torch.empty(count * (n // 2 + 1) * 2, dtype=torch.float32, device=x.device)
    _check(_lib().rsim_rfft(_ptr(x), int(n), count, _ptr(spec), _stream(stream)), "rsim_rfft")
    return spec.view(count, n // 2 + 1, 2)


@_on_stream
def irfft(spec, n: int, stream=None):
    torch = _torch()
    _require_cuda(spec)
    count = int(spec.numel()) // ((n // 2 + 1) * 2)
    x = torch.empty(count * n, dtype=torch.float32, device=spec.device)
    _check(_lib().rsim_irfft(_ptr(spec), int(n), count, _ptr(x), _stream(stream)), "rsim_irfft")
    return x.view(count, n)


@_on_stream
def image_rir(geom, refl, off, length, h, max_len: int, order: int = 8, fs: float = 16000.0,
              c0: float = 343.0, stream=None):
    """Image-method RIRs (eq. 1) written into h at off[r] .. off[r] + length[r].

    geom: float64 [n_rir, 9] (room Lx Ly Lz, source xyz, mic xyz, metres),
    refl: float64 [n_rir], off: int64 [n_rir], length: int32 [n_rir], all on the
    GPU; max_len (host) >= every length."""
    torch = _torch()
    _require_cuda(geom, refl, off, length, h)
    if geom.dtype != torch.float64 or refl.dtype != torch.float64 or h.dtype != torch.float32:
        raise ValueError("rsim.image_rir: geom and refl are float64, h is float32")
    n = int(refl.numel())
    if geom.numel() != 9 * n or off.numel() != n or length.numel() != n:
        raise ValueError("rsim.image_rir: geom [n, 9], refl, off and length [n]")
    _check(_lib().rsim_image_rir(_ptr(geom), _ptr(refl), n, int(order), float(fs), float(c0), _ptr(h),
                                 int(h.numel()), _ptr(off), _ptr(length), int(max_len), _stream(stream)),
           "rsim_image_rir")
    return h


@_on_stream
def simulate_rooms(db: DeviceBatch, geom, refl, alpha, eta_db: float, order: int = 8, fs: float = 16000.0,
                   c0: float = 343.0, y=None, ws=None, tune: Optional[RsimTune] = None, use_graph: bool = False,
                   stream=None):
    """Image-method RIRs (eq. 1) into db.h for every RIR slot (geom float64
    [U*S*J, 9], refl float64 [U*S*J] on the GPU), then cut + mix, as one call
    (one graph with use_graph)."""
    _require_cuda(geom, refl, alpha)
    if y is None:
        y = db.new_output()
    if ws is None:
        ws = db.workspace(tune)
    s = db.struct()
    _check(_lib().rsim_simulate_rooms(ctypes.byref(s), _ptr(db.x), _ptr(db.h), _ptr(geom), _ptr(refl), int(order),
                                      float(fs), float(c0), _ptr(alpha), float(eta_db), _ptr(db.rir_len), _ptr(y),
                                      _ptr(ws), int(ws.numel()), ctypes.byref(tune) if tune else None,
                                      int(bool(use_graph)), _stream(stream)),
           "rsim_simulate_rooms")
    return y


@_on_stream
def reverb_energy(db: DeviceBatch, x=None, h=None, stream=None):
    """Energies of the reverberant sources at the mics, float64 [U*S*J] on the
    GPU (rsim_reverb_energy; call after the cut)."""
    torch = _torch()
    e = torch.empty(db.U * db.S * db.J, dtype=torch.float64, device=db.device)
    s = db.struct()
    _check(_lib().rsim_reverb_energy(ctypes.byref(s), _ptr(db.x if x is None else x), _ptr(db.h if h is None else h),
                                     _ptr(e), _stream(stream)), "rsim_reverb_energy")
    return e


def snr_gains_reverb(energy: np.ndarray, snr_db: Sequence[float]) -> np.ndarray:
    """Host gain rule of the reverberant-at-mic reading (rsim_snr_gains_reverb):
    energy [I, J] -> alpha [I, J]."""
    E = np.ascontiguousarray(energy, np.float64)
    I, J = E.shape
    s = np.ascontiguousarray(snr_db, np.float64)
    a = np.zeros(I * J, np.float32)
    _check(_lib().rsim_snr_gains_reverb(E.ctypes.data, s.ctypes.data, I, J, a.ctypes.data), "rsim_snr_gains_reverb")
    return a.reshape(I, J)


def batch_gains_reverb(db: DeviceBatch, snr_db: np.ndarray, energy: np.ndarray) -> np.ndarray:
    """alpha [U*S*J] (float32, host) of the reverberant-at-mic rule from the
    energies (reverb_energy, copied to the host)."""
    U, S, J = db.U, db.S, db.J
    a = np.zeros(U * S * J, np.float32)
    n_src = db.host.n_src
    E = np.asarray(energy, np.float64).reshape(U, S, J)
    for u in range(U):
        I = int(n_src[u])
        if I:
            a[u * S * J:(u * S + I) * J] = snr_gains_reverb(E[u, :I], snr_db[u * S:u * S + I]).reshape(-1)
    return a


MEL_WIN, MEL_HOP, MEL_BANDS = 512, 160, 128


def mel_frames(T) -> np.ndarray:
    """Whole 512-sample frames every 160 samples in T samples."""
    T = np.asarray(T, np.int64)
    return np.where(T >= MEL_WIN, 1 + (T - MEL_WIN) // MEL_HOP, 0)


@_on_stream
def logmel(db: DeviceBatch, y, stream=None):
    """128 log-Mel features per frame of every (utterance, mic) output
    (rsim_logmel; call after the mix).  Returns (feat, off, cap): frame t of
    (u, j) is feat[off[u] + (j cap[u] + t) * 128 : + 128] for
    t < mel_frames(out_len[u])."""
    torch = _torch()
    _require_cuda(y)
    cap = mel_frames(db.host.out_stride)
    sizes = cap * db.J * MEL_BANDS
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    total = int(sizes.sum())
    feat = torch.empty(max(total, 1), dtype=torch.float32, device=db.device)
    # the device copy of the offsets stays referenced by db until the next call
    db.mel_off = torch.from_numpy(off).to(db.device)
    s = db.struct()
    _check(_lib().rsim_logmel(ctypes.byref(s), _ptr(y), _ptr(feat), _ptr(db.mel_off), int(feat.numel()),
                              int(cap.max()) if cap.size else 0, _stream(stream)), "rsim_logmel")
    return feat, off, cap


def feature_layout(db: DeviceBatch):
    """(off, cap, total) of the features of every (utterance, mic): frame t
    of (u, j) at off[u] + (j cap[u] + t) * 128, cap[u] the frames of
    out_stride[u] samples."""
    cap = mel_frames(db.host.out_stride)
    sizes = cap * db.J * MEL_BANDS
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return off, cap, int(sizes.sum())


@_on_stream
def simulate_logmel(db: DeviceBatch, alpha, eta_db: float, feat=None, ws=None, tune: Optional[RsimTune] = None,
                    use_graph: bool = False, stream=None):
    """Cut + mix of one epoch with the log-Mel front end fused into the mix
    (rsim_simulate_logmel): the features of every mic output, no y.  Returns
    (feat, off, cap) as logmel()."""
    torch = _torch()
    _require_cuda(alpha)
    off, cap, total = feature_layout(db)
    if feat is None:
        feat = torch.empty(max(total, 1), dtype=torch.float32, device=db.device)
    db.mel_off = torch.from_numpy(off).to(db.device)
    s = db.struct()
    if ws is None:
        n = int(_lib().rsim_simulate_logmel_workspace_bytes(ctypes.byref(s), ctypes.byref(tune) if tune else None))
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=db.device)
    _check(_lib().rsim_simulate_logmel(ctypes.byref(s), _ptr(db.x), _ptr(db.h), _ptr(alpha), float(eta_db),
                                       _ptr(db.rir_len), _ptr(feat), _ptr(db.mel_off), int(feat.numel()),
                                       _ptr(ws), int(ws.numel()), ctypes.byref(tune) if tune else None,
                                       int(bool(use_graph)), _stream(stream)), "rsim_simulate_logmel")
    return feat, off, cap


def fft_filter_log2n(db: DeviceBatch) -> np.ndarray:
    """Per utterance, the transform size (log2) of eqs. 4-5 that the library
    assigns (rsim_fft_filter_sizes): it holds the whole convolution with the
    uncut RIRs, a bound for any cut."""
    b = db.host
    if not db.U:
        return np.zeros(0, np.int64)
    src = np.ascontiguousarray(b.src_len, np.int32)
    l0 = np.ascontiguousarray(b.rir_len0, np.int32)
    out = np.zeros(db.U, np.int32)
    _check(_lib().rsim_fft_filter_sizes(src.ctypes.data, l0.ctypes.data, db.U, db.S, db.J, out.ctypes.data),
           "rsim_fft_filter_sizes")
    return out.astype(np.int64)


@_on_stream
def fft_filter(db: DeviceBatch, alpha, y=None, chunk: int = 16, stream=None):
    """Eqs. 4-5: full-length FFT filtering and mixing of the batch (after the
    cut), for comparison with the overlap-add path.  Utterances are grouped
    by their transform size (fft_filter_log2n); each group is one call."""
    torch = _torch()
    _require_cuda(alpha)
    if y is None:
        y = db.new_output()
    l2s = fft_filter_log2n(db)
    S, J = db.S, db.J
    empty = np.nonzero(l2s == 0)[0]
    if empty.size:  # no samples or no taps: no output
        db.out_len[torch.as_tensor(empty, device=db.device)] = 0
    for l2 in np.unique(l2s[l2s > 0]):
        idx = np.nonzero(l2s == l2)[0]
        sub = db if idx.size == db.U else db.select(idx)
        if sub is db:
            a = alpha
        else:
            u = torch.as_tensor(idx, device=db.device)
            rows = ((u[:, None] * S + torch.arange(S, device=db.device)[None, :])[:, :, None] * J
                    + torch.arange(J, device=db.device)[None, None, :]).reshape(-1)
            a = alpha[rows].contiguous()
        s = sub.struct()
        n = int(_lib().rsim_fft_filter_workspace_bytes(ctypes.byref(s), int(l2), int(chunk)))
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=db.device)
        _check(_lib().rsim_fft_filter(ctypes.byref(s), _ptr(db.x), _ptr(db.h), _ptr(a), _ptr(y), int(l2), int(chunk),
                                      _ptr(ws), int(ws.numel()), _stream(stream)), "rsim_fft_filter")
        if sub is not db:
            db.out_len[torch.as_tensor(idx, device=db.device)] = sub.out_len
    return y


def snr_gains(p_dry: Sequence[float], snr_db: Sequence[float], n_mic: int) -> np.ndarray:
    """Host SNR gain rule of the library (rsim_snr_gains)."""
    I = len(p_dry)
    p = np.ascontiguousarray(p_dry, np.float64)
    s = np.ascontiguousarray(snr_db, np.float64)
    a = np.zeros(I * n_mic, np.float32)
    _check(_lib().rsim_snr_gains(p.ctypes.data, s.ctypes.data, I, int(n_mic), a.ctypes.data),
           "rsim_snr_gains")
    return a.reshape(I, n_mic)


def tune_table(cost_fft: Sequence[float], cost_mac: Sequence[float], one_size: bool = False,
               variant: Optional[Sequence[int]] = None) -> RsimTune:
    """An FFT-size cost table (rsim_tune); one_size picks one N for the whole
    batch; variant[f] (0 = default, 1..4) is the kernel variant of family f."""
    t = RsimTune()
    for k in range(7):
        t.cost_fft[k] = float(cost_fft[k])
        t.cost_mac[k] = float(cost_mac[k])
    t.one_size = int(bool(one_size))
    for f in range(6):
        t.variant[f] = int(variant[f]) if variant is not None else 0
    return t


class DeviceBatch:
    """A batch descriptor with its per-utterance arrays resident on the GPU.

    Built from any object with the fields of synth.Batch (n_utt, n_mic, max_src,
    n_src, src_len, src_off, rir_off, rir_len0, out_off, out_stride, x, h,
    y_len).  x, h are uploaded once; y is allocated here.
    """

    def __init__(self, b, device="cuda", order: Optional[np.ndarray] = None,
                 fft_log2n: Optional[np.ndarray] = None, hop: Optional[np.ndarray] = None,
                 upload_data: bool = True):
        torch = _torch()
        self.host = b
        self.U, self.J, self.S = int(b.n_utt), int(b.n_mic), int(b.max_src)
        dev = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)  # noqa: E731
        self.n_src = t(b.n_src, torch.int32)
        self.src_len = t(b.src_len, torch.int32)
        self.src_off = t(b.src_off, torch.int64)
        self.rir_off = t(b.rir_off, torch.int64)
        self.rir_len0 = t(b.rir_len0, torch.int32)
        self.rir_len = self.rir_len0.clone()
        self.n_c = torch.empty_like(self.rir_len0)
        self.out_off = t(b.out_off, torch.int64)
        self.out_stride = t(b.out_stride, torch.int32)
        self.out_len = torch.zeros(self.U, dtype=torch.int32, device=dev)
        self.order = None if order is None else t(order, torch.int32)
        self.fft_log2n = None if fft_log2n is None else t(fft_log2n, torch.int32)
        self.fft_sizes = size_bits(fft_log2n)
        self.hop = None if hop is None else t(hop, torch.int32)
        self.x = t(b.x, torch.float32) if upload_data else None
        self.h = t(b.h, torch.float32) if upload_data else None
        self.x_len = int(np.asarray(b.x).size)
        self.h_len = int(np.asarray(b.h).size)
        self.y_len = int(b.y_len)
        self.max_rir_len0 = int(np.max(b.rir_len0)) if np.asarray(b.rir_len0).size else 0
        self.device = dev

    def select(self, idx) -> "DeviceBatch":
        """The utterances idx (host ints, distinct) as a batch of their own:
        their descriptor rows (cut lengths included) gathered on the device, in
        the parent's processing order; the sources, RIRs and output layout are
        the parent's (x, h shared, outputs land where the parent's would)."""
        torch = _torch()
        dev = self.device
        u = torch.as_tensor(np.asarray(idx, np.int64), device=dev)
        S, J = self.S, self.J
        slots = (u[:, None] * S + torch.arange(S, device=dev)[None, :]).reshape(-1)
        rirs = (slots[:, None] * J + torch.arange(J, device=dev)[None, :]).reshape(-1)
        sub = object.__new__(DeviceBatch)
        sub.host = None
        sub.U, sub.J, sub.S = int(u.numel()), J, S
        sub.n_src = self.n_src[u].contiguous()
        sub.src_len = self.src_len[u].contiguous()
        sub.src_off = self.src_off[slots].contiguous()
        sub.rir_off = self.rir_off[rirs].contiguous()
        sub.rir_len0 = self.rir_len0[rirs].contiguous()
        sub.rir_len = self.rir_len[rirs].contiguous()
        sub.n_c = self.n_c[rirs].contiguous()
        sub.out_off = self.out_off[u].contiguous()
        sub.out_stride = self.out_stride[u].contiguous()
        sub.out_len = torch.zeros(sub.U, dtype=torch.int32, device=dev)
        sub.order = None
        if self.order is not None:
            # the parent's processing order restricted to idx
            rank = torch.empty_like(self.order)
            rank[self.order.long()] = torch.arange(self.U, dtype=rank.dtype, device=dev)
            sub.order = torch.argsort(rank[u], stable=True).to(torch.int32)
        sub.fft_log2n = None if self.fft_log2n is None else self.fft_log2n[u].contiguous()
        sub.fft_sizes = self.fft_sizes
        sub.hop = None if self.hop is None else self.hop[u].contiguous()
        sub.x, sub.h = self.x, self.h
        sub.x_len, sub.h_len, sub.y_len = self.x_len, self.h_len, self.y_len
        sub.max_rir_len0 = int(self.rir_len0[rirs].max().item()) if rirs.numel() else 0
        sub.device = dev
        return sub

    def struct(self, rir_len=None, out_len=None) -> RsimBatch:
        """The C descriptor of this batch; rir_len / out_len replace the
        batch's own cut-length and output-length arrays when given."""
        s = RsimBatch()
        s.n_utt, s.n_mic, s.max_src, s.max_rir_len0 = self.U, self.J, self.S, self.max_rir_len0
        s.x_len, s.h_len, s.y_len = self.x_len, self.h_len, self.y_len
        s.n_src, s.src_len, s.src_off = _ptr(self.n_src), _ptr(self.src_len), _ptr(self.src_off)
        s.rir_off, s.rir_len0 = _ptr(self.rir_off), _ptr(self.rir_len0)
        s.rir_len = _ptr(self.rir_len if rir_len is None else rir_len)
        s.out_off, s.out_stride = _ptr(self.out_off), _ptr(self.out_stride)
        s.out_len = _ptr(self.out_len if out_len is None else out_len)
        s.order, s.fft_log2n, s.hop = _ptr(self.order), _ptr(self.fft_log2n), _ptr(self.hop)
        s.fft_sizes = self.fft_sizes if self.fft_log2n is not None else 0
        return s

    def workspace_bytes(self, tune: Optional[RsimTune] = None, backward: bool = False) -> int:
        s = self.struct()
        return int(_lib().rsim_mix_workspace_bytes(ctypes.byref(s), ctypes.byref(tune) if tune else None,
                                                   int(backward)))

    def workspace(self, tune: Optional[RsimTune] = None, backward: bool = False):
        torch = _torch()
        n = self.workspace_bytes(tune, backward)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)

    def new_output(self):
        torch = _torch()
        return torch.empty(max(self.y_len, 1), dtype=torch.float32, device=self.device)


def size_bits(fft_log2n) -> int:
    """The descriptor's fft_sizes word for forced sizes given on the host: bit
    m for every log2 size m in 9..15 that occurs (0 when none is given, which
    leaves every size provided for)."""
    if fft_log2n is None:
        return 0
    bits = 0
    for m in np.unique(np.asarray(fft_log2n)):
        if 9 <= int(m) <= 15:
            bits |= 1 << int(m)
    return bits


def _one(db: DeviceBatch, u: int) -> RsimBatch:
    """Descriptor of utterance u alone (views into db's device arrays)."""
    S, J = db.S, db.J
    s = db.struct()
    s.n_utt = 1
    s.n_src += 4 * u
    s.src_len += 4 * u
    s.src_off += 8 * u * S
    s.rir_off += 8 * u * S * J
    s.rir_len0 += 4 * u * S * J
    s.rir_len += 4 * u * S * J
    s.out_off += 8 * u
    s.out_stride += 4 * u
    s.out_len += 4 * u
    s.order = None
    if db.fft_log2n is not None:
        s.fft_log2n += 4 * u
    if db.hop is not None:
        s.hop += 4 * u
    return s


def single_workspace_bytes(db: DeviceBatch, tune: Optional[RsimTune] = None) -> int:
    s = _one(db, 0)
    return max(1, int(_lib().rsim_mix_workspace_bytes(ctypes.byref(s), ctypes.byref(tune) if tune else None, 0)))


@_on_stream
def simulate_one(db: DeviceBatch, u: int, alpha, eta_db: float, y, ws, tune: Optional[RsimTune] = None,
                 stream=None):
    """Cut + mix of utterance u alone (the plain per-utterance path)."""
    s = _one(db, u)
    a = _ptr(alpha) + 4 * u * db.S * db.J
    _check(_lib().rsim_simulate(ctypes.byref(s), _ptr(db.x), _ptr(db.h), a, float(eta_db), s.rir_len,
                                _ptr(y), _ptr(ws), int(ws.numel()), ctypes.byref(tune) if tune else None,
                                0, _stream(stream)), "rsim_simulate")


@_on_stream
def truncate_batch(db: DeviceBatch, eta_db: float, h=None, stream=None):
    """Cut every RIR slot of the batch; writes db.n_c and db.rir_len."""
    _check(_lib().rsim_truncate_rir(_ptr(db.h if h is None else h), db.h_len, _ptr(db.rir_off),
                                    _ptr(db.rir_len0), int(db.rir_len0.numel()), float(eta_db),
                                    _ptr(db.n_c), _ptr(db.rir_len), _stream(stream)),
           "rsim_truncate_rir")


@_on_stream
def mix(db: DeviceBatch, alpha, y=None, ws=None, tune: Optional[RsimTune] = None, use_graph: bool = False,
        x=None, h=None, stream=None):
    """Eq. (2) for the whole batch with the current db.rir_len (call truncate_batch first)."""
    _require_cuda(alpha)
    if y is None:
        y = db.new_output()
    if ws is None:
        ws = db.workspace(tune)
    s = db.struct()
    _check(_lib().rsim_mix(ctypes.byref(s), _ptr(db.x if x is None else x), _ptr(db.h if h is None else h),
                           _ptr(alpha), _ptr(y), _ptr(ws), int(ws.numel()),
                           ctypes.byref(tune) if tune else None, int(bool(use_graph)), _stream(stream)),
           "rsim_mix")
    return y


@_on_stream
def simulate(db: DeviceBatch, alpha, eta_db: float, y=None, ws=None, tune: Optional[RsimTune] = None,
             use_graph: bool = False, x=None, h=None, stream=None):
    """Cut + mix of one epoch (rsim_simulate): writes db.rir_len and y."""
    _require_cuda(alpha)
    if y is None:
        y = db.new_output()
    if ws is None:
        ws = db.workspace(tune)
    s = db.struct()
    _check(_lib().rsim_simulate(ctypes.byref(s), _ptr(db.x if x is None else x),
                                _ptr(db.h if h is None else h), _ptr(alpha), float(eta_db),
                                _ptr(db.rir_len), _ptr(y), _ptr(ws), int(ws.numel()),
                                ctypes.byref(tune) if tune else None, int(bool(use_graph)),
                                _stream(stream)), "rsim_simulate")
    return y


STATIC_SCRATCH_BYTES = 128 << 20  # RSIM_STATIC_SCRATCH_BYTES


@_on_stream
def simulate_static(db: DeviceBatch, alpha, eta_db: float, y, tune: Optional[RsimTune] = None, stream=None):
    """Cut + mix of one epoch without any allocation by the library or here
    (rsim_simulate_static): y (and db's arrays) are the caller's, the
    workspace is the library's static scratch on this device.  Calls on one
    device must not overlap."""
    _require_cuda(alpha, y)
    s = db.struct()
    _check(_lib().rsim_simulate_static(ctypes.byref(s), _ptr(db.x), _ptr(db.h), _ptr(alpha), float(eta_db),
                                       _ptr(db.rir_len), _ptr(y), ctypes.byref(tune) if tune else None,
                                       _stream(stream)), "rsim_simulate_static")
    return y


@_on_stream
def mix_backward(db: DeviceBatch, alpha, grad_y, x=None, h=None, ws=None, tune: Optional[RsimTune] = None,
                 need_alpha: bool = True, stream=None, rir_len=None, out_len=None):
    """Adjoint of `mix` (rsim_mix_backward): (grad_x, grad_h, grad_alpha) in the
    layouts of x, h and alpha, for the cut lengths rir_len (default: the
    current db.rir_len).  grad_h is zero beyond each cut length; grad_alpha is
    None unless need_alpha.  The call's schedule writes the output lengths
    into out_len (default: db.out_len)."""
    torch = _torch()
    x = db.x if x is None else x
    h = db.h if h is None else h
    _require_cuda(alpha, grad_y, x, h)
    if ws is None:
        ws = db.workspace(tune, backward=True)
    # zeros: parts of the packed arrays that belong to no utterance keep a zero gradient
    gx = torch.zeros(max(db.x_len, 1), dtype=torch.float32, device=db.device)
    gh = torch.zeros(max(db.h_len, 1), dtype=torch.float32, device=db.device)
    ga = torch.zeros(max(db.U * db.S * db.J, 1), dtype=torch.float32, device=db.device) if need_alpha else None
    s = db.struct(rir_len=rir_len, out_len=out_len)
    _check(_lib().rsim_mix_backward(ctypes.byref(s), _ptr(x), _ptr(h), _ptr(alpha), _ptr(grad_y), _ptr(gx),
                                    _ptr(gh), _ptr(ga), _ptr(ws), int(ws.numel()),
                                    ctypes.byref(tune) if tune else None, _stream(stream)),
           "rsim_mix_backward")
    return gx[: db.x_len], gh[: db.h_len], (ga[: db.U * db.S * db.J] if need_alpha else None)


class _MixFunction:
    """Built lazily so that importing this module does not import torch."""

    fn = None

    @classmethod
    def get(cls):
        if cls.fn is None:
            torch = _torch()

            class MixFunction(torch.autograd.Function):
                """y = mix(x, h, alpha) of eq. (2) with the hand-written adjoint.

                x, h: packed float32 sources and RIRs (db's layouts); alpha:
                [U*S*J] gains.  The cut lengths db.rir_len at the forward call
                are constants (no gradient flows through the cut index); the
                backward uses a copy of them taken by the forward, so a later
                cut of the same batch does not change this graph's adjoint.
                Gradients reach whatever alpha was computed from only if alpha
                is a torch expression of it (the host gain rule of batch_gains
                returns numpy and ends the graph there)."""

                @staticmethod
                def forward(ctx, x, h, alpha, db, tune):
                    # zeros: the padding of each mic beyond T_u is part of y too
                    y = torch.zeros(max(db.y_len, 1), dtype=torch.float32, device=db.device)
                    rir_len = db.rir_len.clone()
                    mix(db, alpha, y=y, tune=tune, x=x, h=h)
                    ctx.save_for_backward(x, h, alpha, rir_len)
                    ctx.db, ctx.tune = db, tune
                    return y[: db.y_len]

                @staticmethod
                def backward(ctx, gy):
                    x, h, alpha, rir_len = ctx.saved_tensors
                    gy = gy.contiguous()
                    out_len = torch.empty_like(ctx.db.out_len)
                    gx, gh, ga = mix_backward(ctx.db, alpha, gy, x=x, h=h, tune=ctx.tune,
                                              need_alpha=ctx.needs_input_grad[2], rir_len=rir_len,
                                              out_len=out_len)
                    return (gx if ctx.needs_input_grad[0] else None,
                            gh if ctx.needs_input_grad[1] else None,
                            ga, None, None)

            cls.fn = MixFunction
        return cls.fn


def mix_autograd(db: DeviceBatch, x, h, alpha, tune: Optional[RsimTune] = None):
    """Differentiable eq. (2): returns y (layout of db's outputs, length
    db.y_len); backward runs rsim_mix_backward."""
    return _MixFunction.get().apply(x, h, alpha, db, tune)


@_on_stream
def source_power(db: DeviceBatch, x=None, stream=None):
    torch = _torch()
    p = torch.empty(db.U * db.S, dtype=torch.float64, device=db.device)
    s = db.struct()
    _check(_lib().rsim_source_power(ctypes.byref(s), _ptr(db.x if x is None else x), _ptr(p),
                                    _stream(stream)), "rsim_source_power")
    return p


def batch_gains(db: DeviceBatch, snr_db: np.ndarray, power: Optional[np.ndarray] = None) -> np.ndarray:
    """alpha [U*S*J] (float32, host) from the dry powers (device kernel) and the
    per-source SNRs, through the library's gain rule."""
    if power is None:
        power = source_power(db).cpu().numpy()
    U, S, J = db.U, db.S, db.J
    a = np.zeros(U * S * J, np.float32)
    n_src = db.host.n_src
    for u in range(U):
        I = int(n_src[u])
        if I:
            a[u * S * J:(u * S + I) * J] = snr_gains(power[u * S:u * S + I],
                                                     snr_db[u * S:u * S + I], J).reshape(-1)
    return a
