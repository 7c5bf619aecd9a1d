"""Plain, slow, obviously correct FP64 oracle of the room-simulator hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or run
this module: it exists so that the GPU results can be checked against the
paper's definitions.  It shares no code, tables or helpers with the GPU path.

What it computes, with the passage each function follows:

* cut_rir      -- the RIR tail cut-off, Sec. 2.3, eqs. (7)-(9), with the
                  precision rule below (the paper states no precision).
* dry_power,
  snr_gains    -- the gains alpha_ij of the mixing model, eq. (2).  The paper
                  gives no formula; the rule used is the dry-signal SNR rule
                  (target unscaled, noise i scaled so that the dry-power ratio
                  equals the requested SNR, same gain at every microphone).
* convolve     -- the linear convolution h * x of eq. (2), computed directly in
                  the time domain (the work counted by eq. (3)).  The method's
                  overlap-add FFT filtering (eq. (6)) reaches this same result
                  up to rounding, so the oracle is the definition itself.
* mix, mix_at  -- eq. (2): y_j[n] = sum_i alpha_ij (h_ij * x_i)[n].
* mix_backward -- the adjoint of eq. (2) with respect to x, h and alpha.
* reverb_energy,
  snr_gains_reverb -- the other reading of eq. (2)'s per-(i, j) gains: the
                  SNR measured at each mic on the reverberant signals.

Precision rule for the cut (float32, round to nearest even, no flush of
subnormals): q[n] = fl32(h[n]^2); P = max q; s = fl32(10^(-eta/10)) computed in
binary64 and rounded once (eta = +inf gives s = 0); p_th = fl32(P s);
n_c = the last index with q[n] >= p_th (samples equal to the threshold are
kept); the kept length is min(n_c + 2, L0) because eq. (9) keeps indices
0..n_c+1.  A non-finite q (NaN or overflow) keeps the whole RIR and raises the
flag.  An empty RIR has n_c = -1 and L = 0.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np


def _assert_no_ftz() -> None:
    tiny = np.float32(1e-45)  # the smallest float32 subnormal
    if not (tiny > 0 and np.float32(tiny * np.float32(1.0)) > 0):
        raise RuntimeError("float32 subnormals are flushed; the cut rule needs them")


_assert_no_ftz()


def cut_scale(eta_db: float) -> np.float32:
    """s = 10^(-eta/10) in binary64, rounded once to float32 (Sec. 2.3, eq. 7)."""
    eta = float(eta_db)
    if math.isnan(eta) or eta < 0.0:
        raise ValueError("eta must be >= 0 dB (or +inf for no cut)")
    if math.isinf(eta):
        return np.float32(0.0)
    return np.float32(10.0 ** (-eta / 10.0))


def cut_rir(h: np.ndarray, eta_db: float) -> Tuple[int, int, bool]:
    """Cut index n_c, kept length L and non-finite flag of one RIR.

    Sec. 2.3: p_th = max h^2 * 10^(-eta/10) (eq. 7); n_c is the smallest m such
    that every h^2[n] with n > m lies below p_th (eq. 8), i.e. the last index
    whose power reaches p_th; the cut RIR keeps n = 0..n_c+1 (eq. 9).
    """
    h32 = np.asarray(h, dtype=np.float32)
    L0 = int(h32.size)
    if L0 == 0:
        return -1, 0, False
    q = h32 * h32                       # float32 products, one rounding each
    if not np.all(np.isfinite(q)):
        return L0 - 1, L0, True
    P = q.max()
    p_th = np.float32(P * cut_scale(eta_db))
    above = np.nonzero(q >= p_th)[0]
    n_c = int(above[-1])                # exists: q[argmax] = P >= p_th
    return n_c, min(n_c + 2, L0), False


def dry_power(x: np.ndarray) -> float:
    """Mean power of a dry source, in FP64."""
    x64 = np.asarray(x, dtype=np.float64)
    return float(np.mean(x64 * x64)) if x64.size else 0.0


def snr_gains(p_dry: Sequence[float], snr_db: Sequence[float], n_mic: int) -> np.ndarray:
    """alpha [I, J] of eq. (2) under the dry-signal SNR rule.

    alpha_0j = 1 (the target, i = 0, is not scaled).  For a noise source i >= 1
    with dry power P_i and requested SNR s_i dB: alpha_ij = sqrt(P_0 / (P_i 10^(s_i/10))),
    so that 10 log10(P_0 / (alpha_ij^2 P_i)) = s_i.  A silent noise (P_i = 0)
    gets alpha = 0.
    """
    I = len(p_dry)
    a = np.zeros((I, n_mic), np.float64)
    if I == 0:
        return a
    a[0, :] = 1.0
    p0 = float(p_dry[0])
    for i in range(1, I):
        pi = float(p_dry[i])
        a[i, :] = 0.0 if pi <= 0.0 else math.sqrt(p0 / (pi * 10.0 ** (float(snr_db[i]) / 10.0)))
    return a


def reverb_energy(x: np.ndarray, h: np.ndarray) -> float:
    """Energy of a reverberant source at a mic, E = sum_n ((h * x)[n])^2, in
    FP64 from the direct convolution (h is the cut RIR)."""
    c = convolve(x, h)
    return float(np.dot(c, c))


def snr_gains_reverb(energy: np.ndarray, snr_db: Sequence[float]) -> np.ndarray:
    """alpha [I, J] of eq. (2) under the reverberant-at-mic SNR rule.

    The paper names alpha_ij per source and mic but gives no rule; this is
    the rule that measures the SNR at each mic on the reverberant signals:
    alpha_0j = 1 and, for a noise source i >= 1 with energy E_ij = ||h_ij * x_i||^2
    at mic j and requested SNR s_i dB, alpha_ij = sqrt(E_0j / (E_ij 10^(s_i/10))),
    so that 10 log10(E_0j / (alpha_ij^2 E_ij)) = s_i at every mic.  A silent
    noise (E_ij = 0) or a silent target at that mic (E_0j = 0) gives 0.
    """
    E = np.asarray(energy, np.float64)
    I, J = E.shape if E.size else (0, 0)
    a = np.zeros((I, J), np.float64)
    if I == 0:
        return a
    a[0, :] = 1.0
    for i in range(1, I):
        for j in range(J):
            e0, ei = float(E[0, j]), float(E[i, j])
            a[i, j] = 0.0 if ei <= 0.0 or e0 <= 0.0 else math.sqrt(e0 / (ei * 10.0 ** (float(snr_db[i]) / 10.0)))
    return a


def convolve(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Linear convolution (h * x)[n] = sum_k h[k] x[n-k], length Nx + L - 1.

    numpy.convolve evaluates the sum directly in the time domain (no FFT).
    An empty signal or an empty RIR (a RIR of length 0 has no taps) gives an
    empty result: it contributes nothing to eq. (2)."""
    x64 = np.asarray(x, dtype=np.float64)
    h64 = np.asarray(h, dtype=np.float64)
    if x64.size == 0 or h64.size == 0:
        return np.zeros(0, np.float64)
    return np.convolve(x64, h64)


def _cut_rirs(rirs, lengths):
    return [[np.asarray(rirs[i][j], np.float32)[: int(lengths[i][j])] for j in range(len(rirs[i]))]
            for i in range(len(rirs))]


def out_length(nx: int, lengths: Sequence[Sequence[int]]) -> int:
    """Common output length of one utterance: Nx + max_ij L_ij - 1 (0 if empty)."""
    lmax = max((int(l) for row in lengths for l in row), default=0)
    return nx + lmax - 1 if (nx > 0 and lmax > 0) else 0


def mix(sources: Sequence[np.ndarray], rirs: Sequence[Sequence[np.ndarray]],
        alpha: np.ndarray) -> np.ndarray:
    """Eq. (2): y_j[n] = sum_i alpha_ij (h_ij * x_i)[n], every mic zero-padded
    to the common length Nx + max L - 1.  `rirs` are the (already cut) RIRs."""
    I = len(sources)
    J = len(rirs[0]) if I else 0
    nx = len(sources[0]) if I else 0
    T = out_length(nx, [[len(r) for r in row] for row in rirs])
    y = np.zeros((J, T), np.float64)
    for j in range(J):
        for i in range(I):
            c = convolve(sources[i], rirs[i][j])
            y[j, : c.size] += float(alpha[i][j]) * c
    return y


def mix_at(sources: Sequence[np.ndarray], rirs: Sequence[Sequence[np.ndarray]],
           alpha: np.ndarray, j: int, idx: Sequence[int]) -> np.ndarray:
    """y_j[n] of eq. (2) at the sample indices `idx` only, each as its own sum."""
    out = np.zeros(len(idx), np.float64)
    for t, n in enumerate(idx):
        acc = 0.0
        for i in range(len(sources)):
            x = np.asarray(sources[i], np.float64)
            h = np.asarray(rirs[i][j], np.float64)
            k_lo = max(0, n - (x.size - 1))
            k_hi = min(h.size - 1, n)
            if k_hi >= k_lo:
                k = np.arange(k_lo, k_hi + 1)
                acc += float(alpha[i][j]) * float(np.dot(h[k], x[n - k]))
        out[t] = acc
    return out


def mix_backward(sources: Sequence[np.ndarray], rirs: Sequence[Sequence[np.ndarray]],
                 alpha: np.ndarray, grad_y: np.ndarray):
    """Adjoint of eq. (2).  With g_j = dLoss/dy_j (length T of `mix`):

    dx_i[n]     = sum_j alpha_ij sum_k h_ij[k] g_j[n+k]      (n < Nx)
    dh_ij[k]    = alpha_ij sum_n x_i[n] g_j[n+k]             (k < L_ij)
    dalpha_ij   = sum_n g_j[n] (h_ij * x_i)[n]

    Correlations are evaluated directly (numpy.correlate, no FFT).  No gradient
    flows through the cut index, which is piecewise constant in h.
    """
    I = len(sources)
    J = len(rirs[0]) if I else 0
    nx = len(sources[0]) if I else 0
    g = np.asarray(grad_y, np.float64)
    dx = np.zeros((I, nx), np.float64)
    dh = [[np.zeros(len(rirs[i][j]), np.float64) for j in range(J)] for i in range(I)]
    da = np.zeros((I, J), np.float64)
    for i in range(I):
        x = np.asarray(sources[i], np.float64)
        for j in range(J):
            h = np.asarray(rirs[i][j], np.float64)
            L = h.size
            if L == 0 or nx == 0:
                continue
            seg = g[j, : nx + L - 1]
            a = float(alpha[i][j])
            dx[i] += a * np.correlate(seg, h, mode="valid")[:nx]
            r = np.correlate(seg, x, mode="valid")[:L]
            dh[i][j] = a * r
            da[i, j] = float(np.dot(seg, convolve(x, h)))
    return dx, dh, da


def mix_backward_at(sources: Sequence[np.ndarray], rirs: Sequence[Sequence[np.ndarray]],
                    alpha: np.ndarray, grad_y: np.ndarray, i: int, j: int,
                    x_idx: Sequence[int], h_idx: Sequence[int]):
    """Samples of the adjoint of eq. (2), each as its own direct sum:
    dx_i[n] for n in x_idx (summed over every mic) and dh_ij[k] for k in h_idx,
    plus dalpha_ij in full."""
    g = np.asarray(grad_y, np.float64)
    J = len(rirs[0])
    x = np.asarray(sources[i], np.float64)
    nx = x.size
    dx = np.zeros(len(x_idx), np.float64)
    for t, n in enumerate(x_idx):
        acc = 0.0
        for jj in range(J):
            h = np.asarray(rirs[i][jj], np.float64)
            L = h.size
            acc += float(alpha[i][jj]) * float(np.dot(h, g[jj, n: n + L])) if L else 0.0
        dx[t] = acc
    h = np.asarray(rirs[i][j], np.float64)
    L = h.size
    a = float(alpha[i][j])
    dh = np.array([a * float(np.dot(x, g[j, k: k + nx])) if k < L else 0.0 for k in h_idx])
    da = float(np.dot(g[j, : nx + L - 1], convolve(x, h))) if L and nx else 0.0
    return dx, dh, da


def simulate(sources: Sequence[np.ndarray], rirs: Sequence[Sequence[np.ndarray]],
             snr_db: Sequence[float], eta_db: float, alpha: np.ndarray = None):
    """One utterance end to end: cut every RIR (eqs. 7-9), compute the gains,
    then mix (eq. 2).  Returns (y, n_c [I][J], L [I][J], alpha)."""
    I = len(sources)
    J = len(rirs[0]) if I else 0
    ncs = [[0] * J for _ in range(I)]
    Ls = [[0] * J for _ in range(I)]
    for i in range(I):
        for j in range(J):
            n_c, L, _ = cut_rir(rirs[i][j], eta_db)
            ncs[i][j], Ls[i][j] = n_c, L
    if alpha is None:
        alpha = snr_gains([dry_power(s) for s in sources], snr_db, J)
    cut = _cut_rirs(rirs, Ls)
    return mix(sources, cut, alpha), ncs, Ls, alpha
