"""FFT-size selection table (eq. (6) and the paragraph after it).

For every utterance the schedule kernel evaluates, for each N = 2^m,
    n_b (I + J) c_fft(N) + n_b I J c_mac(N) + I J c_fft(N),   n_b = ceil(Nx / (N - L + 1)),
and keeps the cheapest N, or (one_size, the default) the one N with the
smallest cost summed over the batch.  The paper's cost model counts multiplications
(eq. (6)); the kernels do I + J transforms per block (source spectra are shared
across mics and the sum over sources is taken in the spectral domain), so the
built-in model uses that count with 2.5 N log2 N per real FFT.  `tune()`
replaces the model by measured times of the kernels themselves and stores the
table next to this file, keyed by the device name.
"""
from __future__ import annotations

import json
import math
import os
from typing import List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tune_table.json")
LOG2N = list(range(9, 16))


def model_costs() -> Tuple[List[float], List[float]]:
    f = [2.5 * (1 << m) * m for m in LOG2N]
    c = [8.0 * ((1 << m) / 2 + 1) for m in LOG2N]
    return f, c


def eq6_cost(nx: float, nh: float, I: float, J: float, N: int) -> float:
    """The paper's multiplication count of OLA filtering (eq. 6), with the
    block count read as ceil(Nx / (N - Nh + 1))."""
    nb = math.ceil(nx / (N - nh + 1))
    return I * J * (nb * (4 * N * math.log2(N) + 2 * N) + 2 * N * math.log2(N))


def td_cost(nx: float, nh: float, I: float, J: float) -> float:
    """Direct time-domain convolution (eq. 3)."""
    return I * J * nx * nh


def fft_cost(nx: float, nh: float, I: float, J: float, N: int) -> float:
    """Full-length FFT filtering (eq. 5)."""
    return I * J * (6 * N * math.log2(N) + 2 * N)


def costs(tune) -> Tuple[List[float], List[float]]:
    if tune is None:
        return model_costs()
    return list(tune.cost_fft), list(tune.cost_mac)


def device_name() -> str:
    """Key of this GPU in the table: ISA name and compute-unit count."""
    try:
        import torch

        p = torch.cuda.get_device_properties(torch.cuda.current_device())
        arch = getattr(p, "gcnArchName", "") or p.name
        return f"{arch.split(':')[0]}-{p.multi_processor_count}cu"
    except Exception:  # noqa: BLE001
        return "unknown"


class _Probe:
    """Descriptor of U identical utterances (I sources of Nx samples, J mics,
    RIRs of L taps) with packed, non-overlapping offsets."""

    def __init__(self, U: int, I: int, J: int, nx: int, L: int):
        import numpy as np

        self.n_utt, self.n_mic, self.max_src = U, J, I
        self.n_src = np.full(U, I, np.int32)
        self.src_len = np.full(U, nx, np.int32)
        self.src_off = (np.arange(U * I, dtype=np.int64) * nx).reshape(U, I)
        self.rir_len0 = np.full(U * I * J, L, np.int32)
        self.rir_off = np.arange(U * I * J, dtype=np.int64) * L
        T = nx + L - 1
        self.out_stride = np.full(U, T, np.int32)
        self.out_off = np.arange(U, dtype=np.int64) * (J * T)
        self.y_len = U * J * T
        self.x = np.zeros(0, np.float32)
        self.h = np.zeros(0, np.float32)
        self.x_len, self.h_len = U * I * nx, U * I * J * L


def tune(sizes=LOG2N, blocks: int = 8, reps: int = 3, save: bool = True, verbose: bool = False):
    """Measure c_fft(N) and c_mac(N) (ns per transform and per spectral
    product, whole-GPU throughput) with the mix kernels themselves.

    For each N two probes of identical utterances run with N forced and hop
    N/2 (so every probe has `blocks` blocks): (I, J) = (1, 1) and (3, 2).  The
    time per utterance is modelled as blocks ((I + J) + I J k) c_f + I J c_f,
    with c_m = k c_f and k the ratio of the flop counts 8 (N/2 + 1) and
    2.5 N log2 N; c_f is the mean of the two probes' estimates."""
    if True:  # switched off until the crash below is understood
        raise RuntimeError("the measuring tuner is switched off: one of its runs ended in a host "
                           "segmentation fault whose cause is not yet found; the built-in cost "
                           "model is used instead")
    import numpy as np
    import torch

    from . import rsim

    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.Stream(device=dev)
    cost_f, cost_m = [0.0] * 7, [0.0] * 7
    mf, mm = model_costs()
    for m in sizes:
        N = 1 << m
        hop, L = N // 2, N // 2
        nx = blocks * hop
        U = max(2048, (1 << 24) // nx)
        k = mm[m - 9] / mf[m - 9]
        ratios = []
        for I, J in ((1, 1), (3, 2)):
            pr = _Probe(U, I, J, nx, L)
            db = rsim.DeviceBatch(pr, device=dev, fft_log2n=np.full(U, m, np.int32),
                                  hop=np.full(U, hop, np.int32), upload_data=False)
            g = torch.Generator(device=dev)
            g.manual_seed(1234 + m)
            db.x = torch.randn(pr.x_len, device=dev, generator=g)
            db.h = torch.randn(pr.h_len, device=dev, generator=g)
            db.x_len, db.h_len = pr.x_len, pr.h_len
            alpha = torch.ones(U * I * J, device=dev)
            y = db.new_output()
            ws = db.workspace(None)
            with torch.cuda.stream(stream):
                rsim.mix(db, alpha, y=y, ws=ws)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    rsim.mix(db, alpha, y=y, ws=ws)
                e1.record(stream)
            e1.synchronize()
            t_utt = e0.elapsed_time(e1) / reps * 1e6 / U  # ns per utterance
            units = blocks * ((I + J) + I * J * k) + I * J
            ratios.append(t_utt / units)
            del db, y, ws, alpha
        cf_ = float(np.mean(ratios))
        cost_f[m - 9], cost_m[m - 9] = cf_, cf_ * k
        if verbose:
            print(f"N={N}: c_fft={cf_:.2f} ns (probe ratios {ratios[0]:.2f}, {ratios[1]:.2f})", flush=True)
    entry = {"cost_fft": cost_f, "cost_mac": cost_m, "unit": "ns"}
    if save:
        data = {}
        if os.path.exists(TABLE):
            with open(TABLE) as f:
                data = json.load(f)
        data[device_name()] = entry
        with open(TABLE, "w") as f:
            json.dump(data, f, indent=1)
    return rsim.tune_table(cost_f, cost_m)


def load(which: str = "auto"):
    """An RsimTune from the stored table ('auto': this device's entry if any;
    'model': the built-in model, i.e. None), or from a JSON path."""
    from . import rsim

    if which == "model":
        return None
    path = TABLE if which == "auto" else which
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    entry = data if "cost_fft" in data else data.get(device_name())
    if not entry:
        return None
    return rsim.tune_table(entry["cost_fft"], entry["cost_mac"], entry.get("one_size", True))


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="measure the FFT-size cost table on this GPU")
    ap.add_argument("--out", default=TABLE, help="JSON file to merge this device's entry into")
    args = ap.parse_args()
    import torch

    from . import rsim

    torch.cuda.set_device(0)
    rsim.init()
    TABLE = args.out
    t = tune(save=True, verbose=True)
    print(json.dumps({device_name(): {"cost_fft": list(t.cost_fft), "cost_mac": list(t.cost_mac)}}))
