"""FFT-size selection table (eq. (6) and the paragraph after it).

For every utterance the schedule kernel evaluates, for each N = 2^m,
    n_b (I + J) c_fft(N) + n_b I J c_mac(N) + I J c_fft(N),   n_b = ceil(Nx / (N - L + 1)),
and keeps the cheapest N.  The paper's cost model counts multiplications
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
    try:
        import torch

        return torch.cuda.get_device_name(0)
    except Exception:  # noqa: BLE001
        return "unknown"


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
    entry = data.get(device_name()) if which == "auto" else data
    if entry is None and which == "auto" and len(data) == 1:
        entry = next(iter(data.values()))
    if not entry:
        return None
    return rsim.tune_table(entry["cost_fft"], entry["cost_mac"])
