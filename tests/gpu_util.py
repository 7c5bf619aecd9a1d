"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def max_rel_err(got, ref):
    """max |got - ref| / max |ref| (0/0 counts as 0)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    peak = float(np.max(np.abs(ref))) if ref.size else 0.0
    err = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    if peak == 0.0:
        return err
    return err / peak


def host_workers() -> int:
    """Threads for oracle sums: numpy's direct convolution releases the GIL.
    At most 16 (a GPU host's share of cores)."""
    return max(1, min(16, os.cpu_count() or 1))


def pmap(fn, items):
    """[fn(a) for a in items], evaluated on host threads, in order."""
    items = list(items)
    if len(items) <= 1:
        return [fn(a) for a in items]
    with ThreadPoolExecutor(host_workers()) as ex:
        return list(ex.map(fn, items))


TOL = 1e-5  # max-abs error relative to the output peak, per (utterance, mic)
