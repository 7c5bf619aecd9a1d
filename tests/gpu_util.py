"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
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


TOL = 1e-5  # max-abs error relative to the output peak, per (utterance, mic)
