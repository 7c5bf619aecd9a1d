"""Oracle sums for the GPU tests in worker processes (numpy's direct
convolution holds the interpreter lock, so threads do not run it in
parallel).  The workers import the oracle themselves; nothing of the GPU
path is imported here."""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

_POOL = None


def workers() -> int:
    """At most 16 (a GPU host's share of cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _one_thread():
    # one compute thread per worker: the pool already fills the cores, and
    # numpy's BLAS (the dot products) would otherwise start its own pool of
    # threads in every worker
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(1)
    except ImportError:
        pass


def pool() -> ProcessPoolExecutor:
    global _POOL
    if _POOL is None:
        _POOL = ProcessPoolExecutor(workers(), mp_context=mp.get_context("spawn"), initializer=_one_thread)
    return _POOL


def pmap(fn, items, timeout: float = 240.0):
    """[fn(a) for a in items] in the worker processes, in order (fn must be a
    module-level function); raises TimeoutError past `timeout` seconds."""
    items = list(items)
    if len(items) <= 1:
        return [fn(a) for a in items]
    return list(pool().map(fn, items, chunksize=1, timeout=timeout))


def mix_mic(args):
    """y_j of eq. (2) for one mic: (sources, the mic's cut RIRs per source,
    the mic's gains per source, output length T) -> float64 [T]."""
    import oracle

    xs, cuts, alpha, T = args
    r = oracle.mix(xs, [[c] for c in cuts], np.asarray(alpha, np.float64).reshape(-1, 1))[0]
    out = np.zeros(T)
    out[: r.size] = r
    return out


def backward_source(args):
    """The adjoint's terms of one source: (x_i, its cut RIRs per mic, its
    gains per mic, g [J][T]) -> (dx_i, [dh_ij], [dalpha_ij])."""
    import oracle

    x, cuts, alpha, g = args
    dx, dh, da = oracle.mix_backward([x], [cuts], np.asarray(alpha, np.float64).reshape(1, -1), g)
    return dx[0], dh[0], da[0]
