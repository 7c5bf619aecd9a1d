"""FFT-size selection table (eq. (6) and the paragraph after it).

For every utterance the schedule kernel evaluates, for each N = 2^m,
    n_b (I + J) c_fft(N) + n_b I J c_mac(N) + I J c_fft(N),   n_b = ceil(Nx / (N - L + 1)),
and keeps the cheapest N, or (one_size, the default) the one N with the
smallest cost summed over the batch.  The paper's cost model counts multiplications
(eq. (6)); the kernels do I + J transforms per block (source spectra are shared
across mics and the sum over sources is taken in the spectral domain), so the
built-in model uses that count with 2.5 N log2 N per real FFT.  `tune()`
times the filter-and-mix kernels of every size and kernel variant on a batch
(eager launches on one stream) and scales the model per size to the measured
times; it also picks each kernel family's variant (the work split of
rsim_tune.variant) and, by timing the whole batch both ways, whether one size
serves the batch or each utterance takes its own.  Tables are stored keyed by
the device name.
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


# Kernel families (workgroup of 32 << f threads) of each log2 N, and the
# kernel variants (rsim_tune.variant codes) each family has.
FAMILY = {9: 0, 10: 1, 11: 1, 12: 2, 13: 3, 14: 4, 15: 5}
VARIANTS = {0: (1, 2, 3, 4), 1: (1, 2, 3, 4), 2: (1, 2, 3, 4), 3: (1, 2, 3, 4), 4: (1, 2, 3, 4), 5: (4,)}
DEFAULT_VARIANT = 2
SAME_WITHIN = 0.02  # relative time difference taken as timing noise


def utt_cost(nx: int, I: int, J: int, lmax: int, m: int, cost_fft, cost_mac) -> Optional[float]:
    """The schedule's cost of one utterance at N = 2^m with the default hop
    N - lmax + 1, or None if N cannot serve it (or the size is disabled)."""
    c = cost_fft[m - 9]
    N = 1 << m
    if not c > 0 or N < lmax:
        return None
    B = N - lmax + 1
    nb = (nx + B - 1) // B
    return nb * ((I + J) * c + I * J * cost_mac[m - 9]) + I * J * c


def batch_log2n(shapes, cost_fft, cost_mac) -> int:
    """The one size the schedule picks for a batch of (nx, I, J, lmax): the
    smallest summed cost among the sizes every utterance can use, else 0."""
    tot = {}
    for m in LOG2N:
        cs = [utt_cost(nx, I, J, lmax, m, cost_fft, cost_mac) for nx, I, J, lmax in shapes]
        if all(c is not None for c in cs):
            tot[m] = sum(cs)
    return min(tot, key=tot.get) if tot else 0


def utterance_log2n(nx: int, I: int, J: int, lmax: int, cost_fft, cost_mac) -> int:
    """The size the schedule picks for one utterance on its own (0 if none)."""
    best, l2 = None, 0
    for m in LOG2N:
        c = utt_cost(nx, I, J, lmax, m, cost_fft, cost_mac)
        if c is not None and (best is None or c < best):
            best, l2 = c, m
    return l2


def batch_shapes(db) -> List[Tuple[int, int, int, int, int]]:
    """(u, Nx, I, J, longest kept RIR) of every utterance with work, from the
    batch's current (cut) RIR lengths."""
    import numpy as np

    n_src = db.n_src.cpu().numpy()
    nx = db.src_len.cpu().numpy()
    L = db.rir_len.cpu().numpy().reshape(db.U, db.S * db.J)
    out = []
    for u in range(db.U):
        I = int(n_src[u])
        lmax = int(L[u, : I * db.J].max()) if I else 0
        if I and nx[u] > 0 and lmax > 0:
            out.append((u, int(nx[u]), I, db.J, lmax))
    return out


def measure(db, alpha, sizes=LOG2N, reps: int = 3, min_probe: int = 64, stream=None,
            verbose: bool = False) -> dict:
    """Time the filter-and-mix kernels of every FFT size and kernel variant on
    the caller's batch (already cut: rsim.truncate_batch).

    The probe of size N is the batch's utterances whose longest kept RIR is at
    most N/2 (so the hop N - L + 1 is at least half the block), all forced to
    N with the default hop; a size with fewer than min_probe such utterances
    (fewer than the batch's own count if smaller) is not measured.  Each
    (size, variant) runs once untimed and then reps times eagerly on one
    stream; the mean time per call is kept, with the built-in model's cost of
    the same probe, so that the fit can scale the model per size."""
    import numpy as np
    import torch

    from . import rsim

    shapes = batch_shapes(db)
    if not shapes:
        raise ValueError("the batch has no utterance with work to time")
    mf, mm = model_costs()
    dev = db.device
    if stream is None:
        stream = torch.cuda.Stream(device=dev)
    # Every tensor the timed calls read (the probe's descriptor, its forced
    # sizes and gains, the output and workspace) is made on the timing
    # stream itself, after it has waited for the caller's work, so the
    # library never reads a tensor that another stream is still writing.
    stream.wait_stream(torch.cuda.current_stream(dev))
    S, J = db.S, db.J
    out = {"utterances": len(shapes), "reps": reps, "sizes": {}}
    with torch.cuda.stream(stream):
        y = db.new_output()
        for m in sizes:
            N = 1 << m
            rows = [sh for sh in shapes if sh[4] <= N // 2]
            if not rows or len(rows) < min(min_probe, len(shapes)):
                continue
            idx = [sh[0] for sh in rows]
            probe = db.select(idx)
            probe.fft_log2n = torch.full((probe.U,), m, dtype=torch.int32, device=dev)
            probe.fft_sizes = 1 << m
            probe.hop = None
            u = torch.as_tensor(np.asarray(idx, np.int64), device=dev)
            slot = (u[:, None] * S + torch.arange(S, device=dev)[None, :]).reshape(-1)
            a = alpha[(slot[:, None] * J + torch.arange(J, device=dev)[None, :]).reshape(-1)].contiguous()
            model = float(sum(utt_cost(nx, I, Jm, lmax, m, mf, mm) for _, nx, I, Jm, lmax in rows))
            f = FAMILY[m]
            times = {}
            for v in VARIANTS[f]:
                var = [0] * 6
                var[f] = v
                t = rsim.tune_table(mf, mm, True, var)
                ws = probe.workspace(t)
                rsim.mix(probe, a, y=y, ws=ws, tune=t, stream=stream)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    rsim.mix(probe, a, y=y, ws=ws, tune=t, stream=stream)
                e1.record(stream)
                e1.synchronize()
                times[v] = e0.elapsed_time(e1) / reps
                del ws
            out["sizes"][m] = {"utterances": len(idx), "model": model, "ms": times}
            if verbose:
                print(f"N={N}: {len(idx)} utterances, " +
                      ", ".join(f"variant {v}: {ms:.3f} ms" for v, ms in times.items()), flush=True)
    stream.synchronize()
    if rsim.device_status():
        raise RuntimeError("a timing run set the device status word")
    if not out["sizes"]:
        raise ValueError("no FFT size had enough utterances to time")
    return out


def fit(measured: dict) -> dict:
    """A tune-table entry from measure()'s times (or the "measured" field of
    a stored entry).

    Per family, the variant with the smallest time relative to the best
    variant, summed over the family's measured sizes; the library default
    is kept unless that sum is smaller by more than SAME_WITHIN per size.  Per measured size m, k(m) = the time with that variant / the
    model's cost of the probe; a size not measured takes k of the nearest
    measured size (the larger on a tie).  The costs are the built-in model's
    scaled by k (ns per model unit), so the schedule's summed cost of a batch
    approximates its time at each size and the one-size rule picks the size
    that ran fastest."""
    mf, mm = model_costs()
    sizes = {}
    for m, rec in measured["sizes"].items():
        sizes[int(m)] = {"utterances": int(rec["utterances"]), "model": float(rec["model"]),
                         "ms": {int(v): float(t) for v, t in rec["ms"].items()}}
    if not sizes:
        raise ValueError("no measured size")
    variant = [0] * 6
    for f in range(6):
        ms = [m for m in sizes if FAMILY[m] == f]
        common = [v for v in VARIANTS[f] if all(v in sizes[m]["ms"] for m in ms)]
        if not ms or not common:
            continue
        score = {v: sum(sizes[m]["ms"][v] / min(sizes[m]["ms"].values()) for m in ms) for v in common}
        best = min(score, key=lambda v: (score[v], v != DEFAULT_VARIANT))
        # the default stays unless another variant is faster by more than the
        # timing noise (SAME_WITHIN per size)
        if DEFAULT_VARIANT in score and score[DEFAULT_VARIANT] <= score[best] + SAME_WITHIN * len(ms):
            best = DEFAULT_VARIANT
        variant[f] = best
    k = {}
    for m, rec in sizes.items():
        v = variant[FAMILY[m]]
        t = rec["ms"][v] if v else min(rec["ms"].values())
        k[m] = t * 1e6 / rec["model"]
    cost_fft, cost_mac = [], []
    for m in LOG2N:
        km = k[m] if m in k else k[min(k, key=lambda q: (abs(q - m), -q))]
        cost_fft.append(km * mf[m - 9])
        cost_mac.append(km * mm[m - 9])
    return {"cost_fft": cost_fft, "cost_mac": cost_mac, "one_size": True, "variant": variant, "unit": "ns",
            "measured": {"sizes": {str(m): {"utterances": r["utterances"], "model": r["model"],
                                            "ms": {str(v): t for v, t in sorted(r["ms"].items())}}
                                   for m, r in sorted(sizes.items())}}}


def choose_policy(ms_one_size: float, ms_per_utterance: float) -> bool:
    """one_size for the table: one FFT size per batch unless choosing per
    utterance ran faster by more than the timing noise."""
    return not ms_per_utterance < ms_one_size * (1.0 - SAME_WITHIN)


def measure_policy(db, alpha, entry: dict, reps: int = 3, stream=None) -> dict:
    """Time the whole batch with the fitted table under both size policies
    (one size per batch, a size per utterance): eager launches on one stream,
    one untimed call then reps timed ones each."""
    import torch

    from . import rsim

    dev = db.device
    if stream is None:
        stream = torch.cuda.Stream(device=dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    out = {}
    with torch.cuda.stream(stream):
        y = db.new_output()
        for key, one in (("one_size", True), ("per_utterance", False)):
            t = entry_to_tune(dict(entry, one_size=one))
            ws = db.workspace(t)
            rsim.mix(db, alpha, y=y, ws=ws, tune=t, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                rsim.mix(db, alpha, y=y, ws=ws, tune=t, stream=stream)
            e1.record(stream)
            e1.synchronize()
            out[key] = e0.elapsed_time(e1) / reps
            del ws
    stream.synchronize()
    return out


def keep_sizes_from_batch_size(entry: dict, shapes) -> int:
    """With one size per batch: disable (cost 0) every size below the one the
    schedule picks for `shapes` ((nx, I, J, lmax) of the tuned batch) and
    return that size's log2 (0, and nothing changed, when no size serves every
    utterance or the policy is a size per utterance).  A batch that one size
    serves is served by every larger one, so no batch loses its plan; the
    kernel families of the disabled sizes are then neither sized nor launched
    (an empty family still costs a launch in the epoch's graph)."""
    if not entry.get("one_size", True):
        return 0
    l2 = batch_log2n(shapes, entry["cost_fft"], entry["cost_mac"])
    if l2:
        for m in LOG2N:
            if m < l2:
                entry["cost_fft"][m - 9] = 0.0
                entry["cost_mac"][m - 9] = 0.0
        entry["sizes_from"] = l2
    return l2


def entry_to_tune(entry: dict):
    from . import rsim

    return rsim.tune_table(entry["cost_fft"], entry["cost_mac"], entry.get("one_size", True),
                           entry.get("variant"))


def tune(db, alpha, save: Optional[str] = None, policy: bool = True, prune: bool = True, **kw):
    """measure() then fit(), then (policy) the size policy by measure_policy(),
    then (prune, with one size per batch) keep_sizes_from_batch_size() on this
    batch: the RsimTune for this GPU and the table entry.  With save, the
    entry is merged into that JSON file under device_name()."""
    entry = fit(measure(db, alpha, **kw))
    if policy:
        pm = measure_policy(db, alpha, entry, reps=kw.get("reps", 3), stream=kw.get("stream"))
        entry["one_size"] = choose_policy(pm["one_size"], pm["per_utterance"])
        entry["policy_ms"] = pm
    if prune:
        keep_sizes_from_batch_size(entry, [s[1:] for s in batch_shapes(db)])
    if save:
        data = {}
        if os.path.exists(save):
            with open(save) as f:
                data = json.load(f)
        data[device_name()] = entry
        with open(save, "w") as f:
            json.dump(data, f, indent=1)
    return entry_to_tune(entry), entry


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
    return entry_to_tune(entry)


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="measure the FFT-size and kernel-variant table on this GPU "
                                             "with a synthetic batched workload")
    ap.add_argument("--out", default=TABLE, help="JSON file to merge this device's entry into")
    ap.add_argument("--n-utt", type=int, default=2048)
    ap.add_argument("--eta", type=float, default=20.0)
    args = ap.parse_args()
    import torch

    import synth

    from . import rsim

    torch.cuda.set_device(0)
    rsim.init()
    b = synth.make_config2(n_utt=args.n_utt)
    db = rsim.DeviceBatch(b)
    alpha = torch.from_numpy(rsim.batch_gains(db, b.snr_db)).cuda()
    rsim.truncate_batch(db, args.eta)
    _, e = tune(db, alpha, save=args.out, verbose=True)
    print(json.dumps({device_name(): e}))
