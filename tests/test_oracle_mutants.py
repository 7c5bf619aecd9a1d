"""Planted mistakes in the oracle, each of which its pins must catch (CPU).

Every mutant below edits one expression in the source of one oracle
function: a dropped term or factor, a flipped comparison or sign, an index
off by one, a transposed operand, a swapped reading of the paper.  The edited
function is loaded in place of the original (wherever a module holds it), the
pins of that oracle module run, and at least one of them must fail.  An edit
that no longer matches the oracle's source fails as well, so the list follows
the oracle when it changes.  The pins themselves run unedited in their own
modules; this file only checks that they are strong enough.
"""
import inspect
import sys
import textwrap

import pytest

from oracle import image_oracle, logmel_oracle, rsim_oracle
from tests import test_image_oracle, test_logmel_oracle, test_oracle_pins

PINS = {rsim_oracle: test_oracle_pins, image_oracle: test_image_oracle, logmel_oracle: test_logmel_oracle}

# (module, function, text in its source, replacement, the mistake)
MUTANTS = [
    # the cut, eqs. 7-9
    (rsim_oracle, "cut_scale", "10.0 ** (-eta / 10.0)", "10.0 ** (-eta / 20.0)", "threshold in amplitude dB"),
    (rsim_oracle, "cut_scale", "return np.float32(0.0)", "return np.float32(1e-30)", "eta = inf still cuts"),
    (rsim_oracle, "cut_rir", "q >= p_th", "q > p_th", "a tap at the threshold is dropped"),
    (rsim_oracle, "cut_rir", "min(n_c + 2, L0)", "min(n_c + 1, L0)", "eq. 9 keeps one tap less"),
    (rsim_oracle, "cut_rir", "above[-1]", "above[0]", "first crossing instead of the last"),
    (rsim_oracle, "cut_rir", "q = h32 * h32", "q = np.abs(h32)", "amplitude instead of power"),
    (rsim_oracle, "cut_rir", "return L0 - 1, L0, True", "return L0 - 1, L0, False", "non-finite flag lost"),
    (rsim_oracle, "cut_rir", "return -1, 0, False", "return 0, 0, False", "empty RIR cut index"),
    # the gains of eq. 2
    (rsim_oracle, "snr_gains", "math.sqrt(p0 / (pi * 10.0 ** (float(snr_db[i]) / 10.0)))",
     "p0 / (pi * 10.0 ** (float(snr_db[i]) / 10.0))", "power ratio used as a gain"),
    (rsim_oracle, "snr_gains", "10.0 ** (float(snr_db[i]) / 10.0)", "10.0 ** (-float(snr_db[i]) / 10.0)",
     "SNR sign flipped"),
    (rsim_oracle, "snr_gains", "0.0 if pi <= 0.0", "1.0 if pi <= 0.0", "silent noise left at gain 1"),
    (rsim_oracle, "dry_power", "np.mean(x64 * x64)", "np.mean(np.abs(x64))", "mean magnitude as power"),
    (rsim_oracle, "reverb_energy", "np.dot(c, c)", "np.sum(np.abs(c))", "sum of magnitudes as energy"),
    (rsim_oracle, "snr_gains_reverb", "math.sqrt(e0 / (ei *", "math.sqrt(ei / (e0 *", "energies swapped"),
    (rsim_oracle, "snr_gains_reverb", "e0, ei = float(E[0, j])", "e0, ei = float(E[0, 0])",
     "mic 0's target energy at every mic"),
    # the convolution and mixing of eq. 2
    (rsim_oracle, "convolve", "np.convolve(x64, h64)", "np.convolve(x64, h64[::-1])", "correlation"),
    (rsim_oracle, "convolve", "np.convolve(x64, h64)", "np.convolve(x64, h64)[:-1]", "last sample dropped"),
    (rsim_oracle, "convolve", "return np.zeros(0, np.float64)", "return np.zeros(x64.size, np.float64)",
     "an empty RIR gives zeros of the source length"),
    (rsim_oracle, "out_length", "nx + lmax - 1", "nx + lmax", "output one sample long"),
    (rsim_oracle, "mix", "float(alpha[i][j])", "float(alpha[j][i])", "gain matrix transposed"),
    (rsim_oracle, "mix", "y[j, : c.size] +=", "y[j, : c.size] =", "sources overwrite instead of summing"),
    (rsim_oracle, "mix_at", "k_hi = min(h.size - 1, n)", "k_hi = min(h.size - 2, n)", "last tap dropped"),
    (rsim_oracle, "mix_at", "float(alpha[i][j]) * float(np.dot(h[k], x[n - k]))",
     "float(np.dot(h[k], x[n - k]))", "gain dropped"),
    (rsim_oracle, "simulate", "_cut_rirs(rirs, Ls)", "_cut_rirs(rirs, ncs)", "cut index used as length"),
    # the adjoint
    (rsim_oracle, "mix_backward", 'np.correlate(seg, h, mode="valid")', 'np.convolve(seg, h, mode="valid")',
     "dx by convolution instead of correlation"),
    (rsim_oracle, "mix_backward", "dh[i][j] = a * r", "dh[i][j] = r", "gain dropped from dh"),
    (rsim_oracle, "mix_backward", "float(np.dot(seg, convolve(x, h)))", "a * float(np.dot(seg, convolve(x, h)))",
     "gain multiplied into dalpha"),
    (rsim_oracle, "mix_backward", 'np.correlate(seg, x, mode="valid")[:L]',
     'np.correlate(seg[1:], x, mode="valid")[:L]', "dh shifted by one tap"),
    (rsim_oracle, "mix_backward", "dx[i] += a *", "dx[i] = a *", "dx keeps the last mic only"),
    (rsim_oracle, "mix_backward_at", "g[jj, n: n + L]", "g[jj, n + 1: n + 1 + L]", "dx shifted by one sample"),
    (rsim_oracle, "mix_backward_at", "a * float(np.dot(x, g[j, k: k + nx]))", "float(np.dot(x, g[j, k: k + nx]))",
     "gain dropped from dh"),
    # the image method, eq. 1
    (image_oracle, "image_taps", "idx * L[ax] + (L[ax] - s[ax])", "idx * L[ax] - s[ax]", "odd images misplaced"),
    (image_oracle, "image_taps", "g = (ga + gb + gc)", "g = (ga + gb)", "reflections on one axis not counted"),
    (image_oracle, "image_taps", "np.ceil((d * float(fs)) / float(c0))", "np.floor((d * float(fs)) / float(c0))",
     "tap rounded down"),
    (image_oracle, "image_taps", "(d * float(fs)) / float(c0)", "(d * float(c0)) / float(fs)",
     "delay with fs and c0 swapped"),
    (image_oracle, "image_taps", "amp = pw[g] / d", "amp = pw[g] / (d * d)", "1/d^2 attenuation"),
    (image_oracle, "image_taps", "pw[k] = p\n        p = p * float(refl)", "p = p * float(refl)\n        pw[k] = p",
     "one reflection too many"),
    (image_oracle, "image_taps", "np.where(idx % 2 == 0,", "np.where(idx % 2 == 1,", "even and odd images swapped"),
    (image_oracle, "image_taps", "0.005 <= s[ax]", "0.0 <= s[ax]", "source on the wall accepted"),
    (image_oracle, "image_rir", "np.rint(amp", "np.floor(amp", "amplitudes truncated, not rounded"),
    (image_oracle, "image_rir", "keep = n < length", "keep = n < length - 1", "last tap dropped"),
    # the log-Mel front end (Sec. 3)
    (logmel_oracle, "hz_to_mel", "2595.0 * np.log10", "1127.0 * np.log10", "natural-log constant on log10"),
    (logmel_oracle, "filterbank", "(FS / WIN)", "(FS / 2 / WIN)", "bin frequencies halved"),
    (logmel_oracle, "filterbank", "lo, c, hi = edges[b], edges[b + 1], edges[b + 2]",
     "lo, c, hi = edges[b], edges[b + 1], edges[b + 1] + (edges[b + 1] - edges[b])", "triangles symmetric in Hz"),
    (logmel_oracle, "n_frames", "1 + (int(T) - WIN) // HOP", "(int(T) - WIN) // HOP", "one frame short"),
    (logmel_oracle, "n_frames", "if T >= WIN else 0", "if T > WIN else 0", "a signal of one window has no frame"),
    (logmel_oracle, "power_spectra", "np.arange(WIN) / WIN)", "np.arange(WIN) / (WIN - 1))", "symmetric Hann"),
    (logmel_oracle, "power_spectra", "X.real ** 2 + X.imag ** 2", "np.abs(X)", "magnitude instead of power"),
    (logmel_oracle, "power_spectra", "np.arange(F)[:, None] * HOP", "np.arange(F)[:, None] * (HOP + 1)",
     "hop off by one"),
    (logmel_oracle, "mel_energies", "power_spectra(y) @", "np.sqrt(power_spectra(y)) @", "magnitudes into the bands"),
    (logmel_oracle, "logmel", "np.log(mel_energies(y) + FLOOR)", "np.log(np.maximum(mel_energies(y), FLOOR))",
     "floor as a clamp, not an offset"),
    (logmel_oracle, "logmel", "np.log(mel_energies(y) + FLOOR)", "np.log10(mel_energies(y) + FLOOR)", "log10"),
    (logmel_oracle, "stack", "feat[starts + i]", "feat[starts + i * step]", "stacked frames spaced by the step"),
]


def _edited(mod, fname, old, new):
    src = textwrap.dedent(inspect.getsource(getattr(mod, fname)))
    assert src.count(old) == 1, f"{mod.__name__}.{fname}: the text to edit occurs {src.count(old)} times"
    ns = {}
    exec(compile(src.replace(old, new), f"<{fname}, edited>", "exec"), vars(mod), ns)
    return ns[fname]


def _pin_cases(module):
    """(name, function, keyword arguments) of every pin in `module`, with its
    parametrize marks expanded."""
    for name, fn in vars(module).items():
        if not (name.startswith("test_") and inspect.isfunction(fn)):
            continue
        combos = [{}]
        for m in getattr(fn, "pytestmark", []):
            if m.name != "parametrize":
                continue
            names = m.args[0]
            names = [s.strip() for s in names.split(",")] if isinstance(names, str) else list(names)
            rows = []
            for c in combos:
                for v in m.args[1]:
                    v = getattr(v, "values", v)
                    rows.append({**c, **dict(zip(names, (v,) if len(names) == 1 else v))})
            combos = rows
        params = set(inspect.signature(fn).parameters)
        for c in combos:
            assert set(c) == params, f"{name} takes fixtures; the mutant runner passes parameters only"
            yield name, fn, c


def _failing_pin(module):
    for name, fn, kw in _pin_cases(module):
        try:
            fn(**kw)
        except (Exception, pytest.fail.Exception):   # an assertion, pytest.raises, or the mistake raising
            return f"{name}{kw or ''}"
    return None


def test_pin_runner_passes_on_the_unedited_oracle():
    # the runner itself: every pin passes when nothing is planted
    for module in PINS.values():
        assert _failing_pin(module) is None


@pytest.mark.parametrize("mod,fname,old,new,why", MUTANTS, ids=[f"{m[1]}: {m[4]}" for m in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, mod, fname, old, new, why):
    orig = getattr(mod, fname)
    mutant = _edited(mod, fname, old, new)
    for m in list(sys.modules.values()):
        if m is not None and getattr(m, fname, None) is orig:
            monkeypatch.setattr(m, fname, mutant)
    caught = _failing_pin(PINS[mod])
    assert caught is not None, f"no pin catches: {why}"
