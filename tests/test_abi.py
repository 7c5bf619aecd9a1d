"""The C ABI library: it loads, exports every symbol the header declares, and
its host-side validation returns the documented codes without a GPU."""
import ctypes
import math
import os
import re

import numpy as np

from paper_1712_03439_amd import rsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "rsim.h")).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)  # declarations only, not comments
    return sorted(set(re.findall(r"\b(rsim_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_header_symbol():
    lib = rsim.lib()
    syms = header_symbols()
    assert "rsim_mix" in syms and "rsim_truncate_rir" in syms
    for name in syms:
        assert hasattr(lib, name), name
    assert sorted(rsim.EXPORTS) == syms


def test_strerror_and_version():
    lib = rsim.lib()
    for code in range(6):
        assert lib.rsim_strerror(code)
    assert lib.rsim_version() == rsim.ABI_VERSION == 10200


def test_truncate_rejects_bad_eta_before_touching_the_gpu():
    lib = rsim.lib()
    dummy = ctypes.c_void_p(1)
    for eta in (-1.0, float("nan")):
        assert lib.rsim_truncate_rir(dummy, 10, dummy, dummy, 1, eta, None, dummy, None) == rsim.RSIM_EINVAL
    assert lib.rsim_truncate_rir(None, 10, None, None, 1, 20.0, None, None, None) == rsim.RSIM_EINVAL
    assert lib.rsim_truncate_rir(None, 0, None, None, 0, 20.0, None, None, None) == rsim.RSIM_OK


def test_ola_validation_codes():
    lib = rsim.lib()
    p = ctypes.c_void_p(1)
    assert lib.rsim_ola_convolve(None, 10, p, 4, 512, 0, p, p, 1 << 30, None) == rsim.RSIM_EINVAL
    assert lib.rsim_ola_convolve(p, 10, p, 4, 1000, 0, p, p, 1 << 30, None) == rsim.RSIM_EUNSUPPORTED
    assert lib.rsim_ola_convolve(p, 10, p, 4, 256, 0, p, p, 1 << 30, None) == rsim.RSIM_EUNSUPPORTED
    assert lib.rsim_ola_convolve(p, 10, p, 4, 65536, 0, p, p, 1 << 30, None) == rsim.RSIM_EUNSUPPORTED
    # hop + nh - 1 > fft_n
    assert lib.rsim_ola_convolve(p, 10, p, 400, 512, 200, p, p, 1 << 30, None) == rsim.RSIM_EUNSUPPORTED
    # RIR longer than the FFT (default hop would be < 1)
    assert lib.rsim_ola_convolve(p, 10, p, 600, 512, 0, p, p, 1 << 30, None) == rsim.RSIM_EUNSUPPORTED
    assert lib.rsim_ola_convolve(p, 10, p, 4, 512, 0, p, None, 0, None) == rsim.RSIM_EWORKSPACE
    assert lib.rsim_ola_workspace_bytes(1000) == 0
    assert lib.rsim_ola_workspace_bytes(8192) > 0


def _host_batch(U=3, J=2, S=2):
    b = rsim.RsimBatch()
    b.n_utt, b.n_mic, b.max_src, b.max_rir_len0 = U, J, S, 100
    b.x_len, b.h_len, b.y_len = 1000, 1000, 1000
    p = ctypes.c_void_p(8)
    for f in ("n_src", "src_len", "src_off", "rir_off", "rir_len0", "rir_len", "out_off",
              "out_stride", "out_len"):
        setattr(b, f, p.value)
    return b


def test_mix_validation_codes():
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    b = _host_batch()
    need = lib.rsim_mix_workspace_bytes(ctypes.byref(b), None, 0)
    assert need > 0
    assert lib.rsim_mix_workspace_bytes(ctypes.byref(b), None, 1) > need
    # too small a workspace
    assert lib.rsim_mix(ctypes.byref(b), p, p, p, p, p, need - 1, None, 0, None) == rsim.RSIM_EWORKSPACE
    # missing data pointers
    assert lib.rsim_mix(ctypes.byref(b), None, p, p, p, p, need, None, 0, None) == rsim.RSIM_EINVAL
    # ... except for an array of length 0: the call gets past the argument
    # checks (and, without a GPU, stops at the device: RSIM_EDEVICE)
    nox = _host_batch()
    nox.x_len = 0
    assert lib.rsim_mix(ctypes.byref(nox), None, p, p, p, p, need, None, 0, None) != rsim.RSIM_EINVAL
    # bad descriptor scalars
    bad = _host_batch()
    bad.n_mic = 0
    assert lib.rsim_mix(ctypes.byref(bad), p, p, p, p, p, need, None, 0, None) == rsim.RSIM_EINVAL
    bad = _host_batch()
    bad.src_off = None
    assert lib.rsim_mix(ctypes.byref(bad), p, p, p, p, p, need, None, 0, None) == rsim.RSIM_EINVAL
    assert lib.rsim_mix(None, p, p, p, p, p, need, None, 0, None) == rsim.RSIM_EINVAL
    empty = _host_batch(U=0)
    assert lib.rsim_mix(ctypes.byref(empty), None, None, None, None, None, 0, None, 0, None) == rsim.RSIM_OK
    # simulate: eta must be >= 0 and a cut-length output is needed
    assert lib.rsim_simulate(ctypes.byref(b), p, p, p, -3.0, p, p, p, need, None, 0, None) == rsim.RSIM_EINVAL
    assert lib.rsim_simulate(ctypes.byref(b), p, p, p, 20.0, None, p, p, need, None, 0, None) == rsim.RSIM_EINVAL


def test_workspace_grows_with_the_batch():
    lib = rsim.lib()
    small = _host_batch(U=2, J=2, S=2)
    big = _host_batch(U=200, J=8, S=4)
    assert lib.rsim_mix_workspace_bytes(ctypes.byref(big), None, 0) > \
        lib.rsim_mix_workspace_bytes(ctypes.byref(small), None, 0)


def test_rfft_validation():
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    assert lib.rsim_rfft(p, 1000, 1, p, None) == rsim.RSIM_EUNSUPPORTED
    assert lib.rsim_rfft(p, 65536, 1, p, None) == rsim.RSIM_EUNSUPPORTED
    assert lib.rsim_irfft(None, 1024, 2, p, None) == rsim.RSIM_EINVAL
    assert lib.rsim_rfft(p, 1024, 0, p, None) == rsim.RSIM_OK


def test_snr_gains_host_rule_matches_oracle():
    import oracle

    r = np.random.default_rng(4)
    for _ in range(50):
        I = int(r.integers(1, 5))
        p = list(r.uniform(1e-4, 1.0, I))
        snr = [0.0] + list(r.uniform(0, 30, I - 1))
        got = rsim.snr_gains(p, snr, 3)
        ref = oracle.snr_gains(p, snr, 3).astype(np.float32)
        np.testing.assert_array_max_ulp(got, ref, maxulp=1)
    assert np.all(rsim.snr_gains([1.0, 0.0], [0.0, 10.0], 2)[1] == 0.0)
    lib = rsim.lib()
    assert lib.rsim_snr_gains(None, None, 2, 2, None) == rsim.RSIM_EINVAL
    assert lib.rsim_snr_gains(None, None, 0, 2, None) == rsim.RSIM_OK


def test_mix_backward_validation_codes():
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    b = _host_batch()
    need = lib.rsim_mix_workspace_bytes(ctypes.byref(b), None, 1)
    args = lambda **k: [k.get(n, p) for n in ("x", "h", "alpha", "gy", "gx", "gh", "ga")]  # noqa: E731
    # too small a workspace
    assert lib.rsim_mix_backward(ctypes.byref(b), *args(), p, need - 1, None, None) == rsim.RSIM_EWORKSPACE
    # every data pointer but grad_alpha is required
    for name in ("x", "h", "alpha", "gy", "gx", "gh"):
        assert lib.rsim_mix_backward(ctypes.byref(b), *args(**{name: None}), p, need, None, None) == \
            rsim.RSIM_EINVAL, name
    bad = _host_batch()
    bad.n_mic = 0
    assert lib.rsim_mix_backward(ctypes.byref(bad), *args(), p, need, None, None) == rsim.RSIM_EINVAL
    empty = _host_batch(U=0)
    assert lib.rsim_mix_backward(ctypes.byref(empty), *([None] * 7), None, 0, None, None) == rsim.RSIM_OK


def test_one_size_tune_field_reaches_the_workspace_query():
    # the tune table is accepted by the size query with either policy
    lib = rsim.lib()
    b = _host_batch()
    f, m = [2.5 * (1 << k) * k for k in range(9, 16)], [8.0 * ((1 << k) / 2 + 1) for k in range(9, 16)]
    for one in (False, True):
        t = rsim.tune_table(f, m, one_size=one)
        assert lib.rsim_mix_workspace_bytes(ctypes.byref(b), ctypes.byref(t), 0) > 0


def test_tune_table_layout_and_validation():
    # rsim_tune: 7 + 7 floats, one_size, variant[6] (int32), no padding
    assert ctypes.sizeof(rsim.RsimTune) == 84
    assert rsim.RsimTune.variant.offset == 60 and rsim.RsimTune.one_size.offset == 56
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    b = _host_batch()
    f, m = [2.5 * (1 << k) * k for k in range(9, 16)], [8.0 * ((1 << k) / 2 + 1) for k in range(9, 16)]
    for code in range(5):
        t = rsim.tune_table(f, m, True, [code] * 6)
        assert lib.rsim_mix_workspace_bytes(ctypes.byref(b), ctypes.byref(t), 0) > 0, code
    bad = []
    for field, val in (("variant", 5), ("variant", -1), ("cost_fft", -1.0), ("cost_mac", math.nan),
                       ("cost_fft", math.inf)):
        t = rsim.tune_table(f, m, True)
        getattr(t, field)[2] = val
        bad.append(t)
    for t in bad:
        r = ctypes.byref(t)
        assert lib.rsim_mix_workspace_bytes(ctypes.byref(b), r, 0) == 0
        assert lib.rsim_mix(ctypes.byref(b), p, p, p, p, p, 1 << 30, r, 0, None) == rsim.RSIM_EINVAL
        assert lib.rsim_simulate(ctypes.byref(b), p, p, p, 20.0, p, p, p, 1 << 30, r, 0, None) == rsim.RSIM_EINVAL
        assert lib.rsim_mix_backward(ctypes.byref(b), p, p, p, p, p, p, p, p, 1 << 30, r, None) == rsim.RSIM_EINVAL


def test_variant_sets_the_mic_split_of_the_workspace():
    # with fewer utterances than compute units, one mic per pass splits an
    # utterance of two mics into two work items (400 items, each with a
    # scratch slot); two mics per pass do not, and its 200 items are split
    # into block ranges instead (shared RIR spectra and seam buffers)
    lib = rsim.lib()
    b = _host_batch(U=200, J=2)
    f, m = [2.5 * (1 << k) * k for k in range(9, 16)], [8.0 * ((1 << k) / 2 + 1) for k in range(9, 16)]
    one = lib.rsim_mix_workspace_bytes(ctypes.byref(b), ctypes.byref(rsim.tune_table(f, m, True, [1] * 6)), 0)
    two = lib.rsim_mix_workspace_bytes(ctypes.byref(b), ctypes.byref(rsim.tune_table(f, m, True, [2] * 6)), 0)
    dflt = lib.rsim_mix_workspace_bytes(ctypes.byref(b), ctypes.byref(rsim.tune_table(f, m, True)), 0)
    assert dflt == two and one != two


def test_image_rir_validation_codes():
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    ok = dict(n=4, order=8, fs=16000.0, c0=343.0, h_len=1000, max_len=100)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.rsim_image_rir(p, p, a["n"], a["order"], a["fs"], a["c0"], p, a["h_len"], p, p,
                                  a["max_len"], None)

    for bad in (dict(n=-1), dict(order=-1), dict(order=17), dict(fs=0.0), dict(fs=math.nan),
                dict(c0=-343.0), dict(c0=math.inf), dict(max_len=-1), dict(h_len=-5)):
        assert call(**bad) == rsim.RSIM_EINVAL, bad
    assert call(n=0) == rsim.RSIM_OK and call(max_len=0) == rsim.RSIM_OK
    assert call(max_len=32769) == rsim.RSIM_EUNSUPPORTED
    assert lib.rsim_image_rir(None, p, 4, 8, 16000.0, 343.0, p, 1000, p, p, 100, None) == rsim.RSIM_EINVAL


def test_simulate_rooms_validation_codes():
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    b = _host_batch()
    need = lib.rsim_mix_workspace_bytes(ctypes.byref(b), None, 0)

    def call(bb=b, order=8, fs=16000.0, c0=343.0, eta=20.0, x=p, ws_bytes=need):
        return lib.rsim_simulate_rooms(ctypes.byref(bb) if bb is not None else None, x, p, p, p, order, fs, c0,
                                       p, eta, p, p, p, ws_bytes, None, 0, None)

    assert call(bb=None) == rsim.RSIM_EINVAL
    assert call(order=17) == rsim.RSIM_EINVAL and call(fs=-1.0) == rsim.RSIM_EINVAL
    assert call(eta=-1.0) == rsim.RSIM_EINVAL and call(x=None) == rsim.RSIM_EINVAL
    assert call(ws_bytes=need - 1) == rsim.RSIM_EWORKSPACE
    long = _host_batch()
    long.max_rir_len0 = 40000
    assert call(bb=long) == rsim.RSIM_EUNSUPPORTED


def test_reverb_energy_and_gain_validation():
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    b = _host_batch()
    assert lib.rsim_reverb_energy(None, p, p, p, None) == rsim.RSIM_EINVAL
    assert lib.rsim_reverb_energy(ctypes.byref(b), None, p, p, None) == rsim.RSIM_EINVAL
    assert lib.rsim_reverb_energy(ctypes.byref(_host_batch(U=0)), None, None, None, None) == rsim.RSIM_OK
    assert lib.rsim_snr_gains_reverb(None, None, 2, 0, None) == rsim.RSIM_EINVAL
    # the host rule against the oracle's
    import oracle
    rng = np.random.default_rng(3)
    E = rng.uniform(0.01, 9.0, (3, 2))
    E[2, 1] = 0.0
    snr = [0.0, 4.0, 17.0]
    got = rsim.snr_gains_reverb(E, snr)
    ref = oracle.snr_gains_reverb(E, snr).astype(np.float32)
    assert np.allclose(got, ref, rtol=2e-7, atol=0)


def test_fft_filter_validation_codes():
    lib = rsim.lib()
    p = ctypes.c_void_p(8)
    b = _host_batch()
    need = lib.rsim_fft_filter_workspace_bytes(ctypes.byref(b), 12, 4)
    assert need == 3 * 2 * 4 * 4096 * 8  # 3 max_src chunk N complex floats
    for l2, chunk in ((0, 4), (21, 4), (12, 0)):
        assert lib.rsim_fft_filter_workspace_bytes(ctypes.byref(b), l2, chunk) == 0
        assert lib.rsim_fft_filter(ctypes.byref(b), p, p, p, p, l2, chunk, p, need, None) == rsim.RSIM_EINVAL
    assert lib.rsim_fft_filter(ctypes.byref(b), p, p, p, p, 12, 4, p, need - 1, None) == rsim.RSIM_EWORKSPACE
    assert lib.rsim_fft_filter(ctypes.byref(b), None, p, p, p, 12, 4, p, need, None) == rsim.RSIM_EINVAL


def test_binding_structs_match_the_header(tmp_path):
    # every field offset and the size of the ctypes mirrors of rsim_batch and
    # rsim_tune, as the C compiler lays out the declarations in include/
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = []
    for cname, cls in (("rsim_batch", rsim.RsimBatch), ("rsim_tune", rsim.RsimTune)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include "rsim.h"\nint main(void) {\n' + "\n".join(lines) +
                   "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                          text=True).stdout.splitlines())
    for cname, cls in (("rsim_batch", rsim.RsimBatch), ("rsim_tune", rsim.RsimTune)):
        assert int(got[f"{cname} size"]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname} {fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_forced_sizes_hint_limits_the_workspace():
    # with forced sizes, fft_sizes names the sizes in use: only their kernel
    # families get scratch; 0 provides for every size
    lib = rsim.lib()
    b = _host_batch()
    b.fft_log2n = ctypes.c_void_p(8).value
    b.fft_sizes = 0
    every = lib.rsim_mix_workspace_bytes(ctypes.byref(b), None, 0)
    b.fft_sizes = 1 << 14
    one = lib.rsim_mix_workspace_bytes(ctypes.byref(b), None, 0)
    assert 0 < one < every
    b.fft_sizes = (1 << 14) | (1 << 12)
    two = lib.rsim_mix_workspace_bytes(ctypes.byref(b), None, 0)
    assert one < two < every
    assert rsim.size_bits(None) == 0 and rsim.size_bits(np.array([14, 12, 14, 16, 8])) == (1 << 14) | (1 << 12)


def test_full_length_transform_sizes():
    # N = 2^ceil(log2(Nx + L0max - 1)) per utterance, L0max over its slots;
    # 0 without samples or taps
    lib = rsim.lib()
    src = np.array([100, 1, 5000, 0, 7], np.int32)
    l0 = np.array([[29, 3], [1, 0], [0, 4097], [50, 50], [0, 0]], np.int32).reshape(-1)
    out = np.full(5, -1, np.int32)
    assert lib.rsim_fft_filter_sizes(src.ctypes.data, l0.ctypes.data, 5, 1, 2, out.ctypes.data) == rsim.RSIM_OK
    assert list(out) == [7, 1, 14, 0, 0]
    assert lib.rsim_fft_filter_sizes(src.ctypes.data, l0.ctypes.data, -1, 1, 2, out.ctypes.data) == rsim.RSIM_EINVAL
