"""The benchmark's host-side contract (CPU only): one GPU only, the counter
traffic taken only for the kernel and sources it was measured on, and the
kernel symbol each tune variant runs."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("field,value,expect", [(None, None, True), ("source_sha256", "0" * 64, False),
                                                ("kernel", "void rsim::other(rsim::MixArgs)", False)])
def test_counter_traffic_only_for_its_kernel_and_sources(tmp_path, monkeypatch, field, value, expect):
    kernel = bench.mix_kernel_name(14, [0, 1, 2, 2, 2, 4])
    entry = {"kernel": kernel, "source_sha256": bench.source_digest(),
             "fetch_bytes_per_launch": 1000.5, "write_bytes_per_launch": 24.0}
    if field:
        entry[field] = value
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(entry))
    monkeypatch.setattr(bench, "COUNTERS", str(path))
    got = bench.counter_traffic(kernel)
    assert got == (1024 if expect else None)


def test_missing_or_unreadable_counters_give_no_traffic(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "absent.json"))
    assert bench.counter_traffic("k") is None
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    monkeypatch.setattr(bench, "COUNTERS", str(bad))
    assert bench.counter_traffic("k") is None


def test_kernel_symbol_of_each_variant():
    # variant codes 1..4 = (mic accumulators, waves per SIMD) (1, 2), (2, 1),
    # (2, 2), (1, 4); 0 is the library default (2); the 32768 family runs 4
    assert bench.mix_kernel_name(14, [0] * 6) == "void rsim::mix_kernel<512, 2, 1, false>(rsim::MixArgs)"
    assert bench.mix_kernel_name(14, [0, 0, 0, 0, 3, 0]) == "void rsim::mix_kernel<512, 2, 2, false>(rsim::MixArgs)"
    assert bench.mix_kernel_name(13, [0, 0, 0, 1, 0, 0]) == "void rsim::mix_kernel<256, 1, 2, false>(rsim::MixArgs)"
    assert bench.mix_kernel_name(15, [0, 0, 0, 0, 0, 2]) == "void rsim::mix_kernel<1024, 1, 4, false>(rsim::MixArgs)"
    assert bench.mix_kernel_name(9, None) == "void rsim::mix_kernel<32, 2, 1, false>(rsim::MixArgs)"


def test_error_record_of_a_parity_case():
    # the error leg reports max |gpu - ref| / max |ref| per workload, and
    # inf when a cut length differs from the oracle's
    import numpy as np

    import oracle
    import synth

    b = synth.make_config2(n_utt=2, epoch=3)
    xs, hs, snrs = b.sources(0), b.rirs(0), list(b.snrs(0))
    ref, _, Ls, _ = oracle.simulate(xs, hs, snrs, 20.0)
    outs = [ref[j].astype(np.float32) for j in range(b.n_mic)]
    _, e = bench._forward_error(("w", xs, hs, snrs, 20.0, Ls, outs))
    assert 0.0 <= e <= 1e-7
    bad = [row[:] for row in Ls]
    bad[0][0] += 1
    assert bench._forward_error(("w", xs, hs, snrs, 20.0, bad, outs))[1] == float("inf")
    info = bench.host_info()
    assert info["os_cpu_count"] >= 1 and "cpu_model" in info


def test_counter_digest_ignores_comments_only():
    text = 'int a = 1; // note\n/* block\n note */ const char* s = "a // b"; char q = \'"\';\n\n  int b; /* x */\n'
    assert bench._code_only(text) == 'int a = 1;\n const char* s = "a // b"; char q = \'"\';\n  int b;'
    assert bench._code_only(text.replace("note", "other note")) == bench._code_only(text)
    assert bench._code_only(text.replace("a = 1", "a = 2")) != bench._code_only(text)
