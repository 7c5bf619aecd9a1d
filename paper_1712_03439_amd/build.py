"""Build librsim.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

    python -m paper_1712_03439_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "rsim.hip")
HDRS = [os.path.join(HERE, "csrc", "fft_engine.hpp"), os.path.join(HERE, "csrc", "kernels.hpp"),
        os.path.join(ROOT, "include", "rsim.h")]
LIB = os.path.join(HERE, "librsim.so")
ARCH = os.environ.get("RSIM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def command(out: str = LIB, extra=()) -> list:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # Packed FP32 instructions are kept out of the generated code.
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"),
        *extra, SRC, "-o", out,
    ]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp, extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = res.stdout
    # hipcc's host pass does not know the device-only feature flag.
    noise = "is not a recognized feature for this target"
    lines = [ln for ln in out.splitlines() if noise not in ln and "ignoring feature" not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
