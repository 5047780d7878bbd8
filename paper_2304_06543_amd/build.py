"""Build liblbdd.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

    python -m paper_2304_06543_amd.build

The library is written next to this file.  Packed-FP32 instructions are
disabled for all device code (the kernels are integer-only anyway).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbdd.so")
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def build(out: str = LIB, verbose: bool = False) -> str:
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature and says so: harmless
    noise = [l for l in p.stderr.splitlines() if l.strip() and "packed-fp32-ops" not in l
             and "not a recognized feature" not in l]
    if p.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + p.stderr)
    if verbose and noise:
        print("\n".join(noise), file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
