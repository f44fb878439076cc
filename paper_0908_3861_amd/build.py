"""Build libbsf.so (hand-written HIP for gfx950) in the package directory.

    python -m paper_0908_3861_amd.build

Compiles ``csrc/bsf.hip`` with hipcc for gfx950 only.  Packed-FP32 instructions are
disabled: the kernels are float64/int64 code, and the packed forms are not wanted.
Floating-point contraction is off: the double-double arithmetic depends on every
product and sum being rounded as written (fusing ``p = a*b; s = p + e`` into one FMA
breaks the error-free transforms).  The FMAs the kernels want are explicit.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "bsf.hip")
LIB = os.path.join(HERE, "libbsf.so")
ARCH = os.environ.get("BSF_OFFLOAD_ARCH", "gfx950")


def hipcc_command(out: str) -> list[str]:
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-ffp-contract=off", "-Wno-unused-command-line-argument",
        "-I", os.path.join(HERE, "..", "include"),
        "-o", out, SRC,
    ]


def build(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libbsf.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
