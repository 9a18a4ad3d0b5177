"""Build step of the HIP library: hipcc for gfx950 into ``libgspca.so`` in-tree.

``python -m paper_0811_1081_amd.build`` compiles every source under ``csrc/``
into one shared library next to this file.  Packed-FP32 instructions are
disabled (the compiler is told the target lacks them), and no fast-math flag
is used, so FP32 division and square root stay IEEE-rounded.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB_PATH = os.path.join(HERE, "libgspca.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libgspca.so")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def flags():
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-fno-fast-math", "-ffp-contract=fast",
        "-Wall", "-Wno-unused-result",
        "-I" + INCLUDE, "-I" + CSRC,
    ]


def build(verbose: bool = False) -> str:
    """Compile all HIP sources into libgspca.so (always recompiles)."""
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *flags(), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
