"""Build libg6mi.so in-tree with hipcc for gfx950.

Packed-FP32 instruction selection is switched off (``-packed-fp32-ops``):
every float operation is issued as an ordinary VOP instruction.  Run
``python -m paper_0902_4463_amd.build`` or call :func:`build`.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libg6mi.so")
SOURCES = [os.path.join(CSRC, "g6mi_kernels.hip"), os.path.join(CSRC, "g6mi_batch.hip"),
           os.path.join(CSRC, "g6mi_hermite.hip"), os.path.join(CSRC, "g6mi_spatial.hip"),
           os.path.join(CSRC, "g6mi_api.cpp")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libg6mi")


def flags(extra=()):
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", *extra]


def build(verbose: bool = False, extra=(), out: str = LIB) -> str:
    """Compile the library to ``out``; ``extra`` adds compiler options such
    as -DG6MI_TILE=512 (the tuning knobs in csrc/g6mi_internal.h)."""
    cmd = [hipcc(), *flags(extra), "-shared", "-o", out + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
