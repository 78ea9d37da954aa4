"""Compile the CPU oracle (plain C, float64, OpenMP over i-particles).

``-ffp-contract=off`` keeps the compiler from fusing multiply-adds, so the
arithmetic is exactly the term-by-term float64 evaluation written in the
source.  Run ``python -m oracle.build`` or call :func:`build`.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "g6_oracle.c")
LIB = os.path.join(HERE, "libg6oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
