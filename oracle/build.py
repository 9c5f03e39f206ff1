"""Build the C oracle (``liboracle.so``) with gcc and OpenMP.

Test infrastructure: compiled next to its source so that it travels with the
tree.  ``python -m oracle.build`` rebuilds it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mmpm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-std=c11", "-Wall", "-Wextra",
        "-shared", "-fPIC", "-o", LIB + ".tmp", SRC,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        return build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
