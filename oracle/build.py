"""Build step for the plain-C oracle (test infrastructure only).

Compiles ``oracle/csrc/lse_oracle.c`` into ``oracle/liblse_oracle.so`` with gcc:
-O3, OpenMP, no fast-math, no FMA contraction (the compensated sums rely on
every addition being rounded on its own), no -march=native (the library may
run on a different host CPU than the one that built it, so it keeps to the
baseline x86-64 instruction set: SSE2, no AVX).
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "lse_oracle.c")
LIB = os.path.join(HERE, "liblse_oracle.so")
FLAGS = ["-O3", "-fopenmp"]
BUILD_NOTE = "gcc -O3 -fopenmp -ffp-contract=off, no -march=native (baseline x86-64: SSE2, no AVX)"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *FLAGS, "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
