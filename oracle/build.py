"""Build the CPU oracle shared library (plain C, gcc, FP64).

Test infrastructure: compiled next to this file as ``libvplbm_oracle.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vplbm_oracle.c")
LIB = os.path.join(HERE, "libvplbm_oracle.so")

# Portable x86-64 level (the library also runs on the GPU host's CPU);
# no FMA contraction so every rounding follows the written expression.
CFLAGS = ["-O3", "-march=x86-64-v2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
