"""Compile the FP64 CPU oracle (test infrastructure) into a shared library.

The oracle is plain C99 built with gcc: no fast-math and no FMA contraction,
so every operation is a correctly rounded IEEE double operation. OpenMP
spreads independent pairs over the host cores.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["fiber_oracle.c", "fiber_exact.c", "fiber_validate.c"]
LIB = os.path.join(HERE, "liboracle_fiber.so")


def gcc_cmd(srcs, out):
    return ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
            "-o", out, *srcs, "-lm"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = gcc_cmd(srcs, LIB + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
