"""Compile the CPU oracle (plain C + OpenMP) into ``oracle/liboracle.so``.

Test infrastructure only: building the checker is not using it.  The flags
keep the arithmetic IEEE-exact (no fast-math, no contraction of a*b+c into an
FMA except where the source calls fmaf explicitly).
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stencil_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = f"{OUT}.tmp{os.getpid()}"  # per process, so that two builders never share a file
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
