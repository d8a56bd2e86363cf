"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liborc.so with g++."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "conegauss_oracle.cpp")
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False, out: str = None, extra=(), opt: str = "-O2") -> str:
    """Builds the oracle into `out` (default oracle/liborc.so), with extra compiler flags
    if given (an instrumented build for tests)."""
    out = out or LIB
    cmd = ["g++", opt, "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", *extra,
           "-shared", "-fPIC", "-o", out + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
