"""Builds the HIP library libconegauss.so for gfx950 (hipcc, one object per source,
then a shared link).  Run directly or through __graft_entry__.build()."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libconegauss.so")
ARCH = os.environ.get("CG_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          # contract a*b+c only within one source expression, so that the forward render and
          # the backward replay (same expressions, different kernels) round identically
          "-ffp-contract=on",
          "-Wall", "-Wno-unused-function",
          # no packed-FP32 instructions in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str, verbose: bool, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = ["hipcc", *COMMON, *extra, "-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_variant(out: str, extra_compile=(), extra_link=(), verbose: bool = False, jobs: int = 8) -> str:
    """The library built into `out` with extra compiler and linker flags (objects in a
    folder `obj` beside it), e.g. an instrumented build for tests of the host code."""
    out_dir = os.path.join(os.path.dirname(os.path.abspath(out)), "obj")
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, out_dir, tuple(extra_compile)), sources()))
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-fPIC", *extra_link, "-o", out, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
