"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The FP64 oracle, built with g++ -fsanitize=address,undefined, runs every entry point
  on small scenes (all filters, floors, compositions, orders, camera models, crops, an
  empty scene and an empty crop, the gradient and the supersampled reference).
* The library, its host code built with the same sanitizers (the kernels as usual),
  runs the argument checks of every entry point, the profiling and debugging
  switches, and the render server's scheduler under its CPU stand-in executor.

Each runs in a child process that preloads the matching ASan runtime; a sanitizer
report ends it with a non-zero status.  The instrumented builds go to a temporary
folder."""
import glob
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# sanitizer flags; the library's are given to the host compilation only
ORACLE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
HOST_FLAGS = []
for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"):
    HOST_FLAGS += ["-Xarch_host", flag]
HOST_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1", "OMP_NUM_THREADS": "2"}


def _run(driver, lib_path, runtime, timeout):
    env = dict(os.environ, **ENV, LD_PRELOAD=runtime)
    r = subprocess.run([sys.executable, os.path.join(HERE, driver), lib_path], env=env, capture_output=True,
                       text=True, timeout=timeout, cwd=ROOT)
    report = r.stderr[-6000:]
    assert r.returncode == 0, f"exit {r.returncode}\n{r.stdout[-2000:]}\n{report}"
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    return r.stdout


def _gcc_asan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clang_asan():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/*/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_oracle_under_asan_ubsan(tmp_path):
    runtime = _gcc_asan()
    if runtime is None:
        pytest.skip("gcc's ASan runtime is not installed")
    from oracle import build_oracle
    lib = build_oracle.build(out=str(tmp_path / "liborc_san.so"), extra=ORACLE_FLAGS, opt="-O1")
    out = _run("san_oracle_driver.py", lib, runtime, timeout=600)
    assert "ran clean" in out


def test_host_abi_under_asan_ubsan(tmp_path):
    runtime = _clang_asan()
    if runtime is None:
        pytest.skip("clang's ASan runtime is not installed")
    try:
        subprocess.run(["hipcc", "--version"], capture_output=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("hipcc is not available")
    from paper_2609_13397_amd import build_lib
    lib = build_lib.build_variant(str(tmp_path / "libcg_san.so"), HOST_FLAGS, HOST_LINK)
    out = _run("san_abi_driver.py", lib, runtime, timeout=600)
    assert "ran clean" in out
