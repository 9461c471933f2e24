"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The FP64 oracle: tests/c/oracle_sanitize.c compiles oracle/omega_oracle.c
  into a program that calls every exported routine (ragged lattices, NaN
  inputs, invalid arguments) and is built with gcc's sanitizers.
- The host side of libomega: the library is rebuilt with the sanitizers on
  its host code only (GPU code is compiled as usual), and the plain C client
  tests/c/abi_check.c (host-only entry points and the validation that runs
  before anything is enqueued) is linked against it.
The sanitizers abort on the first out-of-bounds access, use after free,
leak or undefined operation; a clean run prints "ok".
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"), "-o", str(exe),
                    "-lm"], check=True)
    env = dict(SAN_ENV, OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="no ROCm compilers")
def test_library_host_code_under_sanitizers(tmp_path):
    lib = tmp_path / "libomega.so"
    csrc = os.path.join(ROOT, "paper_1412_8754_amd", "csrc")
    # sanitizers on the host compilation only: each flag behind -Xarch_host
    host_san = ["-Xarch_host", "-fsanitize=address",
                "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                    "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    *host_san, "-I", os.path.join(ROOT, "include"),
                    os.path.join(csrc, "omega_kernels.hip"), os.path.join(csrc, "omega_api.hip"),
                    "-o", str(lib)], check=True, capture_output=True)
    exe = tmp_path / "abi_check"
    subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_check.c"), "-o", str(exe), str(lib),
                    "-Wl,-rpath," + str(tmp_path), "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=SAN_ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
