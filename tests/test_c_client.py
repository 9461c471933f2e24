"""The C interface from a plain C program (no Python, no torch): compile
tests/c/abi_check.c with gcc against include/omega.h, link libomega.so and run
the host-only checks."""
import os
import shutil
import subprocess

import pytest

from paper_1412_8754_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_program_uses_the_interface(tmp_path):
    lib = _abi.LIB_PATH
    assert lib.exists(), "build libomega.so first"
    exe = tmp_path / "abi_check"
    subprocess.run(["gcc", "-std=c11", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_check.c"),
                    "-o", str(exe), str(lib), "-Wl,-rpath," + str(lib.parent), "-lm"],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
