"""The C ABI from a C program: tests/native/abi_c.c is compiled as C11 with
gcc against include/acopf.h, linked to libacopf.so and run (host calls
only).  No GPU needed."""
import os
import shutil
import subprocess

import pytest

from paper_2203_10587_amd import acopf as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_program_uses_the_abi(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    A.lib()  # raises with a build hint if the library is missing
    libdir = os.path.dirname(A.LIB_PATH)
    exe = str(tmp_path / "abi_c")
    cmd = ["gcc", "-std=c11", "-Wall", "-Werror", "-O1", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "native", "abi_c.c"), "-o", exe,
           "-L" + libdir, "-l:libacopf.so", "-Wl,-rpath," + libdir,
           "-Wl,-rpath-link,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, (run.returncode, run.stdout, run.stderr)
    assert "abi_c ok" in run.stdout
