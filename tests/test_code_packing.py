"""The 16-bit packed stencil codes the sweeps read (``csrc/codes.h``): an
exhaustive host check that packing and unpacking are inverse on every code
word the neighbourhood evaluation (Algorithm 1, App. B cases) can produce, and
that a solid face keeps only its solid bit.  Built from the library's own
header with the host compiler; no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2407_19868_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_code_packing_exhaustive(tmp_path):
    exe = tmp_path / "code_packing"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, os.path.join(HERE, "code_packing.cpp"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == f"ok {37 ** 3}"
