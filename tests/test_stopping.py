"""The convergence decision of every check (``csrc/stopping.h``): stop rules r < tol
and eps_q < tol (Algorithm 1's evaluation every M sweeps, §7.1's criterion), the
FP32 floor gate with its plateau reading of the residual history, and the
hand-overs of the FP32-DC form.  One host case per branch, then invariants over
every combination of flags, stall counts and residual levels (a spent budget
never sweeps on; Stop only where the rule holds, never from eps_q near the FP32
floor and never from the FP32 phase of FP32-DC; FP64 ignores the floor
signals).  Built from the library's own header with the host compiler; no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2407_19868_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_check_decisions(tmp_path):
    exe = tmp_path / "stopping"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, os.path.join(HERE, "stopping.cpp"), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok 41 7680"
