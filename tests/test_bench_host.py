"""Host logic of bench.py (no GPU needed): the one-GPU refusal, the algorithmic
bytes per voxel of the roofline, and the counter-traffic lookup that holds only
while the kernel sources are those the counters were taken on."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_algorithmic_bytes_per_voxel(bench):
    # four fields (u, v, w, p) read once and written once, plus the face flags
    # of the three velocity components at one bit each
    for form, elem in (("fp64", 8), ("fp32", 4)):
        assert bench.BYTES_PER_VOXEL[form] == 4 * 2 * elem + 3 / 8


def test_traffic_follows_the_committed_profile(bench):
    text = open(bench.TRAFFIC_PROFILE).read()
    rows = dict(line.split(":", 1) for line in text.splitlines() if line.startswith("traffic_bytes_per_launch_"))
    for form in ("fp64", "fp32", "fp64_two_step", "fp32_two_step"):
        assert f"traffic_bytes_per_launch_{form}" in rows
    # the profile is committed with the sources it was measured on
    assert f"kernel_source_sha256: {bench.kernel_source_hash()}" in text
    for form in ("fp64", "fp32"):
        got = bench.measured_traffic(form)
        assert got == float(rows[f"traffic_bytes_per_launch_{form}"])
        # counted traffic of one sweep launch over three 256^3 instances lies
        # between the algorithmic bytes and 1.25 times them
        alg = bench.BYTES_PER_VOXEL[form] * 3 * 256 ** 3
        assert alg <= got <= 1.25 * alg


def test_traffic_is_withheld_for_other_sources(bench, tmp_path, monkeypatch):
    changed = tmp_path / "kernels.hip"
    changed.write_bytes(open(bench.KERNEL_SOURCES[0], "rb").read() + b"\n// edited\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(changed)] + bench.KERNEL_SOURCES[1:])
    assert bench.measured_traffic("fp64") is None
    assert bench.measured_traffic("fp32") is None
