"""Host logic of bench.py (no GPU): the one-GPU guard, the workload choices,
and the rule that the measured HBM traffic is reported only for the kernel
source and workload the counters were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stdout


@pytest.mark.parametrize("workload", ["3d", "2d", "2d-thresholded", "small", "batch",
                                      "sequence", "sequence2d", "topopt"])
def test_every_workload_parses(workload, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", workload])
    assert bench.parse().workload == workload


def test_traffic_only_for_the_profiled_source_and_workload(monkeypatch):
    kernel = "interior_solve<double>"
    m = bench.MEASURED_TRAFFIC[kernel]
    assert bench.measured_traffic(kernel, "cantilever2d_simp_512x256") is None
    assert bench.measured_traffic("no_such_kernel", m["workload"]) is None
    # the committed kernel source is the profiled one, and the profile
    # summary quotes the same figure
    assert bench.measured_traffic(kernel, m["workload"]) == m["bytes"]
    with open(os.path.join(ROOT, m["profile"])) as fh:
        assert f"{m['bytes'] / 1e9:.3f} GB" in fh.read()
    # a changed source voids the figure
    monkeypatch.setitem(m, "sha256_prefix", "0" * 16)
    assert bench.measured_traffic(kernel, m["workload"]) is None
