"""bench.py's contract on the CPU: one-GPU refusal, the per-unit work figures
the roofline uses, and the committed HBM-traffic summary it reads."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_per_unit_flops_at_orders_4_6():
    npts = 4 * 6 * 6
    # (parent point, child box) pair: 16 complex columns x npts real weights, centring, geometry
    assert bench.flops_per_unit("propagate", npts) == 9654.0
    # (target, cousin box) pair: value and normal-derivative rows, weights, epilogue
    assert bench.flops_per_unit("targets", npts) == 17868.0


def test_per_unit_flops_of_one_kernel_per_pass():
    npts = 4 * 6 * 6
    # a pass carries 8 complex columns; its geometry and epilogue terms stay
    assert bench.flops_per_unit("propagate", npts, nk=1) == 4 * npts * 8 + 2 * npts + 150 == 5046.0
    assert bench.flops_per_unit("targets", npts, nk=1) == 4 * npts * 8 + 4 * npts * 6 + 10 * npts + 300 == 9804.0
    st = {"kernels_per_pass": 1, "timing": {"propagate": {"launches": 8, "ms": 2.0, "units": 10.0}}}
    assert bench.kernel_table(st, 1, npts)["propagate"]["flop"] == 50460.0
    st["kernels_per_pass"] = 0          # host-only plans report 0: both kernels
    assert bench.kernel_table(st, 1, npts)["propagate"]["flop"] == 96540.0


def test_per_unit_flops_at_orders_5_5():
    npts = 5 * 5 * 5
    # (parent point, child box) pair: 16 complex columns x npts real weights, centring, geometry
    assert bench.flops_per_unit("propagate", npts) == 8400.0
    # (target, cousin box) pair: value and normal-derivative rows, weights, epilogue
    assert bench.flops_per_unit("targets", npts) == 15550.0
    assert bench.flops_per_unit("unknown", npts) == 0.0
    assert bench.bytes_per_unit("nm_correct") == 68.0


def test_traffic_summary_is_read_only_for_its_workload_and_kernel(monkeypatch):
    vals = {}
    for line in open(bench.TRAFFIC):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != bench.kernel_sha():
        pytest.skip("propagation source changed since the counters were taken")
    t = bench.traffic_per_launch("propagate", "fp32", 153600, 4, 6)
    assert t == float(vals["hbm_bytes_per_launch"]) and t > 0
    assert bench.traffic_per_launch("propagate", "fp64", 153600, 4, 6) is None
    assert bench.traffic_per_launch("propagate", "fp32", 6144, 4, 6) is None
    assert bench.traffic_per_launch("propagate", "fp32", 153600, 5, 5) is None
    assert bench.traffic_per_launch("targets", "fp32", 153600, 4, 6) is None
    monkeypatch.setattr(bench, "kernel_sha", lambda *a: "0" * 64)
    assert bench.traffic_per_launch("propagate", "fp32", 153600, 4, 6) is None
