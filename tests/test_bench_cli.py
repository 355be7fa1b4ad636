"""The benchmark's command line on the CPU: more than one GPU is refused with a
message before anything touches a device, and the workload table names every
workload the line can report."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workload_table():
    sys.path.insert(0, ROOT)
    import bench
    assert set(bench.WORKLOADS) == {"c1", "c2", "c3"}
    assert set(bench.MULTI) == {"c4", "c5", "loop"}
    assert bench.WORKLOADS["c3"]["precision"] == "bf16x3" and bench.WORKLOADS["c3"]["peak"] == "bf16"
    # the traffic summary belongs to the posterior kernel source it was taken on
    t = bench.traffic_from_profile("bf16x3", "c3")
    assert t is None or 4.0e7 < t < 1.0e8
