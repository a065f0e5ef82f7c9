"""CPU checks of bench.py's command-line contract: more than one GPU is
refused with a message (the build runs on one GPU), and the recorded
traffic figures name the grid they were measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_is_reported_only_for_its_grid():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic(bench.MEASURED_TRAFFIC["n"] + 1) is None
