"""bench.py's command line on the host: more than one GPU is refused with a
message (this engine runs on one GPU), and the HBM-traffic figure is reported
only for the workload and kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_traffic_only_for_its_workload():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.traffic_for("corr256") is None
    t = bench.traffic_for("shells32x10")
    assert t is None or t > 1e6
