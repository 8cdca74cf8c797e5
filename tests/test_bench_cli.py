"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a JSON line saying so, and every workload name is accepted by
the parser."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_workloads_parse():
    sys.path.insert(0, ROOT)
    import bench
    saved = sys.argv
    try:
        for w in ("cavity", "rod-table1", "learned", "batch12", "scene", "loads", "scene-waves"):
            sys.argv = ["bench.py", "--workload", w]
            assert bench.parse().workload == w
    finally:
        sys.argv = saved
