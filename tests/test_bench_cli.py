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


def test_traffic_summary_scales_by_the_copy(tmp_path):
    """The counter summary: per-dispatch means per kernel, each counter scaled
    by what it reads for the 1 GiB copy (here FETCH_SIZE reports half; the
    copy kernel's small dispatches are not the calibration)."""
    sys.path.insert(0, ROOT)
    import bench
    gib_kib = float(1 << 20)
    rows = {"FETCH_SIZE": [("__amd_rocclr_copyBuffer", gib_kib / 2), ("__amd_rocclr_copyBuffer", 3.0),
                           ("__amd_rocclr_copyBuffer", 5.0), ("void ewbem::k_far_vt<ewbem::cd, 1, 4>(x)", 100.0),
                           ("void ewbem::k_far_vt<ewbem::cd, 1, 4>(x)", 300.0), ("void ewbem::k_hmv<1>(y)", 1000.0),
                           ("ewbem::k_hmv_reduce(z)", 10.0)],
            "WRITE_SIZE": [("__amd_rocclr_copyBuffer", gib_kib), ("void ewbem::k_far_vt<ewbem::cd, 1, 4>(x)", 4.0),
                           ("void ewbem::k_hmv<1>(y)", 8.0), ("ewbem::k_hmv_reduce(z)", 2.0)]}
    dirs = []
    for c, rr in rows.items():
        d = tmp_path / c
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w") as f:
            f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            for i, (k, v) in enumerate(rr):
                f.write(f'{i},"{k}",{c},{v}\n')
        dirs.append(str(d))
    log = tmp_path / "run.log"
    log.write_text("# a progress line\n" + json.dumps({"metric": "m", "roofline": {
        "algorithmic_bytes_per_launch": 2000.0 * 1024}}) + "\n")
    out = bench.traffic_summary(dirs[0], dirs[1], str(tmp_path / "t.json"), str(log))
    assert abs(out["copy_calibration"]["fetch_scale"] - 2.0) < 1e-12
    assert abs(out["copy_calibration"]["write_scale"] - 1.0) < 1e-12
    k = out["kernels"]
    assert abs(k["far_vt"]["hbm_bytes"] - (200.0 * 2 + 4.0) * 1024) < 1e-6
    assert abs(out["hbm_bytes_per_matvec"] - ((200 * 2 + 4) + (1000 * 2 + 8) + (10 * 2 + 2)) * 1024) < 1e-6
    # reported only for the operator (algorithmic bytes) the counters were taken on
    assert out["algorithmic_bytes_per_launch"] == 2000.0 * 1024
    p = str(tmp_path / "t.json")
    assert bench.traffic_from_profiles(2000.0 * 1024 * 1.004, p) == out["hbm_bytes_per_matvec"]
    assert bench.traffic_from_profiles(2000.0 * 1024 * 1.02, p) is None
