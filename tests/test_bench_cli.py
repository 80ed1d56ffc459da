"""The benchmark's command-line contract on a machine without a GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_is_well_formed():
    path = os.path.join(ROOT, "profiles", "dalm_iteration_traffic.json")
    rec = json.load(open(path))
    assert len(rec["kernel_source_sha256"]) == 64
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    assert all(v > 0 for v in rec["hbm_bytes_per_launch_at_workload"].values())


def test_every_workload_leg_is_offered():
    sys.path.insert(0, ROOT)
    import bench
    offered = set(bench.WORKLOADS) | set(bench.E1_WORKLOADS) | set(bench.ALIGN_WORKLOADS) \
        | set(bench.QP_WORKLOADS) | set(bench.UNROLLED_WORKLOADS)
    assert bench.DEFAULT_WORKLOAD in bench.WORKLOADS
    assert {"cab-1200x700-n512", "cab-4800x2100-n2048", "align-1200x11-n1000", "qp-2000x8000-n64",
            "unrolled-1200x700-n256", "e1-800x1000-d100"} <= offered
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for name in offered:
        assert name in r.stdout
    for method in ("dalm", "palm", "adm", "dalm_cg1"):
        assert method in r.stdout

