"""Host-side logic of bench.py (no GPU): the one-GPU guard and the gate on
the committed HBM-traffic record (used only while the apply kernel source
is the one the counters were taken on)."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    rec = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in json.dumps(rec) or "--gpus 1" in json.dumps(rec)


def test_traffic_record_matches_the_apply_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["lognormal160_bsr3"]
    src = os.path.join(ROOT, "paper_2508_04917_amd", "csrc", "apply.hip")
    if rec["apply_source_sha"] != bench.source_sha(src):
        pytest.skip("apply source changed since the counters were taken: the bench reports traffic null")
    assert bench.measured_traffic("lognormal160_bsr3", [16, 20, 20]) == rec["bytes_per_apply"]
    # the record belongs to one workload and partition only
    assert bench.measured_traffic("lognormal160_bsr3", [16, 16, 20]) is None
    assert bench.measured_traffic("aniso160_bsr3", [16, 20, 20]) is None
    # scaled counters: FETCH_SIZE x scale + WRITE_SIZE, KiB per dispatch
    b = (rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] + rec["write_kib_per_dispatch"]) * 1024
    assert abs(b - rec["bytes_per_apply"]) / rec["bytes_per_apply"] < 1e-4
