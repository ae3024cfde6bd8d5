"""bench.py contract checks that need no GPU: one GPU only, the CPU-oracle
baseline leg's fields, and that HBM-traffic profiles reach the bench line
only when they were taken on the current kernel sources (else the line's
roofline.traffic is null)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_baseline_reports_the_oracle_sample():
    b = bench.cpu_baseline(reps=3, steps_per_rep=1, warmup=1)
    assert b["kind"] == "oracle" and b["unit"] == "MNUPS"
    assert b["value"] > 0 and b["cores"] >= 1
    assert "1024x64x8" in b["sample"] and "median of 3" in b["sample"]


def test_traffic_is_reported_only_from_profiles_of_the_current_kernel_sources():
    """A committed counter record is used for the bench line's roofline.traffic
    only while its kernel hash is that of the current sources; else the
    traffic is null."""
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as fh:
        rec = json.load(fh)
    assert bench.HEADLINE in rec
    for name, r in rec.items():
        assert r["bytes_per_launch"] >= r["algorithmic_bytes_per_launch"], name
        got = bench.traffic_for(name, 0)
        if r["kernel_hash"] == bench.kernel_hash():
            assert got == r["bytes_per_launch"], name
        else:
            assert got is None, name
