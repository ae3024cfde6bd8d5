"""bench.py contract checks that need no GPU: one GPU only, the CPU-oracle
baseline leg's fields, and that the committed HBM-traffic profiles were taken
on the current kernel sources (else the bench line's roofline.traffic is
null)."""
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
    b = bench.cpu_baseline(budget_s=0.5)
    assert b["kind"] == "oracle" and b["unit"] == "MNUPS"
    assert b["value"] > 0 and b["cores"] >= 1
    assert "1024x64x8" in b["sample"]


def test_committed_traffic_profiles_match_the_kernel_sources():
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as fh:
        rec = json.load(fh)
    assert bench.HEADLINE in rec
    for name, r in rec.items():
        assert r["kernel_hash"] == bench.kernel_hash(), name
        assert r["bytes_per_launch"] >= r["algorithmic_bytes_per_launch"]
    assert bench.traffic_for(bench.HEADLINE, 0) == rec[bench.HEADLINE]["bytes_per_launch"]
