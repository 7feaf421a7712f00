"""Host-side pieces of bench.py: the one-GPU guard and the oracle timing legs."""
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


def test_cpu_pool_baseline_counts_updates_done():
    out = bench.cpu_pool_baseline(sample_runs=2, lups_per_run=2e5)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS"
    assert 1 <= out["cores"] <= 16
    assert out["value"] > 0
    assert "2 of the 256 batched flat-interface runs" in out["sample"]
