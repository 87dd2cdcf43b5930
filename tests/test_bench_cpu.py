"""The benchmark's command-line contract, without a GPU: one GPU only, and the JSON helpers."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr


def test_memory_roofline_fields():
    sys.path.insert(0, ROOT)
    import bench
    m = bench.memory_roofline(4.0e9, 20.0)
    assert m["algorithmic_gather_bytes_per_step"] == 384
    assert abs(m["algorithmic_gather_GBps"] - 4.0e9 * 384 / 0.020 / 1e9) < 1e-6
    d = bench._profile()
    if d is not None:  # counters taken on the current kernel source
        assert m["hbm_GBps"] > 0 and 0 < m["hbm_frac"] < 1
        assert bench._traffic_from_profile() == d["hbm_bytes_per_launch"]
    json.dumps(m)
