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


def test_flop_counts_per_layout():
    """The method's FP32 operations per step: 3 evaluations of D (trilinear interpolation of four
    quantities, 14 operations each from cell coefficients or 21 from corners, plus 4) and 69 for
    the stage points and updates of eqs. 3 and 5."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.FLOPS_PER_STEP == {"cells": 3 * (4 * 14 + 4) + 69, "nodes": 3 * (4 * 21 + 4) + 69}


def test_cpu_baseline_reports_all_and_one_core():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1812_05902_amd import inputs
    sc = inputs.tiny_bos().replace(n_src=64, rays_per_src=20)
    b = bench.cpu_baseline(sc, inputs.density(sc), inputs.sources(sc), target_s=0.2, single_s=0.1)
    assert b["kind"] == "oracle" and b["unit"] == "rays/s" and b["value"] > 0 and b["cores"] >= 1
    assert b["single_core"]["value"] > 0 and "1 thread" in b["single_core"]["sample"]
    assert b["nproc"] >= 1 and isinstance(b["cpu_model"], str)
    json.dumps(b)


def test_default_workload_is_the_tomo_piv_image():
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--workload", default="tomo_piv_512"' in src
