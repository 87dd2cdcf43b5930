"""The checked build (libpbr_checked.so: every device access of the trace kernels tested against
its buffer, a failed test counted and reported as PBR_ERR_BOUNDS) runs the whole GPU suite in a
child process: every parity test must pass with no access outside its buffer, in both field
layouts, with records, per-source sums, Mie weights, optical chains, source orders, batches, the
surrogate and the allocation-free entry point."""
import os
import subprocess
import sys

import pytest

from paper_1812_05902_amd import pbr

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_1812_05902_amd import pbr
lib = pbr.load(pbr.CHECKED_LIB_PATH)   # every later pbr.load() returns the checked build
assert lib.pbr_checked_build() == 1
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "gpu", "-x", "--timeout", "300",
                      "--timeout-method", "thread", "--ignore", sys.argv[2], sys.argv[3]]))
"""


def test_gpu_suite_on_the_checked_build():
    assert os.path.exists(pbr.CHECKED_LIB_PATH), "build libpbr_checked.so first (python -m paper_1812_05902_amd.build)"
    print("checked build: GPU suite in a child process", flush=True)
    r = subprocess.run([sys.executable, "-u", "-c", CHILD, ROOT, os.path.abspath(__file__), os.path.join(ROOT, "tests")],
                       capture_output=True, text=True, timeout=900, cwd=ROOT)
    tail = r.stdout[-3000:] + r.stderr[-3000:]
    print(tail)
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "failed" not in r.stdout


STEEP = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from paper_1812_05902_amd import inputs, pbr
lib = pbr.load(pbr.CHECKED_LIB_PATH)
assert lib.pbr_checked_build() == 1
n = 24
org, sp = (-0.012, -0.012, 0.113), (1e-3, 1e-3, 1e-3)
base = inputs.tiny_bos().replace(nx=n, ny=n, nz=n, origin=org, spacing=sp, rays_per_src=32)
rng = np.random.default_rng(7)
# (1) node-to-node noise up to 500 kg/m^3 (n - 1 up to 0.11, |grad n| ~ 100 / m: a step of one cell
# bends ~0.05 cells off its straight line); (2) a jump 1.2 -> 500 kg/m^3 across one cell at x = 0
noise = (1.2 + 500.0 * rng.random((n, n, n))).astype(np.float32)
jump = np.full((n, n, n), 1.2, np.float32)
jump[:, :, n // 2:] = 500.0
# particles inside the box and dots in front of it
inside = np.zeros((3000, 4), np.float32)
inside[:, :3] = np.asarray(org) + rng.random((3000, 3)) * (n - 1) * np.asarray(sp)
inside[:, 3] = 1.0
dots = inputs.sources(base.replace(n_src=3000))
runs = 0
for name, rho in (("noise", noise), ("jump", jump)):
    for nodes in (False, True):
        for ds in (1e-3, 2.5e-3, 3e-4):
            for flags in (0, pbr.PBR_PREC_FP64_ALL, pbr.PBR_PREC_SHOCK_FP64, pbr.PBR_LANE_REFILL):
                if nodes and flags == pbr.PBR_LANE_REFILL:
                    continue
                for src in (inside, dots):
                    r = pbr.Renderer.from_scene(base, rho=rho, nodes=nodes)
                    if flags == pbr.PBR_PREC_SHOCK_FP64:   # calibration traces the steep bricks too
                        rep = r.calibrate_precision(ds, tol_px=1e-6, steep_frac=0.1, rays_per_brick=64)
                        assert rep["n_steep"] > 0
                    r.set_exit_recording(0, 7, 1 << 14)
                    st = r.emit_and_trace(src, 32, 11, ds, flags | pbr.PBR_CLEAR_FIRST | pbr.PBR_RECORD_EXITS,
                                          stats=True)   # raises on PBR_ERR_BOUNDS
                    assert st["rays"] == len(src) * 32 and sum(st["status"]) == st["rays"]
                    runs += 1
    print(name, "ok", flush=True)
print("runs", runs)
"""


def test_steep_fields_stay_in_bounds_on_the_checked_build():
    """Fields far steeper than any workload (per-node noise up to 500 kg/m^3, a 1.2 -> 500 kg/m^3
    jump across one cell) with steps of 0.3, 1 and 2.5 cells, sources inside and in front of the
    box, both layouts, FP32, FP64, calibrated mixed precision and lane refill: paths bend far more
    than the face margin the integration assumes, and every device access must still stay inside
    its buffer."""
    assert os.path.exists(pbr.CHECKED_LIB_PATH)
    print("checked build: steep fields in a child process", flush=True)
    r = subprocess.run([sys.executable, "-u", "-c", STEEP, ROOT], capture_output=True, text=True, timeout=600,
                       cwd=ROOT)
    tail = r.stdout[-3000:] + r.stderr[-3000:]
    print(tail)
    assert r.returncode == 0, tail
    assert "runs 84" in r.stdout


BAD_ORDER = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import torch
from paper_1812_05902_amd import inputs, pbr
lib = pbr.load(pbr.CHECKED_LIB_PATH)
assert lib.pbr_checked_build() == 1
sc = inputs.tiny_bos().replace(n_src=40, rays_per_src=16)
r = pbr.Renderer.from_scene(sc)
src = inputs.sources(sc)
flags = pbr.PBR_CLEAR_FIRST | pbr.PBR_SOURCE_ORDER
good = torch.arange(sc.n_src - 1, -1, -1, dtype=torch.int64, device=r.device)
pbr.pbr_set_source_order(r.ctx, good, sc.n_src)
r.emit_and_trace(src, sc.rays_per_src, 5, sc.ds, flags)
img = pbr.u64_image_to_numpy(r.read_image())
assert img.sum() > 0
bad = good.clone()
bad[3] = sc.n_src + 7   # no source index: clamped on every build, counted on this one
bad[9] = -2
pbr.pbr_set_source_order(r.ctx, bad, sc.n_src)
try:
    r.emit_and_trace(src, sc.rays_per_src, 5, sc.ds, flags)
except pbr.PbrError as e:
    assert e.code == pbr.PBR_ERR_BOUNDS, e
    assert "outside their buffers" in str(e), e
    # the rays of the two bad entries, counted where emission and the finish look up their keys
    n = int(str(e).split("checked build: ")[1].split()[0])
    assert n > 0 and n % (2 * sc.rays_per_src) == 0, n
    print("reported:", e, flush=True)
else:
    raise SystemExit("no PBR_ERR_BOUNDS for an order entry outside [0, n_src)")
# the context stays usable: a valid order traces cleanly again, to the same image
pbr.pbr_set_source_order(r.ctx, good, sc.n_src)
r.emit_and_trace(src, sc.rays_per_src, 5, sc.ds, flags)
assert np.array_equal(pbr.u64_image_to_numpy(r.read_image()), img)
print("bad order ok", flush=True)
"""


def test_checked_build_reports_an_order_entry_outside_the_sources():
    """The checked build's report path end to end: a source order with two entries that are no
    source index (the kernels clamp them on every build) makes the trace return PBR_ERR_BOUNDS
    with the count in the message; the same context then traces a valid order cleanly."""
    assert os.path.exists(pbr.CHECKED_LIB_PATH)
    print("checked build: invalid order entries in a child process", flush=True)
    r = subprocess.run([sys.executable, "-u", "-c", BAD_ORDER, ROOT], capture_output=True, text=True, timeout=300,
                       cwd=ROOT)
    tail = r.stdout[-3000:] + r.stderr[-3000:]
    print(tail)
    assert r.returncode == 0, tail
    assert "bad order ok" in r.stdout


SAME_BITS = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from paper_1812_05902_amd import inputs, pbr
lib = pbr.load(pbr.CHECKED_LIB_PATH)
assert lib.pbr_checked_build() == 1
out = {}
for nodes in (False, True):
    sc = inputs.tiny_bos()
    r, st, _ = pbr.trace_scene(sc, nodes=nodes)
    out[f"img{int(nodes)}"] = pbr.u64_image_to_numpy(r.read_image())
np.savez(sys.argv[2], **out)
print("checked images written", flush=True)
"""


def test_checked_build_renders_the_same_bits(tmp_path):
    """The checked build only adds tests: the tiny BOS image in both field layouts is the same bit
    for bit from both libraries (the regular one in this process, the checked one in a child)."""
    import numpy as np
    from paper_1812_05902_amd import inputs
    path = tmp_path / "checked.npz"
    r = subprocess.run([sys.executable, "-u", "-c", SAME_BITS, ROOT, str(path)], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    got = np.load(path)
    for nodes in (False, True):
        rr, _, _ = pbr.trace_scene(inputs.tiny_bos(), nodes=nodes)
        mine = pbr.u64_image_to_numpy(rr.read_image())
        assert mine.sum() > 0
        assert np.array_equal(got[f"img{int(nodes)}"], mine), nodes
