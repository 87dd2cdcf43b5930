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
