"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C++ sources
of the C ABI (argument and state validation, derived optics, the paraxial system matrix, the host
Mie series, workspace planning, the batch and surrogate front ends) are rebuilt with both
sanitizers on their host pass only, linked with the regular objects of the HIP sources into a
second copy of the library, and the CPU ABI tests run against that copy in a child process whose
first loaded library is the sanitizer runtime.  Every report is fatal.  A second child writes past
the end of a host buffer through the library, so the test also shows that the instrumentation is
live."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1812_05902_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# host pass only: the device code of the .hip sources is not instrumented (no GPU sanitizer here)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]

RUN_TESTS = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_1812_05902_amd import pbr
pbr.load(sys.argv[2])          # every later pbr.load() returns this copy
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu", sys.argv[3]]))
"""

OVERRUN = r"""
import ctypes as C, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_1812_05902_amd import pbr
lib = pbr.load(sys.argv[2])
out = np.zeros(64)
m = pbr.mie_params(1e-6, 1.47, 532e-9, (1, 0, 0))
# n says 512 doubles, the buffer holds 64: the library writes past its end
lib.pbr_mie_table(C.byref(m), 1.0, out.ctypes.data_as(C.c_void_p), 512)
print("no report")
"""


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    try:
        hipcc = build._hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("the clang AddressSanitizer runtime is not installed")
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("LD_PRELOAD is already set; the sanitizer runtime must be the first library loaded")
    hip_srcs = [s for s in build.SOURCES if s.endswith(".hip")]
    host_srcs = [s for s in build.SOURCES if s.endswith(".cpp")]
    if not all(os.path.exists(os.path.join(build.BUILD, s[:-4] + ".o")) for s in hip_srcs):
        build.build()
    out = tmp_path_factory.mktemp("san")

    def compile_one(src):
        obj = str(out / (os.path.splitext(src)[0] + ".o"))
        r = subprocess.run([hipcc, "-x", "hip", *build.HIPCC_FLAGS, *SAN, "-c", os.path.join(build.CSRC, src),
                            "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, host_srcs))
    objs += [os.path.join(build.BUILD, s[:-4] + ".o") for s in hip_srcs]
    lib = str(out / "libpbr_sanitized.so")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined", "-shared-libasan", *objs, "-o", lib],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return lib, env


def test_cpu_abi_suite_under_sanitizers(sanitized_lib):
    lib, env = sanitized_lib
    r = subprocess.run([sys.executable, "-c", RUN_TESTS, ROOT, lib, os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       capture_output=True, text=True, env=env, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout and "failed" not in r.stdout, r.stdout[-2000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]


def test_instrumentation_is_live(sanitized_lib):
    lib, env = sanitized_lib
    r = subprocess.run([sys.executable, "-c", OVERRUN, ROOT, lib], capture_output=True, text=True, env=env,
                       timeout=300, cwd=ROOT)
    assert r.returncode != 0 and "no report" not in r.stdout
    assert "heap-buffer-overflow" in r.stderr and "pbr_mie_table" in r.stderr, r.stderr[-4000:]
