"""Builds libpbr.so (the HIP kernels and the C ABI of include/pbr.h) in-tree with hipcc for gfx950.

Usage: ``python -m paper_1812_05902_amd.build``.  Compiles every time it is called.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpbr.so")
# the checked build: the same library with index tests on the device accesses of the trace kernels
CHECKED_LIB = os.path.join(HERE, "libpbr_checked.so")
CHECKED_SOURCES = ["trace.hip", "pbr_api.cpp", "pbr_batch.cpp"]

SOURCES = ["field_prep.hip", "trace.hip", "readout.hip", "mlp.hip", "probe.hip", "bos_map.hip", "piv_pair.hip",
           "pbr_api.cpp", "pbr_mie.cpp", "pbr_batch.cpp", "pbr_surrogate.cpp", "pbr_noalloc.cpp", "source_order.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    # packed-FP32 instructions stay off (they are generated from plain float code otherwise)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Builds libpbr.so and the checked build libpbr_checked.so; returns the path of the first."""
    checked_dir = os.path.join(BUILD, "checked")
    os.makedirs(checked_dir, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(job):
        src, checked = job
        obj = os.path.join(checked_dir if checked else BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, "-x", "hip", *HIPCC_FLAGS, *(["-DPBR_CHECKED=1"] if checked else []),
               "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    # the two trace.hip compiles take most of the time: start them first
    jobs = [("trace.hip", False), ("trace.hip", True)]
    jobs += [(s, False) for s in SOURCES if s != "trace.hip"] + [(s, True) for s in CHECKED_SOURCES if s != "trace.hip"]
    with ThreadPoolExecutor(max_workers=max(2, min(8, os.cpu_count() or 1))) as ex:
        built = dict(zip(jobs, ex.map(compile_one, jobs)))
    regular = [built[(s, False)] for s in SOURCES]
    checked = [built[(s, s in CHECKED_SOURCES)] for s in SOURCES]
    for objs, lib in ((regular, LIB), (checked, CHECKED_LIB)):
        tmp = lib + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
