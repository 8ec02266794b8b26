"""Builds libsncc.so (HIP for gfx950) in place, next to this file.

    python paper_2502_01286_amd/build.py

Each translation unit is compiled to an object with hipcc, then linked into
one shared library.  Floating point is compiled without contraction so the
compensated summation is kept as written; packed FP32 instructions are
disabled.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsncc.so")
PROBE = os.path.join(HERE, "lds_probe")  # LDS bandwidth probe (a program of its own)
ARCH = os.environ.get("SNCC_OFFLOAD_ARCH", "gfx950")

# (source, extra flags, object name): the scoring kernel's tile shapes are
# separate objects built from one source so that they compile in parallel.
N_TILE_SHAPES = 6
SOURCES = [("segment.cpp", [], "segment.o"), ("api.cpp", [], "api.o"),
           ("kernels.hip", [], "kernels.o"), ("fused_kernel.hip", [], "fused_kernel.o")] + [
    ("tile_entry.hip", [f"-DSNCC_TILE_ENTRY_ID={i}"], f"tile_entry_{i}.o")
    for i in range(N_TILE_SHAPES)]

PROBE_SRC = os.path.join(CSRC, "lds_probe.hip")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-x", "hip", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    tmp = tempfile.mkdtemp(prefix="sncc_build_")
    try:
        def compile_one(job):
            src, extra, name = job
            obj = os.path.join(tmp, name)
            cmd = [hipcc, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
            return obj
        def build_probe():
            # the LDS bandwidth probe: a separate program, not linked into the library
            cmd = [hipcc, "-O3", "-std=c++17", "-x", "hip", f"--offload-arch={ARCH}",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", PROBE_SRC,
                   "-o", PROBE + ".tmp"]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compiling lds_probe.hip failed:\n{r.stdout}\n{r.stderr}")
            os.replace(PROBE + ".tmp", PROBE)
        with ThreadPoolExecutor(max_workers=min(len(SOURCES) + 1, os.cpu_count() or 4, 16)) as ex:
            probe = ex.submit(build_probe)
            objs = list(ex.map(compile_one, SOURCES))
            probe.result()
        out_tmp = LIB + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"linking failed:\n{r.stdout}\n{r.stderr}")
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
