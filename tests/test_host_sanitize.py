"""The library's host code (split-and-merge and the work planner) under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: tests/host/
host_checks.cpp compiles segment.cpp and api.cpp as host C++ with g++ (the
kernel launchers are stubs; nothing is launched) and fuzzes segmentation and
plan construction, checking their invariants; any sanitizer report or failed
check ends it with a non-zero status."""

import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "host_checks.cpp")
ROCM = "/opt/rocm"


def test_host_code_under_sanitizers():
    gxx = shutil.which("g++")
    if not gxx or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "host_checks")
        cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-w", SRC, "-o", exe,
               f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-lpthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe, "600", "11"], capture_output=True, text=True, env=env,
                           timeout=600)
        out = r.stdout + r.stderr
        assert r.returncode == 0, out[-4000:]
        assert "0 failures" in out and "Sanitizer" not in out and "runtime error" not in out
