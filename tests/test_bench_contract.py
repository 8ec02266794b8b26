"""Host-side parts of the benchmark's contract (no GPU): one GPU only, and the
HBM traffic figure is taken from a counter summary only when it was measured
on the current scoring-kernel sources."""

import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_used_only_on_matching_sources(tmp_path, monkeypatch):
    bench = _bench_module()
    current = bench.kernel_source_hash()
    assert len(current) == 16 and int(current, 16) >= 0
    # the hash covers the kernel sources themselves
    os.makedirs(tmp_path / "paper_2502_01286_amd" / "csrc")
    for name in bench.KERNEL_SOURCES:
        src = os.path.join(ROOT, "paper_2502_01286_amd", "csrc", name)
        with open(src, "rb") as fh, open(tmp_path / "paper_2502_01286_amd" / "csrc" / name,
                                          "wb") as out:
            out.write(fh.read())
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == current
    path = tmp_path / "profiles" / "tile_kernel_demo_traffic.txt"
    path.write_text(f"# comment: ignored\nkernel_sources_sha256_16: {current}\n"
                    "bytes_per_launch: 1000\nscoring_stage_bytes: 1234\n")
    assert bench.load_traffic("demo") == 1234
    path.write_text(f"kernel_sources_sha256_16: {current}\nbytes_per_launch: 1000\n")
    assert bench.load_traffic("demo") == 1000
    path.write_text("kernel_sources_sha256_16: 0000000000000000\nscoring_stage_bytes: 1234\n")
    assert bench.load_traffic("demo") is None
    assert bench.load_traffic("missing") is None
    # an edited kernel source invalidates the summary
    path.write_text(f"kernel_sources_sha256_16: {current}\nscoring_stage_bytes: 1234\n")
    with open(tmp_path / "paper_2502_01286_amd" / "csrc" / bench.KERNEL_SOURCES[0], "ab") as fh:
        fh.write(b"\n")
    assert bench.load_traffic("demo") is None
