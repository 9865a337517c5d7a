"""bench.py's command-line contract and its use of the committed traffic
summaries, checked without a GPU."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line


def test_measured_traffic_follows_the_committed_summary():
    v = bench.measured_traffic("k_cg_a<float, 4, 1, true, 1>")
    text = open(os.path.join(ROOT, "profiles", "mg_solve_c3_traffic.md")).read()
    src = "paper_1410_1937_amd/csrc/cg.hip"
    sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    fresh = f"source sha256 ({src}): {sha}" in text
    if fresh:
        assert v is not None and 1.0e9 <= v <= 1.3e9   # about 1.07x the 1.007e9 algorithmic bytes
    else:
        assert v is None                              # counters taken on another version of the kernel
    assert bench.measured_traffic("k_no_such_kernel<float>") is None


def test_stale_source_drops_the_traffic(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x_traffic.md").write_text(
        "source sha256 (bench.py): " + "0" * 64 + "\n"
        "traffic_bytes_per_launch k_demo<float>: 123\n"
        "kernel_source k_demo<float>: bench.py\n")
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    assert bench.measured_traffic("k_demo<float>") is None
    sha = hashlib.sha256(open(os.path.join(ROOT, "bench.py"), "rb").read()).hexdigest()
    (prof / "x_traffic.md").write_text(
        f"source sha256 (bench.py): {sha}\n"
        "traffic_bytes_per_launch k_demo<float>: 123\n"
        "kernel_source k_demo<float>: bench.py\n")
    assert bench.measured_traffic("k_demo<float>") == 123
