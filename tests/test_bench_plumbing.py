"""Host-side plumbing of bench.py (no GPU): the multi-GPU refusal and the
measured-traffic lookup, which reports the committed counter figures only
while the peel kernel's source is the one they were taken from."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _source_hash(kernel: str) -> str:
    src = os.path.join(ROOT, "paper_2306_08623_amd", "csrc")
    first = {"k_peel": "nd_peel_kern.h", "k_count_s4": "nd_count.hip"}[kernel]
    return hashlib.sha256(open(os.path.join(src, first), "rb").read() +
                          open(os.path.join(src, "nd_internal.h"), "rb").read()).hexdigest()


def _profile(dirpath, workload: str, peel_digest: str, count_digest: str) -> None:
    with open(os.path.join(dirpath, f"k_peel_{workload}_34.txt"), "w") as f:
        f.write(f"traffic_bytes_per_launch k_peel<3,4> {workload} source {peel_digest}: 123456789\n")
        f.write(f"traffic_bytes_per_launch k_count_s4<3,4> {workload} source {count_digest}: "
                "987654321\n")


def _use_dir(monkeypatch, d):
    monkeypatch.setattr(bench, "profile_path",
                        lambda k, w, r, s: os.path.join(str(d), f"{k}_{w}_{r}{s}.txt"))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "exactly one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_reported_for_matching_source(tmp_path, monkeypatch):
    _profile(tmp_path, "chunglu4m", _source_hash("k_peel"), _source_hash("k_count_s4"))
    _use_dir(monkeypatch, tmp_path)
    assert bench.measured_traffic("k_peel", "chunglu4m", 3, 4) == 123456789
    assert bench.measured_traffic("k_count_s4", "chunglu4m", 3, 4) == 987654321
    assert bench.measured_traffic("k_hier", "chunglu4m", 3, 4) is None


def test_traffic_withheld_for_changed_source_or_other_workload(tmp_path, monkeypatch):
    _use_dir(monkeypatch, tmp_path)
    _profile(tmp_path, "chunglu4m", "0" * 64, "0" * 64)
    assert bench.measured_traffic("k_peel", "chunglu4m", 3, 4) is None
    assert bench.measured_traffic("k_count_s4", "chunglu4m", 3, 4) is None
    _profile(tmp_path, "chunglu4m", _source_hash("k_peel"), _source_hash("k_count_s4"))
    assert bench.measured_traffic("k_peel", "rmat18", 3, 4) is None
    assert bench.measured_traffic("k_peel", "chunglu4m", 2, 3) is None


def test_cpu_sample_is_the_benched_generator_scaled_down():
    g, what = bench.cpu_sample("chunglu4m", 8)
    assert g.n == 4_000_000 >> 8
    assert "exponent 2.1" in what and "communities" in what
