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


def _source_hash() -> str:
    src = os.path.join(ROOT, "paper_2306_08623_amd", "csrc")
    return hashlib.sha256(open(os.path.join(src, "nd_peel.hip"), "rb").read() +
                          open(os.path.join(src, "nd_internal.h"), "rb").read()).hexdigest()


def _profile(path, digest: str) -> None:
    with open(path, "w") as f:
        f.write("traffic_bytes_per_launch k_peel<3,4> rmat18: 123456789\n")
        f.write("traffic_bytes_per_launch k_count_s4<3> rmat18: 987654321\n")
        f.write(f"peel source sha256 (nd_peel.hip + nd_internal.h) when measured: {digest}\n")


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "exactly one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_reported_for_matching_source(tmp_path, monkeypatch):
    prof = tmp_path / "profile.txt"
    _profile(prof, _source_hash())
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    assert bench.measured_traffic("k_peel", "rmat18", 3, 4) == 123456789
    assert bench.measured_traffic("k_count_s4", "rmat18", 3, 4) == 987654321
    assert bench.measured_traffic("k_hier", "rmat18", 3, 4) is None


def test_traffic_withheld_for_changed_source_or_other_workload(tmp_path, monkeypatch):
    prof = tmp_path / "profile.txt"
    _profile(prof, "0" * 64)
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    assert bench.measured_traffic("k_peel", "rmat18", 3, 4) is None
    _profile(prof, _source_hash())
    assert bench.measured_traffic("k_peel", "er2k", 3, 4) is None
    assert bench.measured_traffic("k_peel", "rmat18", 2, 3) is None
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("k_peel", "rmat18", 3, 4) is None
