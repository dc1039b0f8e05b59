"""bench.py's host-side contract (CPU): refusing more than one GPU, and reading measured
traffic only from a profile summary whose source digest matches the current sources."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_needs_matching_digest(tmp_path, monkeypatch):
    digest = bench.source_digest()
    assert len(digest) == 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    body = ("- fetch_bytes_per_launch: `100`\n- write_bytes_per_launch: `23`\n"
            f"- source_sha256: `{digest}`\n")
    (prof / "k_x_pmc.md").write_text(body)
    (prof / "k_y_pmc.md").write_text(body.replace(digest, "0" * 64))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_x", digest)["bytes"] == 123.0
    assert bench.measured_traffic("k_y", digest) is None
    assert bench.measured_traffic("k_missing", digest) is None
