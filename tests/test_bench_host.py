"""Host-side checks of the benchmark script (no GPU): the one-GPU guard and the
rule that the HBM traffic figure comes only from a counter summary taken on the
current kernel source."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_needs_the_current_kernel_source(tmp_path, monkeypatch):
    sha = bench.kernel_sha()
    assert len(sha) == 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    summary = prof / "grid_step_fused4096_counters.md"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile(sha) is None  # no summary
    summary.write_text(f"kernel_source_sha256: {sha}\nhbm_bytes_per_launch: 1206524918\n")
    assert bench.traffic_from_profile(sha) == 1206524918.0
    assert bench.traffic_from_profile("0" * 64) is None  # taken on other source
