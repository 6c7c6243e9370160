"""Host-side logic of bench.py (no GPU): the one-GPU contract and the
measured-traffic record it reads."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_blob_id_matches_git(tmp_path):
    import bench
    if subprocess.run(["git", "--version"], capture_output=True).returncode != 0:
        pytest.skip("git not available")
    src = "paper_1009_5300_amd/csrc/ops.hip"
    ref = subprocess.run(["git", "hash-object", os.path.join(ROOT, src)], capture_output=True, text=True).stdout
    assert bench._blob_id(src) == ref.strip()


def test_traffic_record_is_dropped_when_sources_change(tmp_path, monkeypatch):
    import bench
    src = "paper_1009_5300_amd/csrc/ops.hip"
    good = bench._blob_id(src)
    rec = tmp_path / "traffic.txt"
    rec.write_text(f"kernel_class = fft_planes\nhbm_bytes_per_launch = 123\nblob {src} = {good}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [src])
    assert bench._measured_traffic("fft_planes") == 123.0
    assert bench._measured_traffic("stencil") is None  # another kernel
    rec.write_text(f"kernel_class = fft_planes\nhbm_bytes_per_launch = 123\nblob {src} = {'0' * 40}\n")
    assert bench._measured_traffic("fft_planes") is None  # stale record
    rec.write_text(f"kernel_class = fft_planes\nhbm_bytes_per_solve = 300\nblob {src} = {good}\n")
    assert bench._measured_traffic("fft_planes", 15) == 20.0  # per-solve record, per launch
    assert bench._measured_traffic("fft_planes") is None  # no launch count to divide by
