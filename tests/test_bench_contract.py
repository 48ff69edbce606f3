"""Host-side checks of bench.py's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rejects_multi_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_null_when_kernel_changed(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    f = tmp_path / "t.md"
    f.write_text("kernel_sources_hash: deadbeef0000\nhbm_bytes_per_launch: 1.0e8\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() is None
    f.write_text(f"kernel_sources_hash: {bench.kernel_hash()}\nhbm_bytes_per_launch: 1.0e8\n")
    assert bench.measured_traffic() == 1.0e8
