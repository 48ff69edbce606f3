"""Tile layout of the fused RK4 kernel, checked on the host: the point ->
(x, y) decoding and the region prefix property the stage predicates rely on
(a C++ program built with hipcc from the kernel header; no GPU is used)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not installed")
def test_tile_layout(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = tmp_path / "tile_layout_check"
    src = os.path.join(HERE, "tile_layout_check.hip")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert "bad=0" in r.stdout
