"""Host-side order of the fused kernel's tiles over the XCDs (tile_order.hpp):
built with g++ from tests/tile_order_check.cpp and run on the CPU.  Checks
that the workgroup mapping is a permutation with XCD k receiving the k-th
block of positions, that a batch's tiles are a permutation of the
replica-major list with each XCD's share exact, its tiles longest first and
its load within one replica of the mean, and, for the uneven 96-replica
workload, that whole replicas stay on one XCD and the modelled makespan
(32 CUs per XCD, list scheduling) drops from 144 to at most 128 planes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1610_04914_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_tile_order(tmp_path):
    exe = str(tmp_path / "tile_order_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-I", CSRC,
                    os.path.join(HERE, "tile_order_check.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
