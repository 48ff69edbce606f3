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
    f.write_text("kernel_sources_hash: deadbeef0000\nl2_fabric_bytes_per_launch: 1.0e8\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() is None
    f.write_text(f"kernel_sources_hash: {bench.kernel_hash()}\nl2_fabric_bytes_per_launch: 1.0e8\n")
    assert bench.measured_traffic() == 1.0e8


def test_oracle_all_cores_build_is_identical():
    """The OpenMP build that times the oracle on all host cores computes the
    same states as the single-threaded build the tests use."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import oracle as orc
    g = orc.geom((12, 10, 9), "free")
    p = orc.Params(J=1.0, H=(0.0, 0.1, 0.2), D=0.1, e=(1.0, 0.0, 1.0), lam=0.05, T=1.0,
                   dt=0.1, Dt=0.4)
    s = orc.init_random_sphere(g, 3)
    assert np.array_equal(orc.step(g, p, s, 3), orc.step(g, p, s, 3, all_cores=True))


def test_sign_test_p_values():
    """The batched accuracy sign test: exact two-sided binomial p at 1/2,
    checked against closed forms (all heads in n: 2 / 2^n) and symmetry."""
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    assert bench._binom_two_sided(0, 5) == 2.0 / 32
    assert bench._binom_two_sided(5, 5) == 2.0 / 32
    assert bench._binom_two_sided(2, 4) == 1.0
    for n in (7, 61, 96):
        for k in range(n + 1):
            assert bench._binom_two_sided(k, n) == bench._binom_two_sided(n - k, n)
    # n = 10, k = 2: P(X <= 2) + P(X >= 8) = 2 * (1 + 10 + 45) / 1024
    assert abs(bench._binom_two_sided(2, 10) - 112 / 1024) < 1e-15
