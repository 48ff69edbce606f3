"""Pins of the oracle's random-number path: Philox4x32-10 words, the uniform
map, Box-Muller normals and the random-sphere initial state."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-o", exe,
                           os.path.join(HERE, "philox_rocrand_ref.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    """The oracle's Philox4x32-10 agrees bit for bit with rocRAND's
    independent implementation on random counters and keys (incl. extremes)."""
    r = np.random.default_rng(1)
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6]
    cases += r.integers(0, 2**32, size=(300, 6), dtype=np.uint64).tolist()
    inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True)
    ref = [list(map(int, ln.split())) for ln in out.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, want in zip(cases, ref):
        got = orc.philox4x32_10(c[:4], c[4:])
        assert got == want, (c, got, want)


def test_philox_stream_layout(orc):
    """philox_stream(seed, i0, n, c1, c2, c3) is the block for counter
    (i0+j, c1, c2, c3) with key (seed lo, seed hi)."""
    seed = 0x0123456789ABCDEF
    w = orc.philox_stream(seed, 7, 5, 3, 2, 1)
    for j in range(5):
        assert list(w[j]) == orc.philox4x32_10([7 + j, 3, 2, 1], [seed & 0xFFFFFFFF, seed >> 32])


def test_u01_open_interval_and_exact(orc):
    assert orc.u01(0) == 2.0**-33
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0**-33
    for w in [1, 12345, 2**31, 2**32 - 2]:
        assert orc.u01(w) == (w + 0.5) / 2**32


def test_gauss_statistics(orc):
    """Box-Muller normals: mean 0, variance 1, kurtosis 3, independent
    components, and a Kolmogorov-Smirnov test against N(0,1)."""
    n = 40000
    G = np.array([orc.gauss3(5, i, 3, 0, 0) for i in range(n)])
    assert abs(G.mean()) < 5 / np.sqrt(3 * n)
    assert abs(G.var() - 1) < 5 * np.sqrt(2 / (3 * n))
    assert abs(stats.kurtosis(G.ravel(), fisher=False) - 3) < 0.06
    cc = np.corrcoef(G.T)
    assert np.max(np.abs(cc - np.eye(3))) < 5 / np.sqrt(n)
    for c in range(3):
        assert stats.kstest(G[:, c], "norm").pvalue > 1e-4


def test_gauss_wiring(orc):
    """The three normals use (u0,u1) as one Box-Muller pair and (u2,u3) as the
    second pair's cosine branch, words taken from counter (i, k, r, tag)."""
    seed, i, k, r, tag = 99, 17, 4, 2, 0
    w = orc.philox4x32_10([i, k, r, tag], [seed, 0])
    u = [(x + 0.5) / 2**32 for x in w]
    want = [np.sqrt(-2 * np.log(u[0])) * np.cos(2 * np.pi * u[1]),
            np.sqrt(-2 * np.log(u[0])) * np.sin(2 * np.pi * u[1]),
            np.sqrt(-2 * np.log(u[2])) * np.cos(2 * np.pi * u[3])]
    np.testing.assert_allclose(orc.gauss3(seed, i, k, r, tag), want, rtol=1e-14, atol=1e-15)


def test_random_sphere_init(orc):
    """Random-sphere state: unit length, s_z = 2 u0 - 1 exactly from the tag-1
    words, and uniform on the sphere (z uniform on [-1,1], azimuth uniform)."""
    g = orc.geom((16, 16, 16))
    s = orc.init_random_sphere(g, seed=0)
    N = 16**3
    np.testing.assert_allclose(np.linalg.norm(s, axis=0), 1.0, atol=1e-15)
    w = orc.philox_stream(0, 0, N, 0, 0, 1)
    z = 2 * ((w[:, 0].astype(np.float64) + 0.5) / 2**32) - 1
    assert np.array_equal(s[2], z)
    assert stats.kstest(s[2], "uniform", args=(-1, 2)).pvalue > 1e-4
    ph = np.arctan2(s[1], s[0])
    assert stats.kstest(ph, "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-4
    # different replicas draw different states
    s1 = orc.init_random_sphere(g, seed=0, r=1)
    assert not np.allclose(s1, s)
