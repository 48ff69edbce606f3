"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (max abs difference per spin component; spins are unit vectors,
so absolute = relative): 1e-12 for fp64, 1e-5 for fp32, per step-segment,
starting the oracle from the GPU's own state (chaotic dynamics forbids whole
trajectory comparisons).  Random words and the sphere's z component are
compared bit for bit.  Observables: relative 1e-12 (fp64 reductions).
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as orc
from tests import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def P():
    import paper_1610_04914_amd as P
    P.lib()
    assert torch.cuda.is_available()
    return P


def np_state(lat):
    torch.cuda.synchronize()
    return lat.state.double().cpu().numpy()


def make_lattice(P, shape, bc, prec, s0):
    dt = torch.float64 if prec == "fp64" else torch.float32
    t = torch.tensor(np.asarray(s0), dtype=dt, device="cuda")
    return P.Lattice(shape, bc=bc, precision=prec, state=t)


def rounded(s, prec):
    return s.astype(np.float32).astype(np.float64) if prec == "fp32" else s.copy()


PHYS = {
    "axis": dict(J=1.0, H=(0.1, -0.2, 0.3), D=0.4, e=(1.0, 2.0, 2.0), lam=0.05, T=0.7),
    "zaxis": dict(J=1.0, H=(0.0, 0.0, 0.1), D=0.05, e=(0.0, 0.0, 1.0), lam=0.01, T=1.0),
    "none": dict(J=0.8, H=(0.0, 0.3, 0.0), D=0.0, lam=0.02, T=0.5),
}


def both_params(kind, dt=0.1, Dt=0.4, precession=True, seed=11, **over):
    kw = dict(PHYS[kind])
    kw.update(over)
    gp = dict(kw, dt=dt, Dt=Dt, precession=precession)
    return orc.Params(**gp), __import__("paper_1610_04914_amd").Params(seed=seed, **gp)


def variants(P, prec):
    return P.step_variants(prec)


# ------------------------------------------------------------------- RNG ----
@pytest.mark.parametrize("seed,i0,c1,c2,c3", [(0, 0, 0, 0, 0), (12345, 7, 3, 2, 1),
                                              (2**64 - 1, 2**32 - 100, 2**32 - 1, 5, 1),
                                              (0xDEADBEEFCAFEF00D, 1000, 17, 95, 0)])
def test_philox_words_bitexact(P, seed, i0, c1, c2, c3):
    n = 5000
    out = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
    P.lll_philox4x32_10(seed, i0, n, c1, c2, c3, out.data_ptr(), P._stream())
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).reshape(n, 4)
    want = orc.philox_stream(seed, i0, n, c1, c2, c3)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (7, 5, 3)])
def test_init_random_sphere(P, prec, shape):
    lat = P.Lattice(shape, precision=prec, init="random", seed=42)
    got = np_state(lat)
    want = orc.init_random_sphere(orc.geom(shape), 42, 0)
    if prec == "fp64":
        assert np.array_equal(got[2], want[2])            # z = 2u - 1 is exact
        np.testing.assert_allclose(got[:2], want[:2], rtol=0, atol=4e-16)
    else:
        np.testing.assert_allclose(got, want, rtol=0, atol=1.5e-7)
    lat2 = P.Lattice(shape, precision=prec, init="direction", direction=(1.0, 2.0, 2.0))
    np.testing.assert_allclose(np_state(lat2), np.array([[1 / 3], [2 / 3], [2 / 3]]) * np.ones((1, lat2.N)),
                               atol=1e-7)


# ------------------------------------------------------------------ steps ---
STEP_SHAPES = [((40, 24, 20), "periodic", 7), ((40, 24, 20), "free", 0), ((17, 5, 3), "periodic", 0),
               ((3, 3, 3), "periodic", 0), ((2, 3, 5), "free", 2), ((1, 1, 1), "periodic", 0),
               ((2, 2, 2), "periodic", 0), ((33, 17, 9), "periodic", 4),
               ((40, 36, 1), "periodic", 0), ((7, 1, 1), "free", 0), ((1, 9, 2), "periodic", 0)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,precession", [("axis", True), ("zaxis", True), ("none", True),
                                             ("zaxis", False)])
def test_step_parity_all_variants(P, prec, kind, precession):
    op, gp = both_params(kind, precession=precession)
    for shape, bc, bz in STEP_SHAPES:
        N = int(np.prod(shape))
        s0 = rounded(inputs.unit_spins(N, 100 + N), prec)
        want = orc.step(orc.geom(shape, bc), op, s0, 3)
        for v in variants(P, prec):
            lat = make_lattice(P, shape, bc, prec, s0)
            lat.set_step_config(v, bz)
            lat.step(gp, 3)
            got = np_state(lat)
            err = np.max(np.abs(got - want))
            assert err < TOL[prec], (shape, bc, v, bz, err)
            lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_site_anisotropy(P, prec):
    shape = (12, 10, 9)
    N = 1080
    D, e = inputs.site_anisotropy(N, 5)
    s0 = rounded(inputs.unit_spins(N, 6), prec)
    Dr, er = rounded(D[None, :], prec)[0], rounded(e, prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Dt_ = torch.tensor(Dr, dtype=dt, device="cuda")
    et = torch.tensor(er, dtype=dt, device="cuda")
    op = orc.Params(J=1.0, H=(0, 0, 0.2), lam=0.01, T=0.5, dt=0.1, Dt=0.2, D_site=Dr, e_site=er)
    gp = P.Params(J=1.0, H=(0, 0, 0.2), lam=0.01, T=0.5, dt=0.1, Dt=0.2, D_site=Dt_, e_site=et,
                  seed=3)
    lat = make_lattice(P, shape, "periodic", prec, s0)
    lat.run(gp, first_pulse=0, n_pulses=2)
    want, _, _ = orc.run(orc.geom(shape), op, s0, seed=3, n_pulses=1)
    want, _, _ = orc.run(orc.geom(shape), op, want, seed=3, first_pulse=1, n_pulses=1)
    # two intervals of two steps: still one short segment
    assert np.max(np.abs(np_state(lat) - want)) < 4 * TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["rk4", "rk2mid", "rk5b"])
def test_site_anisotropy_fused_all_variants(P, prec, method):
    """Per-site D_i along per-site axes e_i on the fused steps (every tile shape,
    periodic and free, an odd lattice, z-chunks that leave a ragged last
    chunk): three steps against the oracle's stepper, and one interval with
    the kick as the epilogue and as its own launch."""
    dt_ = torch.float64 if prec == "fp64" else torch.float32
    for shape, bc, bz in (((33, 17, 9), "periodic", 4), ((40, 24, 20), "free", 7),
                          ((12, 10, 9), "periodic", 0)):
        N = int(np.prod(shape))
        D, e = inputs.site_anisotropy(N, 11 + N)
        D, e = rounded(D[None, :], prec)[0], rounded(e, prec)
        s0 = rounded(inputs.unit_spins(N, 12 + N), prec)
        kw = dict(J=1.0, H=(0.05, 0.0, 0.2), lam=0.02, T=0.7, dt=0.1, Dt=0.5)
        op = orc.Params(D_site=D, e_site=e, **kw)
        gp = P.Params(D_site=torch.tensor(D, dtype=dt_, device="cuda"),
                      e_site=torch.tensor(e.reshape(-1), dtype=dt_, device="cuda"), seed=17,
                      integrator=method, **kw)
        g = orc.geom(shape, bc)
        want3 = orc.step(g, op, s0, 3, method=method)
        wantI = orc.step(g, op, s0, 2, method=method)
        wantI, _ = orc.kick(g, op, wantI, op.T, seed=17, r=0, k=4)
        wantI = orc.step(g, op, wantI, 3, method=method)
        for v in variants(P, prec):
            lat = make_lattice(P, shape, bc, prec, s0)
            lat.set_step_config(v, bz)
            lat.step(gp, 3)
            err = np.max(np.abs(np_state(lat) - want3))
            assert err < TOL[prec], (shape, bc, v, bz, err)
            lat.close()
            for fused in (True, False):
                lat = make_lattice(P, shape, bc, prec, s0)
                lat.set_step_config(v, bz)
                lat.set_kick_fusion(fused)
                lat.run(gp, first_pulse=4, n_pulses=1)
                err = np.max(np.abs(np_state(lat) - wantI))
                assert err < TOL[prec], (shape, bc, v, bz, fused, err)
                lat.close()


# ------------------------------------------------------------------ kicks ---
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kick_parity(P, prec):
    shape = (20, 12, 9)
    N = int(np.prod(shape))
    s0 = inputs.unit_spins(N, 8) * (1 + 0.01 * inputs.rng(9).random(N))[None, :]
    s0 = rounded(s0, prec)
    op, gp = both_params("zaxis", Dt=10.0, dt=0.25, seed=77)
    lat = make_lattice(P, shape, "periodic", prec, s0)
    lat.kick_norm_dev(reset=True)
    lat.pulse(gp, 123)
    want, dev = orc.kick(orc.geom(shape), op, s0, op.T, seed=77, r=0, k=123)
    got = np_state(lat)
    assert np.max(np.abs(got - want)) < TOL[prec]
    assert lat.kick_norm_dev() == pytest.approx(dev, rel=1e-5 if prec == "fp32" else 1e-10)
    # T = 0: pure renormalisation
    lat2 = make_lattice(P, shape, "periodic", prec, s0)
    op0, gp0 = both_params("zaxis", Dt=10.0, dt=0.25, seed=77, T=0.0)
    lat2.pulse(gp0, 5)
    np.testing.assert_allclose(np_state(lat2), s0 / np.linalg.norm(s0, axis=0), atol=TOL[prec] * 0.1)


# ------------------------------------------------------------ observables ---
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["axis", "zaxis", "none"])
@pytest.mark.parametrize("shape,bc", [((40, 24, 20), "periodic"), ((17, 5, 3), "free"),
                                      ((1, 1, 1), "periodic"), ((2, 2, 2), "periodic"),
                                      # more work items than blocks, ragged last column run
                                      # and ragged last z-slab
                                      ((300, 100, 170), "periodic"), ((300, 100, 170), "free")])
def test_observables_parity(P, prec, kind, shape, bc):
    N = int(np.prod(shape))
    s0 = rounded(inputs.unit_spins(N, 21) * 1.001, prec)
    op, gp = both_params(kind)
    lat = make_lattice(P, shape, bc, prec, s0)
    got = lat.observables(gp)
    want = orc.observables(orc.geom(shape, bc), op, s0)
    for k in ("E_total", "E_exch", "E_zeeman", "E_anis"):
        assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-13 * N), k
    np.testing.assert_allclose(got["m"], want["m"], rtol=1e-12, atol=1e-15)
    assert got["max_norm_dev"] == pytest.approx(want["max_norm_dev"], rel=1e-12, abs=1e-16)


def test_observables_nonfinite(P):
    shape = (8, 8, 8)
    s0 = inputs.unit_spins(512, 1)
    lat = make_lattice(P, shape, "periodic", "fp32", s0)
    lat.state[1, 77] = float("nan")
    _, gp = both_params("zaxis")
    with pytest.raises(P.LLLError) as ei:
        lat.observables(gp)
    assert ei.value.status == P.LLL_ENONFINITE


# ------------------------------------------------------------- schedule -----
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dt,Dt", [(0.1, 0.4), (0.1, 0.3), (0.2, 0.2)])
@pytest.mark.parametrize("shape,bc", [((40, 24, 20), "periodic"), ((40, 36, 1), "periodic"),
                                      ((23, 9, 5), "free")])
def test_run_per_segment(P, prec, dt, Dt, shape, bc):
    """Each interval (n1 steps, kick, n2 steps) of lll_run against the oracle
    started from the GPU's state before that interval, on every step variant
    (kick as the fused epilogue where the step is fused)."""
    N = int(np.prod(shape))
    op, gp = both_params("zaxis", dt=dt, Dt=Dt, seed=5)
    g = orc.geom(shape, bc)
    for v in variants(P, prec):
        lat = P.Lattice(shape, bc=bc, precision=prec, init="random", seed=9)
        lat.set_step_config(v, 0)
        prev = np_state(lat)
        for q in range(3):
            tr = lat.run(gp, first_pulse=10 + q, n_pulses=1, obs_every=1)
            cur = np_state(lat)
            want, otr, _ = orc.run(g, op, prev, seed=5, first_pulse=10 + q, n_pulses=1, obs_every=1)
            err = np.max(np.abs(cur - want))
            assert err < TOL[prec], (v, q, err)
            o = orc.observables(g, op, cur)
            assert tr[0]["E_total"] == pytest.approx(o["E_total"], rel=1e-12, abs=1e-13 * N)
            np.testing.assert_allclose(tr[0]["m"], o["m"], rtol=1e-12, atol=1e-15)
            prev = cur


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_schedule_identity_bitexact(P, prec):
    """lll_run(K) == step(n1), pulse(k), step(n2) repeated == run(1) + run(K-1),
    bit for bit (the noise is a function of the pulse index only)."""
    shape = (40, 24, 20)
    _, gp = both_params("axis", dt=0.1, Dt=0.5, seed=8)
    for v in variants(P, prec):
        a = P.Lattice(shape, precision=prec, seed=3)
        b = P.Lattice(shape, precision=prec, seed=3)
        c = P.Lattice(shape, precision=prec, seed=3)
        for L in (a, b, c):
            L.set_step_config(v, 0)
        a.run(gp, first_pulse=20, n_pulses=3)
        for k in range(20, 23):
            b.step(gp, 2)
            b.pulse(gp, k)
            b.step(gp, 3)
        c.run(gp, first_pulse=20, n_pulses=1)
        c.run(gp, first_pulse=21, n_pulses=2)
        torch.cuda.synchronize()
        assert torch.equal(a.state, b.state), v
        assert torch.equal(a.state, c.state), v
        # run-to-run determinism
        d = P.Lattice(shape, precision=prec, seed=3)
        d.set_step_config(v, 0)
        d.run(gp, first_pulse=20, n_pulses=3)
        torch.cuda.synchronize()
        assert torch.equal(a.state, d.state)
        # kick as its own launch instead of the fused step's epilogue
        e = P.Lattice(shape, precision=prec, seed=3)
        e.set_step_config(v, 0)
        e.set_kick_fusion(False)
        e.run(gp, first_pulse=20, n_pulses=3)
        a2 = P.Lattice(shape, precision=prec, seed=3)
        a2.set_step_config(v, 0)
        a2.run(gp, first_pulse=20, n_pulses=3)
        torch.cuda.synchronize()
        assert torch.equal(a.state, e.state), v
        assert e.kick_norm_dev() == a2.kick_norm_dev(), v


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_schedule_identity_one_step_intervals(P, prec):
    """Delta t = delta t (n = 1: kick, then the step).  A run of K intervals,
    which applies each next interval's kick as the epilogue of the step before
    it (with that interval's temperature), equals K runs of one interval and
    the pulse/step sequence, bit for bit, with or without measurements in
    between and with the kick fused or in its own launch; the running kick
    maximum is the same too."""
    shape = (40, 24, 20)
    _, gp = both_params("zaxis", dt=0.2, Dt=0.2, lam=0.1, seed=6, precession=False)
    Ts = [2.0, 1.4, 0.9, 0.5, 0.3]
    K = len(Ts)
    for v in variants(P, prec):
        for fused in (True, False):
            lats = [P.Lattice(shape, precision=prec, seed=2) for _ in range(4)]
            for L in lats:
                L.set_step_config(v, 0)
                L.set_kick_fusion(fused)
                L.kick_norm_dev(reset=True)
            a, b, c, d = lats
            a.run(gp, first_pulse=30, n_pulses=K, T_per_pulse=Ts)
            for q in range(K):
                b.run(gp, first_pulse=30 + q, n_pulses=1, T_per_pulse=[Ts[q]])
                c.pulse(dataclasses.replace(gp, T=Ts[q]), 30 + q)
                c.step(gp, 1)
            tr = d.run(gp, first_pulse=30, n_pulses=K, T_per_pulse=Ts, obs_every=2)
            torch.cuda.synchronize()
            for o in (b, c, d):
                assert torch.equal(a.state, o.state), (v, fused)
            assert len({L.kick_norm_dev() for L in lats}) == 1, (v, fused)
            assert len(tr) == K // 2
            o2 = P.Lattice(shape, precision=prec, seed=2)
            o2.set_step_config(v, 0)
            o2.run(gp, first_pulse=30, n_pulses=2, T_per_pulse=Ts[:2])
            assert tr[0]["E_total"] == pytest.approx(o2.observables(gp)["E_total"], rel=1e-14)
            for L in lats + [o2]:
                L.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["rk2mid", "rk5b"])
def test_one_step_intervals_other_integrators(P, prec, method):
    """The carried kick of one-step intervals with the Appendix's integrators
    (RK2 midpoint: fused single-step launches; Butcher's RK5: per-stage path,
    kick in its own launch): a run of K intervals equals K one-interval runs
    bit for bit, with the kick fused and in its own launch."""
    shape = (40, 24, 20)
    _, gp = both_params("zaxis", dt=0.2, Dt=0.2, lam=0.1, seed=7, precession=False)
    gp = dataclasses.replace(gp, integrator=method)
    Ts = [1.8, 1.1, 0.6, 0.4]
    for fused in (True, False):
        a = P.Lattice(shape, precision=prec, seed=3)
        b = P.Lattice(shape, precision=prec, seed=3)
        for L in (a, b):
            L.set_kick_fusion(fused)
            L.kick_norm_dev(reset=True)
        a.run(gp, first_pulse=50, n_pulses=len(Ts), T_per_pulse=Ts)
        for q, T in enumerate(Ts):
            b.run(gp, first_pulse=50 + q, n_pulses=1, T_per_pulse=[T])
        torch.cuda.synchronize()
        assert torch.equal(a.state, b.state), (method, fused)
        assert a.kick_norm_dev() == b.kick_norm_dev(), (method, fused)
        a.close()
        b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_staged_measurements_match_one_by_one(P, prec):
    """The measurements of a run are reduced in groups (at most 1024 per
    launch, here more than one group); the trace and the running sums equal,
    bit for bit, those of one-interval runs measured one at a time.  Through
    the C ABI without a trace buffer, the running sums are the same too."""
    import ctypes
    shape = (8, 8, 8)
    _, gp = both_params("zaxis", dt=0.1, Dt=0.1, seed=3)
    K = 1100
    a = P.Lattice(shape, precision=prec, seed=1)
    b = P.Lattice(shape, precision=prec, seed=1)
    c = P.Lattice(shape, precision=prec, seed=1)
    ta = a.run(gp, first_pulse=0, n_pulses=K, obs_every=1)
    tb = [b.run(gp, first_pulse=q, n_pulses=1, obs_every=1)[0] for q in range(K)]
    pc = gp.c()
    st = P.lib().lll_run(c.h, ctypes.byref(pc), ctypes.c_uint64(0), K, None, 1, None)
    assert st in (P.LLL_OK, P.LLL_WARN_APPLICABILITY), st
    torch.cuda.synchronize()
    assert len(ta) == K
    assert ta == tb
    acc = a.accumulators()
    assert acc == b.accumulators() == c.accumulators()
    assert acc[0] == K
    assert torch.equal(a.state, b.state) and torch.equal(a.state, c.state)
    for L in (a, b, c):
        L.close()


def test_staging_buffer_full_mid_run(P):
    """128^3 fp32: the staging buffer holds 512 measurements (64 KiB of
    partials each), so a run of 520 measured intervals reduces a full buffer
    mid-run and the rest at the end; its trace and running sums equal those
    of two runs of 260, bit for bit."""
    shape = (128, 128, 128)
    _, gp = both_params("zaxis", dt=0.2, Dt=0.2, seed=2)
    a = P.Lattice(shape, precision="fp32", seed=5)
    b = P.Lattice(shape, precision="fp32", seed=5)
    ta = a.run(gp, first_pulse=0, n_pulses=520, obs_every=1)
    tb = b.run(gp, first_pulse=0, n_pulses=260, obs_every=1)
    tb += b.run(gp, first_pulse=260, n_pulses=260, obs_every=1)
    assert ta == tb
    assert a.accumulators() == b.accumulators()
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_one_step_intervals_bitexact(P, prec):
    """Batch with n = 1: one replay of K intervals equals K replays of one
    interval, bit for bit, with and without measurements in between; without
    a trace the measurements still feed the same running sums."""
    reps = BATCH_SETS["mixed"]
    A = P.Batch(reps, precision=prec, dt=0.2, Dt=0.2)
    B = P.Batch(reps, precision=prec, dt=0.2, Dt=0.2)
    C = P.Batch(reps, precision=prec, dt=0.2, Dt=0.2)
    D = P.Batch(reps, precision=prec, dt=0.2, Dt=0.2)
    A.run(first_pulse=5, n_pulses=4)
    for q in range(4):
        B.run(first_pulse=5 + q, n_pulses=1)
    tc = C.run(first_pulse=5, n_pulses=4, obs_every=3)
    assert D.run(first_pulse=5, n_pulses=4, obs_every=3, trace=False) == []
    torch.cuda.synchronize()
    for r in range(len(reps)):
        assert torch.equal(A.state(r), B.state(r)), r
        assert torch.equal(A.state(r), C.state(r)), r
        assert torch.equal(A.state(r), D.state(r)), r
    assert len(tc) == 1
    assert C.accumulators() == D.accumulators()
    for X in (A, B, C, D):
        X.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_temperature_ramp(P, prec):
    shape = (17, 9, 11)
    op, gp = both_params("zaxis", dt=0.2, Dt=0.2, lam=0.1, seed=4, precession=False)
    Ts = [2.0, 1.5, 1.0, 0.5]
    lat = P.Lattice(shape, precision=prec, seed=1)
    prev = np_state(lat)
    g = orc.geom(shape)
    for q, T in enumerate(Ts):
        lat.run(gp, first_pulse=q, n_pulses=1, T_per_pulse=[T])
        cur = np_state(lat)
        want, _, _ = orc.run(g, op, prev, seed=4, first_pulse=q, n_pulses=1, T_per_pulse=[T])
        assert np.max(np.abs(cur - want)) < TOL[prec]
        prev = cur


# --------------------------------------------------- full-size, sampled -----
def _cutout(s, shape, centre, rad):
    """(3, (2rad+1)^3) periodic cut-out around centre and its global site ids."""
    Lx, Ly, Lz = shape
    cx, cy, cz = centre
    r = np.arange(-rad, rad + 1)
    xs = (cx + r) % Lx
    ys = (cy + r) % Ly
    zs = (cz + r) % Lz
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    ids = (X + Lx * (Y + Ly * Z)).ravel()
    return s[:, ids], ids.astype(np.uint32)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_full_size_sampled(P, prec):
    """128^3 headline lattice in the benchmark's launch configuration: one
    interval of two steps (step with the fused kick epilogue, then a step);
    sampled sites are recomputed by the oracle on a free-boundary cut-out of
    radius 8 with the sites' global noise counters."""
    shape = (128, 128, 128)
    import bench
    op, gp = both_params("zaxis", dt=0.2, Dt=0.4, seed=0)
    lat = P.Lattice(shape, precision=prec, init="random", seed=0)
    bench.configure_lattice(lat, prec, shape)
    s0 = np_state(lat)
    lat.run(gp, first_pulse=7, n_pulses=1)
    s1 = np_state(lat)
    rng = np.random.default_rng(2)
    cen = [tuple(c) for c in rng.integers(0, 128, size=(24, 3))] + [(0, 0, 0), (127, 127, 127),
                                                                      (31, 15, 64), (32, 16, 0)]
    rad = 8
    n = 2 * rad + 1
    gc = orc.geom((n, n, n), "free")
    mid = (n**3) // 2
    for c in cen:
        cut, ids = _cutout(s0, shape, c, rad)
        st = orc.step(gc, op, cut, 1)
        st, _ = orc.kick_indexed(gc, op, st, op.T, seed=0, r=0, k=7, site_id=ids)
        st = orc.step(gc, op, st, 1)
        i = c[0] + 128 * (c[1] + 128 * c[2])
        err = np.max(np.abs(st[:, mid] - s1[:, i]))
        assert err < TOL[prec], (c, err)
    # observables at full size
    got = lat.observables(gp)
    want = orc.observables(orc.geom(shape), op, s1)
    assert got["E_total"] == pytest.approx(want["E_total"], rel=1e-12, abs=1e-13 * 128**3)
    np.testing.assert_allclose(got["m"], want["m"], rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_headline_interval_full_size(P, prec):
    """The headline workload's own interval on the whole 128^3 lattice, in the
    benchmark's tuned launch configuration (kick fused where it is tuned so):
    dt = 0.2, Dt = 2 (n = 10: five steps, kick, five steps; Eq. (7)), J = 1,
    H = (0, 0, 0.1), D = 0.05 along z, lambda = 0.01, T = 1.  Two intervals,
    each against the oracle started from the GPU's state before it: every spin
    component, the measured observables and the interval's largest kick
    deviation."""
    import bench
    shape = (128, 128, 128)
    N = int(np.prod(shape))
    ph = dict(bench.PHYS)
    gp = P.Params(**ph)
    op = orc.Params(J=ph["J"], H=ph["H"], D=ph["D"], e=ph["e"], lam=ph["lam"], T=ph["T"],
                    dt=ph["dt"], Dt=ph["Dt"], precession=True)
    assert orc.steps_per_interval(op) == 10
    lat = P.Lattice(shape, precision=prec, init="random", seed=0)
    bench.configure_lattice(lat, prec, shape)
    g = orc.geom(shape)
    prev = np_state(lat)
    lat.kick_norm_dev(reset=True)
    for q in range(2):
        with pytest.warns(P.ApplicabilityWarning):  # h_max dt = 1.24 > 0.25 (the workload's own)
            tr = lat.run(gp, first_pulse=q, n_pulses=1, obs_every=1)
        cur = np_state(lat)
        want, otr, odev = orc.run(g, op, prev, seed=0, first_pulse=q, n_pulses=1, obs_every=1)
        err = float(np.max(np.abs(cur - want)))
        assert err < TOL[prec], (q, err)
        gdev = lat.kick_norm_dev(reset=True)
        # | |s'| - 1 | moves by at most sqrt(3) times the largest component error
        assert abs(gdev - odev) <= 2 * TOL[prec], (q, gdev, odev)
        o = orc.observables(g, op, cur)
        for k in ("E_total", "E_exch", "E_zeeman", "E_anis"):
            assert tr[0][k] == pytest.approx(o[k], rel=1e-12, abs=1e-13 * N), (q, k)
        np.testing.assert_allclose(tr[0]["m"], o["m"], rtol=1e-12, atol=1e-15)
        assert tr[0]["max_norm_dev"] == pytest.approx(o["max_norm_dev"], rel=1e-12, abs=1e-16)
        prev = cur
    lat.close()


def test_max_size_sampled(P):
    """A lattice just under the 2^31 - 1 site limit and ragged in x and y
    (1023 x 1025 x 2047 = 2,146,433,025 sites, 25.8 GB per fp32 state copy)
    in the default launch configuration: one interval of two steps with the
    kick epilogue.  Sampled sites, the last ones included, against the oracle
    on free-boundary cut-outs of radius 8 with the sites' global noise
    counters; the observables against fp64 reductions of the whole state done
    here with torch (z-slabs of 256 planes, periodic bonds to +x, +y, +z)."""
    shape = (1023, 1025, 2047)
    Lx, Ly, Lz = shape
    N = Lx * Ly * Lz
    assert N < 2**31 - 1
    op, gp = both_params("zaxis", dt=0.2, Dt=0.4, seed=0)
    lat = P.Lattice(shape, precision="fp32", init="random", seed=0)
    rng = np.random.default_rng(31)
    cen = [tuple(int(v) for v in c) for c in zip(rng.integers(0, Lx, 12), rng.integers(0, Ly, 12),
                                                 rng.integers(0, Lz, 12))]
    cen += [(0, 0, 0), (Lx - 1, Ly - 1, Lz - 1), (Lx - 1, 0, Lz - 1), (0, Ly - 1, Lz - 2)]
    rad = 8
    n = 2 * rad + 1
    r = np.arange(-rad, rad + 1)
    cuts = []
    for cx, cy, cz in cen:
        Z, Y, X = np.meshgrid((cz + r) % Lz, (cy + r) % Ly, (cx + r) % Lx, indexing="ij")
        ids = (X + Lx * (Y + Ly * Z.astype(np.int64))).ravel()
        st = lat.state[:, torch.from_numpy(ids).cuda()].double().cpu().numpy()
        cuts.append((ids, st))
    lat.run(gp, first_pulse=3, n_pulses=1)
    torch.cuda.synchronize()
    gc = orc.geom((n, n, n), "free")
    mid = (n**3) // 2
    for (cx, cy, cz), (ids, st) in zip(cen, cuts):
        st = orc.step(gc, op, st, 1)
        st, _ = orc.kick_indexed(gc, op, st, op.T, seed=0, r=0, k=3, site_id=ids.astype(np.uint32))
        st = orc.step(gc, op, st, 1)
        i = cx + Lx * (cy + Ly * cz)
        got = lat.state[:, i].double().cpu().numpy()
        err = np.max(np.abs(st[:, mid] - got))
        assert err < TOL["fp32"], ((cx, cy, cz), err)
    got = lat.observables(gp)
    v = lat.state.view(3, Lz, Ly, Lx)
    bonds = anis = 0.0
    msum = np.zeros(3)
    n2max, n2min = -1.0, 9.0
    for z0 in range(0, Lz, 256):
        z1 = min(z0 + 256, Lz)
        c = v[:, z0:z1].double()
        msum += c.sum(dim=(1, 2, 3)).cpu().numpy()
        n2 = (c * c).sum(0)
        n2max, n2min = max(n2max, float(n2.max())), min(n2min, float(n2.min()))
        del n2
        anis += float((c[2] * c[2]).sum())
        bonds += float((c * c.roll(-1, dims=3)).sum()) + float((c * c.roll(-1, dims=2)).sum())
        bonds += float((c[:, :-1] * c[:, 1:]).sum())
        bonds += float((c[:, -1] * v[:, z1 % Lz].double()).sum())
        del c
    J, H, D = op.J, op.H, op.D
    e_exch = -J * bonds
    e_zee = -(H[0] * msum[0] + H[1] * msum[1] + H[2] * msum[2])
    e_anis = -D * anis
    assert got["E_exch"] == pytest.approx(e_exch, rel=1e-10)
    assert got["E_zeeman"] == pytest.approx(e_zee, rel=1e-10, abs=1e-5)
    assert got["E_anis"] == pytest.approx(e_anis, rel=1e-10)
    assert got["E_total"] == pytest.approx(e_exch + e_zee + e_anis, rel=1e-10)
    np.testing.assert_allclose(got["m"], msum / N, rtol=1e-9, atol=1e-13)
    dev = max(np.sqrt(n2max) - 1.0, 1.0 - np.sqrt(n2min))
    assert got["max_norm_dev"] == pytest.approx(dev, rel=1e-12, abs=1e-15)
    lat.close()


# ------------------------------------------------------------------ batch ---
BATCH_SETS = {
    "mixed": [dict(L=(8, 8, 8), T=0.5, lam=0.02, seed=11, replica=0),
              dict(L=(12, 12, 12), T=1.5, lam=0.005, seed=12, replica=1),
              dict(L=(5, 6, 7), T=1.0, lam=0.05, seed=13, replica=2, H=(0, 0, 0.2)),
              dict(L=(24, 24, 24), T=0.3, lam=0.01, seed=14, replica=3, D=0.05),
              dict(L=(17, 9, 3), T=2.0, lam=0.03, seed=15, replica=4, bc="free")],
    # degenerate and flat replicas next to one large enough for the fused step
    # and for several observables blocks: a single spin, an open chain, a
    # periodic 2-D plane, a free 1-site-thick slab
    "degenerate": [dict(L=(1, 1, 1), T=1.0, lam=0.05, seed=21, replica=0, H=(0, 0, 0.3)),
                   dict(L=(7, 1, 1), T=0.8, lam=0.02, seed=22, replica=1, bc="free"),
                   dict(L=(40, 36, 1), T=1.2, lam=0.01, seed=23, replica=2),
                   dict(L=(9, 11, 1), T=0.4, lam=0.03, seed=24, replica=3, bc="free", D=0.05),
                   dict(L=(64, 48, 40), T=1.0, lam=0.01, seed=25, replica=4, H=(0.1, 0, 0))],
}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("which", sorted(BATCH_SETS))
def test_batch_matches_oracle(P, prec, which):
    reps = BATCH_SETS[which]
    dt, Dt = 0.1, 0.4
    B = P.Batch(reps, precision=prec, dt=dt, Dt=Dt)
    prev = []
    for r, d in enumerate(reps):
        g = orc.geom(d["L"], d.get("bc", "periodic"))
        want = orc.init_random_sphere(g, d["seed"], d["replica"])
        got = B.state(r).double().cpu().numpy()
        np.testing.assert_allclose(got, want, atol=1.5e-7 if prec == "fp32" else 4e-16)
        prev.append(got)
    for q in range(2):
        tr = B.run(first_pulse=q, n_pulses=1, obs_every=1)
        for r, d in enumerate(reps):
            g = orc.geom(d["L"], d.get("bc", "periodic"))
            op = orc.Params(J=1.0, H=d.get("H", (0, 0, 0)), D=d.get("D", 0.0), lam=d["lam"], T=d["T"],
                            dt=dt, Dt=Dt)
            cur = B.state(r).double().cpu().numpy()
            want, _, _ = orc.run(g, op, prev[r], seed=d["seed"], r=d["replica"], first_pulse=q,
                                 n_pulses=1)
            assert np.max(np.abs(cur - want)) < TOL[prec], (q, r)
            o = orc.observables(g, op, cur)
            assert tr[0][r]["E_total"] == pytest.approx(o["E_total"], rel=1e-12, abs=1e-12)
            prev[r] = cur
    acc = B.accumulators()
    assert all(a[0] == 2 for a in acc)
    B.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lattice_with_replica_key_follows_batch(P, prec):
    """A lone lattice whose kicks use a batch replica's key (seed, replica)
    and that starts from that replica's state follows the replica's
    trajectory (the noise is a function of site, pulse, replica and seed
    only); with replica key 0 it draws different noise."""
    reps = [dict(L=(24, 24, 24), T=1.4, lam=0.01, seed=1000, replica=0),
            dict(L=(48, 48, 48), T=0.8, lam=0.02, seed=1040, replica=40),
            dict(L=(20, 12, 9), T=1.0, lam=0.03, seed=7, replica=5, bc="free")]
    dt, Dt = 0.1, 1.0
    B = P.Batch([dict(r, J=1.0) for r in reps], precision=prec, dt=dt, Dt=Dt)
    lats = []
    for i, r in enumerate(reps):
        lat = P.Lattice(r["L"], precision=prec, bc=r.get("bc", "periodic"), state=B.state(i))
        p = P.Params(J=1.0, lam=r["lam"], T=r["T"], dt=dt, Dt=Dt, seed=r["seed"], replica=r["replica"])
        lats.append((lat, p))
    other = P.Lattice(reps[1]["L"], precision=prec, state=B.state(1))
    p_other = P.Params(J=1.0, lam=reps[1]["lam"], T=reps[1]["T"], dt=dt, Dt=Dt, seed=reps[1]["seed"])
    B.run(first_pulse=3, n_pulses=3)
    for lat, p in lats:
        lat.run(p, first_pulse=3, n_pulses=3)
    other.run(p_other, first_pulse=3, n_pulses=3)
    torch.cuda.synchronize()
    # fp32: batch and lone lattice may run different step kernels (fused tiles
    # vs per-stage launches), whose rounding orders differ over 30 steps
    tol = 1e-12 if prec == "fp64" else 5e-5
    for i, (lat, _) in enumerate(lats):
        d = (lat.state.double() - B.state(i).double()).abs().max().item()
        assert d < tol, (i, d)
    assert (other.state.double() - B.state(1).double()).abs().max().item() > 0.1
    for lat, _ in lats:
        lat.close()
    other.close()
    B.close()


def test_batch_replay_across_pulse_counter_wrap(P):
    """A batch replays its captured schedule for any first pulse, also where the
    pulse index passes 2^32 (the kick's counter word is the index mod 2^32):
    two replays of a two-interval schedule equal one four-interval run bit for
    bit, and a lone lattice keyed like a replica follows that replica."""
    reps = BATCH_SETS["mixed"]
    k0 = 2**32 - 2
    dt, Dt = 0.1, 0.4
    A = P.Batch(reps, precision="fp64", dt=dt, Dt=Dt)
    B = P.Batch(reps, precision="fp64", dt=dt, Dt=Dt)
    C = P.Batch(reps, precision="fp64", dt=dt, Dt=Dt)
    A.run(first_pulse=k0, n_pulses=4)
    B.run(first_pulse=k0, n_pulses=2)
    B.run(first_pulse=k0 + 2, n_pulses=2)  # replay of the same graph
    torch.cuda.synchronize()
    for r in range(len(reps)):
        assert torch.equal(A.state(r), B.state(r)), r
    for r in (1, 4):
        d = reps[r]
        lat = P.Lattice(d["L"], precision="fp64", bc=d.get("bc", "periodic"), state=C.state(r))
        p = P.Params(J=1.0, H=d.get("H", (0, 0, 0)), D=d.get("D", 0.0), lam=d["lam"], T=d["T"],
                     dt=dt, Dt=Dt, seed=d["seed"], replica=d["replica"])
        lat.run(p, first_pulse=k0, n_pulses=4)
        torch.cuda.synchronize()
        err = (lat.state - A.state(r)).abs().max().item()
        assert err < 1e-12, (r, err)
        lat.close()
    for X in (A, B, C):
        X.close()


def test_kernel_timing_samples_fused_launches(P):
    """Dispatch-event timing of the fused step covers a sample of the plain
    launches (one in 16, none with the kick epilogue) and gives a positive
    mean duration."""
    p = P.Params(J=1.0, H=(0.0, 0.0, 0.1), D=0.05, lam=0.01, T=1.0, dt=0.2, Dt=0.4, seed=3)
    lat = P.Lattice((32, 32, 32), precision="fp32", init="random", seed=1)
    lat.set_step_config(1, 16)
    lat.kernel_timing_start()
    lat.step(p, 160)
    ms, n = lat.kernel_timing_stop()
    assert 1 <= n <= 10 and ms > 0.0, (n, ms)
    lat.kernel_timing_start()
    ms0, n0 = lat.kernel_timing_stop()
    assert (ms0, n0) == (0.0, 0)
    lat.close()


def test_lattice_raw_trace_matches_dicts(P):
    """Lattice.run(raw=True) returns the same measurements, as rows of the
    lll_obs fields, as the dict trace of an identical run."""
    p = P.Params(J=1.0, H=(0.0, 0.0, 0.1), D=0.05, lam=0.01, T=1.0, dt=0.2, Dt=0.4, seed=3)
    a = P.Lattice((12, 10, 9), precision="fp64", init="random", seed=1)
    b = P.Lattice((12, 10, 9), precision="fp64", init="random", seed=1)
    rows = a.run(p, first_pulse=0, n_pulses=6, obs_every=2, raw=True)
    dicts = b.run(p, first_pulse=0, n_pulses=6, obs_every=2)
    assert rows.shape == (3, 8)
    assert [P.obs_row_dict(r) for r in rows] == [
        dict(d, m=tuple(float(x) for x in d["m"])) for d in dicts]
    assert a.run(p, first_pulse=6, n_pulses=2, obs_every=0, raw=True).shape == (0, 8)
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_long_run_in_chunks(P, prec):
    """A run longer than one captured graph (1000 pulses) is done as replays of
    chunks a whole number of measurement spacings long: one call of 2100
    pulses measured every 7 (chunks of 994, 994 and 112) ends in the states of
    21 calls of 100 pulses, bit for bit, and its trace equals theirs wherever
    both measure (pulses that are multiples of 7 in calls 0, 7 and 14)."""
    reps = BATCH_SETS["mixed"]
    A = P.Batch(reps, precision=prec, dt=0.2, Dt=0.4)
    B = P.Batch(reps, precision=prec, dt=0.2, Dt=0.4)
    ta = A.run(first_pulse=3, n_pulses=2100, obs_every=7, raw=True)
    tb = [B.run(first_pulse=3 + 100 * c, n_pulses=100, obs_every=7, raw=True) for c in range(21)]
    torch.cuda.synchronize()
    # 100-pulse calls measure at 7, 14, ..., 98 of each call; the long run at
    # every 7th pulse of the whole: compare where both measure
    want = {}
    for c, t in enumerate(tb):
        for m in range(t.shape[0]):
            want[100 * c + 7 * (m + 1)] = t[m]
    assert ta.shape == (300, len(reps), 8)
    common = 0
    for m in range(ta.shape[0]):
        q = 7 * (m + 1)
        if q in want:
            assert np.array_equal(ta[m], want[q]), q
            common += 1
    assert common > 20
    for r in range(len(reps)):
        assert torch.equal(A.state(r), B.state(r)), r
    A.close()
    B.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_long_spacing_in_chunks(P, prec):
    """A measurement spacing above one graph (1200 pulses): each period runs as
    an unmeasured chunk of 1000 and a chunk of 200 measured at its end.  2500
    pulses in one call measure after pulses 1200 and 2400 what the observables
    of 25 unmeasured calls of 100 pulses give there, bit for bit, and end in
    the same states."""
    reps = BATCH_SETS["mixed"]
    A = P.Batch(reps, precision=prec, dt=0.2, Dt=0.4)
    B = P.Batch(reps, precision=prec, dt=0.2, Dt=0.4)
    ta = A.run(first_pulse=3, n_pulses=2500, obs_every=1200, raw=True)
    want = []
    for c in range(25):
        B.run(first_pulse=3 + 100 * c, n_pulses=100)
        if c in (11, 23):
            want.append(B.observables())
    torch.cuda.synchronize()
    assert ta.shape == (2, len(reps), 8)
    for m, obs in enumerate(want):
        for r, o in enumerate(obs):
            row = [o["E_total"], o["E_exch"], o["E_zeeman"], o["E_anis"], *o["m"],
                   o["max_norm_dev"]]
            assert np.array_equal(ta[m, r], np.array(row)), (m, r)
    for r in range(len(reps)):
        assert torch.equal(A.state(r), B.state(r)), r
    A.close()
    B.close()


def test_batch_run_shorter_than_its_spacing(P):
    """1200 pulses with a measurement spacing of 1500: no measurement, chunks
    of 1000 and 200 pulses, the same final states as 12 unmeasured calls of
    100 pulses."""
    reps = BATCH_SETS["mixed"]
    A = P.Batch(reps, precision="fp32", dt=0.2, Dt=0.4)
    B = P.Batch(reps, precision="fp32", dt=0.2, Dt=0.4)
    ta = A.run(first_pulse=11, n_pulses=1200, obs_every=1500, raw=True)
    for c in range(12):
        B.run(first_pulse=11 + 100 * c, n_pulses=100)
    torch.cuda.synchronize()
    assert ta.shape == (0, len(reps), 8)
    for r in range(len(reps)):
        assert torch.equal(A.state(r), B.state(r)), r
    A.close()
    B.close()


# ------------------------------------------- the other workload configs -----
def test_small_fp64_workload_per_segment(P):
    """16^3 periodic fp64 ferromagnet (J = 1, H = 0, D = 0, lambda = 0.01, T = 1,
    dt = 0.1, Dt = 1): three intervals in the tuned launch configuration, each
    against the oracle started from the GPU's state before it."""
    import bench
    shape = (16, 16, 16)
    op = orc.Params(J=1.0, lam=0.01, T=1.0, dt=0.1, Dt=1.0)
    gp = P.Params(J=1.0, H=(0, 0, 0), D=0.0, lam=0.01, T=1.0, dt=0.1, Dt=1.0, seed=0)
    lat = P.Lattice(shape, precision="fp64", init="random", seed=0)
    lat.autotune(gp, cache_path=bench.TUNE_CACHE)
    g = orc.geom(shape)
    prev = np_state(lat)
    np.testing.assert_allclose(prev, orc.init_random_sphere(g, 0), atol=4e-16)
    for q in range(3):
        tr = lat.run(gp, first_pulse=q, n_pulses=1, obs_every=1)
        cur = np_state(lat)
        want, otr, _ = orc.run(g, op, prev, seed=0, first_pulse=q, n_pulses=1, obs_every=1)
        assert np.max(np.abs(cur - want)) < TOL["fp64"], q
        assert tr[0]["E_total"] == pytest.approx(otr[0]["E_total"], rel=1e-11)
        prev = cur
    lat.close()


def test_full_batch_sampled(P):
    """The 96-replica uneven batch (32 each of 24^3, 48^3, 64^3) in fp32 in the
    tuned launch configuration: one interval; one replica of each size is
    recomputed whole by the oracle from the batch's own start state and keys."""
    import bench
    reps = inputs.batch_replicas(seed=0)
    B = P.Batch([dict(r, J=1.0) for r in reps], precision="fp32", dt=0.1, Dt=1.0)
    B.autotune(cache_path=bench.TUNE_CACHE)
    picks = [5, 40, 77]
    s0 = {i: B.state(i).double().cpu().numpy() for i in picks}
    tr = B.run(first_pulse=0, n_pulses=1, obs_every=1)
    for i in picks:
        r = reps[i]
        g = orc.geom(r["L"])
        op = orc.Params(J=1.0, lam=r["lam"], T=r["T"], dt=0.1, Dt=1.0)
        want, _, _ = orc.run(g, op, s0[i], seed=r["seed"], r=r["replica"], first_pulse=0,
                             n_pulses=1)
        cur = B.state(i).double().cpu().numpy()
        assert np.max(np.abs(cur - want)) < TOL["fp32"], i
        o = orc.observables(g, op, cur)
        assert tr[0][i]["E_total"] == pytest.approx(o["E_total"], rel=1e-12, abs=1e-12)
        np.testing.assert_allclose(tr[0][i]["m"], o["m"], rtol=1e-11, atol=1e-14)
    B.close()


def test_full_size_overdamped_sampled(P):
    """256^3 fp32 slow equation (J = 1, D = 0.02 z, lambda = 0.1, dt = Dt = 0.4,
    a pulse every step, first two temperatures of the 2.0 -> 0.5 ramp) in the
    tuned launch configuration; sampled sites against the oracle on free-boundary
    cut-outs of radius 8 with the sites' global noise counters."""
    import bench
    shape = (256, 256, 256)
    Ts = [2.0, 2.0 - 1.5 / 4999]
    op = orc.Params(J=1.0, D=0.02, e=(0, 0, 1), lam=0.1, T=Ts[0], dt=0.4, Dt=0.4,
                    precession=False)
    gp = P.Params(J=1.0, D=0.02, e=(0, 0, 1), lam=0.1, T=Ts[0], dt=0.4, Dt=0.4,
                  precession=False, seed=0)
    lat = P.Lattice(shape, precision="fp32", init="random", seed=0)
    lat.autotune(gp, cache_path=bench.TUNE_CACHE)
    s0 = np_state(lat)
    lat.run(gp, first_pulse=0, n_pulses=2, T_per_pulse=Ts)
    s1 = np_state(lat)
    rng = np.random.default_rng(5)
    cen = [tuple(c) for c in rng.integers(0, 256, size=(16, 3))] + [(0, 0, 0), (255, 255, 255),
                                                                      (64, 0, 63), (1, 128, 64)]
    rad = 8
    n = 2 * rad + 1
    gc = orc.geom((n, n, n), "free")
    mid = (n**3) // 2
    for c in cen:
        cut, ids = _cutout(s0, shape, c, rad)
        st = cut
        for k, T in enumerate(Ts):  # n = 1: kick, then the step
            st, _ = orc.kick_indexed(gc, op, st, T, seed=0, r=0, k=k, site_id=ids)
            st = orc.step(gc, op, st, 1)
        i = c[0] + 256 * (c[1] + 256 * c[2])
        err = np.max(np.abs(st[:, mid] - s1[:, i]))
        assert err < TOL["fp32"], (c, err)
    # observables at full size (several work items per observables block)
    got = lat.observables(gp)
    want = orc.observables(orc.geom(shape), op, s1)
    for k in ("E_total", "E_exch", "E_anis"):
        assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-13 * 256**3), k
    np.testing.assert_allclose(got["m"], want["m"], rtol=1e-11, atol=1e-14)
    assert got["max_norm_dev"] == pytest.approx(want["max_norm_dev"], rel=1e-12, abs=1e-16)
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(40, 24, 20), (96, 96, 64)])  # 75 / 2304 per-site blocks
def test_kick_maximum_same_on_every_fold_path(P, prec, shape):
    """The running maximum of | |s'| - 1 | over the kicks of a run is the same,
    bit for bit, whether each kick's maximum is folded by the next measurement,
    by a reduction before the next kick, or at the end of the run, for both
    kick placements; and it matches the oracle's over the same interval.  The
    larger lattice has more per-block maxima than one pass of the fold loads."""
    op, gp = both_params("zaxis", dt=0.1, Dt=0.4, seed=21)
    got = {}
    for v in (0, 1):
        for fused in (True, False):
            for every in (0, 1, 2):
                lat = P.Lattice(shape, precision=prec, init="random", seed=4)
                lat.set_step_config(v, 0)
                lat.set_kick_fusion(fused)
                lat.kick_norm_dev(reset=True)
                lat.run(gp, first_pulse=0, n_pulses=4, obs_every=every)
                got[(v, fused, every)] = lat.kick_norm_dev()
                lat.close()
    for v in (0, 1):  # bit-identical within one step kernel
        assert len({x for key, x in got.items() if key[0] == v}) == 1, got
    # the unfused and fused steps round differently; d = | |s'| - 1 | ~ 1e-3 is
    # a difference of O(1) numbers, so its fp32 error is absolute (state ulps)
    tol = dict(rel=1e-12) if prec == "fp64" else dict(abs=2e-6)
    assert got[(0, True, 0)] == pytest.approx(got[(1, True, 0)], **tol)
    lat = P.Lattice(shape, precision=prec, init="random", seed=4)
    s0 = np_state(lat)
    want_state, _, dev = orc.run(orc.geom(shape), op, s0, seed=21, first_pulse=0, n_pulses=1)
    lat.kick_norm_dev(reset=True)
    lat.run(gp, first_pulse=0, n_pulses=1)
    assert lat.kick_norm_dev() == pytest.approx(dev, **tol)
    lat.close()


# ------------------------------------------------- other integrators (RK2, RK5) ---
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["rk2mid", "rk5b"])
@pytest.mark.parametrize("kind,precession", [("zaxis", True), ("axis", True), ("none", False)])
@pytest.mark.parametrize("shape,bc", [((40, 24, 20), "periodic"), ((17, 5, 3), "free")])
def test_integrator_per_segment(P, prec, method, kind, precession, shape, bc):
    """RK2 midpoint and Butcher's RK5 (Appendix) inside the pulse schedule:
    each interval (2 steps, kick, 3 steps) against the oracle's steppers and
    kick started from the GPU's state before it."""
    op, _ = both_params(kind, dt=0.1, Dt=0.5, precession=precession)
    kw = dict(PHYS[kind])
    gp = P.Params(seed=13, dt=0.1, Dt=0.5, precession=precession, integrator=method, **kw)
    lat = P.Lattice(shape, bc=bc, precision=prec, init="random", seed=2)
    g = orc.geom(shape, bc)
    prev = np_state(lat)
    for q in range(2):
        lat.run(gp, first_pulse=q, n_pulses=1)
        cur = np_state(lat)
        want = orc.step(g, op, prev, 2, method=method)
        want, _ = orc.kick(g, op, want, op.T, seed=13, r=0, k=q)
        want = orc.step(g, op, want, 3, method=method)
        err = np.max(np.abs(cur - want))
        assert err < TOL[prec], (q, err)
        prev = cur
    # the step alone
    lat.step(gp, 3)
    want = orc.step(g, op, prev, 3, method=method)
    assert np.max(np.abs(np_state(lat) - want)) < TOL[prec]
    lat.close()


def test_integrator_rejections(P):
    shape = (8, 8, 8)
    lat = P.Lattice(shape, precision="fp64", init="random", seed=2)
    gp = P.Params(J=1.0, lam=0.01, T=0.5, dt=0.1, Dt=0.5, seed=1, integrator="rk5b")
    with pytest.raises(P.LLLError) as ei:
        lat.adjoint(gp, 0, 1, ckpt_every=5, wE=1.0, wm=(0, 0, 0))
    assert ei.value.status == P.LLL_EUNSUPPORTED
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,precession", [("zaxis", True), ("axis", False)])
def test_rk2_fused_all_variants(P, prec, kind, precession):
    """Fused RK2 midpoint (two steps per launch, plus a one-step launch for an
    odd count) in every tile shape and z-chunk, against the oracle's stepper;
    and one interval (2 steps with the kick epilogue, then 3 steps)."""
    op, _ = both_params(kind, dt=0.1, Dt=0.5, precession=precession)
    gp = P.Params(seed=31, dt=0.1, Dt=0.5, precession=precession, integrator="rk2mid", **PHYS[kind])
    for shape, bc, bz in STEP_SHAPES:
        N = int(np.prod(shape))
        s0 = rounded(inputs.unit_spins(N, 200 + N), prec)
        g = orc.geom(shape, bc)
        for nst in (3, 4):
            want = orc.step(g, op, s0, nst, method="rk2mid")
            for v in variants(P, prec):
                lat = make_lattice(P, shape, bc, prec, s0)
                lat.set_step_config(v, bz)
                lat.step(gp, nst)
                err = np.max(np.abs(np_state(lat) - want))
                assert err < TOL[prec], (shape, bc, v, bz, nst, err)
                lat.close()
        want = orc.step(g, op, s0, 2, method="rk2mid")
        want, _ = orc.kick(g, op, want, op.T, seed=31, r=0, k=9)
        want = orc.step(g, op, want, 3, method="rk2mid")
        for v in variants(P, prec):
            for fused in (True, False):
                lat = make_lattice(P, shape, bc, prec, s0)
                lat.set_step_config(v, bz)
                lat.set_kick_fusion(fused)
                lat.run(gp, first_pulse=9, n_pulses=1)
                err = np.max(np.abs(np_state(lat) - want))
                assert err < TOL[prec], (shape, bc, v, bz, fused, err)
                lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,precession", [("zaxis", True), ("axis", False), ("none", True)])
def test_rk5_fused_all_variants(P, prec, kind, precession):
    """Fused Butcher RK5 (two launches per step: stages 1-4, then 5-6) in every
    tile shape and z-chunk, on periodic, free, flat, odd and single-site
    lattices, against the oracle's stepper; and one interval of the schedule
    (2 steps with the kick as the epilogue or as its own launch, then 3 steps)
    against the oracle's steps and kick."""
    op, _ = both_params(kind, dt=0.1, Dt=0.5, precession=precession)
    gp = P.Params(seed=37, dt=0.1, Dt=0.5, precession=precession, integrator="rk5b", **PHYS[kind])
    for shape, bc, bz in STEP_SHAPES:
        N = int(np.prod(shape))
        s0 = rounded(inputs.unit_spins(N, 300 + N), prec)
        g = orc.geom(shape, bc)
        want = orc.step(g, op, s0, 3, method="rk5b")
        for v in variants(P, prec):
            lat = make_lattice(P, shape, bc, prec, s0)
            lat.set_step_config(v, bz)
            lat.step(gp, 3)
            err = np.max(np.abs(np_state(lat) - want))
            assert err < TOL[prec], (shape, bc, v, bz, err)
            lat.close()
        want = orc.step(g, op, s0, 2, method="rk5b")
        want, _ = orc.kick(g, op, want, op.T, seed=37, r=0, k=5)
        want = orc.step(g, op, want, 3, method="rk5b")
        for v in variants(P, prec):
            for fused in (True, False):
                lat = make_lattice(P, shape, bc, prec, s0)
                lat.set_step_config(v, bz)
                lat.set_kick_fusion(fused)
                lat.kick_norm_dev(reset=True)
                lat.run(gp, first_pulse=5, n_pulses=1)
                err = np.max(np.abs(np_state(lat) - want))
                assert err < TOL[prec], (shape, bc, v, bz, fused, err)
                lat.close()


def test_rk5_fused_headline_interval(P):
    """The headline lattice (128^3, fp32, dt = 0.2, Dt = 2) with Butcher RK5 in
    its tuned fused configuration: one interval against the oracle started
    from the GPU's state, element by element."""
    import bench
    shape = (128, 128, 128)
    ph = dict(bench.PHYS)
    gp = P.Params(integrator="rk5b", **ph)
    op = orc.Params(J=ph["J"], H=ph["H"], D=ph["D"], e=ph["e"], lam=ph["lam"], T=ph["T"],
                    dt=ph["dt"], Dt=ph["Dt"], precession=True)
    lat = P.Lattice(shape, precision="fp32", init="random", seed=0)
    v, _ = lat.autotune(gp, cache_path=bench.TUNE_CACHE)
    assert v != 0, "the fused RK5 step is not selected"
    prev = np_state(lat)
    with pytest.warns(P.ApplicabilityWarning):
        lat.run(gp, first_pulse=3, n_pulses=1)
    g = orc.geom(shape)
    want = orc.step(g, op, prev, 5, method="rk5b")
    want, _ = orc.kick(g, op, want, op.T, seed=0, r=0, k=3)
    want = orc.step(g, op, want, 5, method="rk5b")
    err = float(np.max(np.abs(np_state(lat) - want)))
    assert err < TOL["fp32"], err
    lat.close()


# --------------------------------------------------------------- autotuner ---
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_autotune_restores_state_and_reuses_its_cache(P, prec, tmp_path):
    """The autotuner times candidate step configurations on the lattice itself;
    afterwards the state and the running kick maximum are exactly what they
    were, the chosen configuration is written to the cache, a second lattice
    of the same key takes it from the cache, a lattice of another key gets a
    line of its own, and a malformed line is ignored.  Runs after tuning give
    the same bits as runs on an untuned lattice set to the same configuration."""
    cache = tmp_path / "tune.txt"
    cache.write_text("this line is not a cache entry\n")
    shape = (48, 40, 36)
    op, gp = both_params("zaxis", dt=0.1, Dt=0.4, seed=5)
    lat = P.Lattice(shape, precision=prec, init="random", seed=8)
    lat.run(gp, first_pulse=0, n_pulses=2)  # leaves a non-zero kick maximum
    s_before = lat.state.clone()
    dev_before = lat.kick_norm_dev()
    v, b = lat.autotune(gp, cache_path=str(cache))
    torch.cuda.synchronize()
    assert torch.equal(lat.state, s_before)
    assert lat.kick_norm_dev() == dev_before
    assert lat.step_config() == (v, b)
    lines = [l.split() for l in cache.read_text().splitlines()]
    entries = [l for l in lines if len(l) >= 3 and l[0] != "this"]
    assert len(entries) == 1 and (int(entries[0][1]), int(entries[0][2])) == (v, b)
    # same key: read from the cache, no new line
    lat2 = P.Lattice(shape, precision=prec, init="random", seed=9)
    assert lat2.autotune(gp, cache_path=str(cache)) == (v, b)
    lines2 = [l for l in cache.read_text().splitlines() if l.strip()]
    assert len(lines2) == len([l for l in lines if l])
    # another key (other shape): one more line
    lat3 = P.Lattice((16, 24, 20), precision=prec, init="random", seed=9)
    lat3.autotune(gp, cache_path=str(cache))
    assert len([l for l in cache.read_text().splitlines() if l.strip()]) == len(lines2) + 1
    # tuned lattice vs an untuned one set to the same configuration: same bits
    ref = P.Lattice(shape, precision=prec, state=s_before.clone())
    ref.set_step_config(v, b)
    fused = [l for l in entries if len(l) >= 4]
    if fused:
        ref.set_kick_fusion(int(fused[0][3]) != 0)
    lat.run(gp, first_pulse=2, n_pulses=2)
    ref.run(gp, first_pulse=2, n_pulses=2)
    torch.cuda.synchronize()
    assert torch.equal(lat.state, ref.state)
    for L_ in (lat, lat2, lat3, ref):
        L_.close()
