"""Pins of the FP64 oracle against what the paper and the mathematics fix:
closed forms (single spin in a field, noise-only decay), invariants
(conserved total spin, energy dissipation), brute force on tiny lattices,
integrator orders, textbook equilibria (Langevin function, uniaxial
Boltzmann average, open Heisenberg chain) and finite differences for the
adjoint.  A plausible mistake anywhere in the oracle (a dropped term, a wrong
sign or index, a transposed operand) fails at least one of these."""
import itertools
import json
import os

import numpy as np
import pytest
from scipy import integrate

from tests import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def langevin(x):
    return 1.0 / np.tanh(x) - 1.0 / x


# ------------------------------------------------------------------ P8 -----
def _brute_heff_energy(shape, bc, J, H, D, e, s):
    """Dense-adjacency effective field and energy built from coordinates."""
    Lx, Ly, Lz = shape
    N = Lx * Ly * Lz
    coords = [(x, y, z) for z in range(Lz) for y in range(Ly) for x in range(Lx)]
    A = np.zeros((N, N))
    bonds = []
    for i, (x, y, z) in enumerate(coords):
        for ax, L in enumerate(shape):
            for d in (+1, -1):
                c = [x, y, z]
                c[ax] += d
                if not 0 <= c[ax] < L:
                    if bc == "free":
                        continue
                    c[ax] %= L
                j = c[0] + Lx * (c[1] + Ly * c[2])
                A[i, j] += 1.0
                if d == +1:
                    bonds.append((i, j))
    e = np.asarray(e, float) / np.linalg.norm(e)
    se = e @ s
    h = J * (s @ A.T) + np.asarray(H, float)[:, None] + 2 * D * se[None, :] * e[:, None]
    Eex = -J * sum(s[:, i] @ s[:, j] for i, j in bonds)
    Ez = -np.sum(np.asarray(H, float) @ s)
    Ea = -D * np.sum(se**2)
    return h, np.array([Eex, Ez, Ea]), A


SHAPES = [(1, 1, 1), (2, 1, 1), (2, 2, 2), (3, 3, 3), (2, 3, 5), (5, 1, 2)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_heff_energy_brute_force(orc, shape, bc):
    N = int(np.prod(shape))
    s = inputs.unit_spins(N, 3)
    p = orc.Params(J=0.7, H=(0.1, -0.2, 0.3), D=0.4, e=(1.0, 2.0, 2.0))
    g = orc.geom(shape, bc)
    h_ref, E_ref, A = _brute_heff_energy(shape, bc, p.J, p.H, p.D, p.e, s)
    np.testing.assert_allclose(orc.heff(g, p, s), h_ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(orc.energy_parts(g, p, s), E_ref, rtol=1e-13, atol=1e-13)
    assert np.array_equal(A, A.T)  # the stencil is symmetric (used by the adjoint)


def test_heff_is_minus_energy_gradient(orc):
    """h_i = -dE/ds_i, checked by central finite differences."""
    shape = (3, 2, 4)
    N = 24
    s = inputs.unit_spins(N, 5)
    D_site, e_site = inputs.site_anisotropy(N, 6)
    p = orc.Params(J=1.3, H=(0.2, 0.1, -0.4), D_site=D_site, e_site=e_site)
    for bc in ("periodic", "free"):
        g = orc.geom(shape, bc)
        h = orc.heff(g, p, s)
        eps = 1e-6
        for c, i in [(0, 0), (1, 5), (2, 17), (0, 23), (2, 11)]:
            sp = s.copy(); sp[c, i] += eps
            sm = s.copy(); sm[c, i] -= eps
            dE = (orc.energy_parts(g, p, sp).sum() - orc.energy_parts(g, p, sm).sum()) / (2 * eps)
            assert abs(-dE - h[c, i]) < 1e-8


def test_ordered_state_energy_closed_form(orc):
    """Fully aligned state: E_exch = -J * (number of bonds); PBC has 3N bonds,
    free boundaries 3 L^2 (L - 1)."""
    L = 5
    p = orc.Params(J=1.0)
    s = np.zeros((3, L**3)); s[2] = 1
    assert orc.energy_parts(orc.geom((L, L, L)), p, s)[0] == pytest.approx(-3 * L**3)
    assert orc.energy_parts(orc.geom((L, L, L), "free"), p, s)[0] == pytest.approx(-3 * L * L * (L - 1))


# ---------------------------------------------------------- RHS identities --
def test_rhs_identities(orc):
    """f is perpendicular to s (length conserved by the exact flow), and the
    energy dissipation identity sum_i h_i.f_i = lambda sum_i |s_i x h_i|^2
    holds (dE/dt = -lambda sum |s x h|^2 <= 0); the slow equation has the same
    dissipation and no precession part."""
    shape = (4, 3, 2)
    N = 24
    s = inputs.unit_spins(N, 8)
    for prec in (True, False):
        p = orc.Params(J=1.0, H=(0.1, 0.0, 0.5), D=0.3, e=(0, 1, 1), lam=0.07, precession=prec)
        g = orc.geom(shape)
        f = orc.rhs(g, p, s)
        h = orc.heff(g, p, s)
        np.testing.assert_allclose(np.sum(s * f, axis=0), 0.0, atol=1e-14)
        sxh = np.cross(s.T, h.T).T
        assert np.sum(h * f) == pytest.approx(p.lam * np.sum(sxh**2), rel=1e-12)
        if prec:
            p0 = orc.Params(J=1.0, H=(0.1, 0.0, 0.5), D=0.3, e=(0, 1, 1), lam=0.0)
            f0 = orc.rhs(g, p0, s)
            np.testing.assert_allclose(np.sum(h * f0, axis=0), 0.0, atol=1e-13)


# ------------------------------------------------------------------ P1/P2 --
def _single_spin_exact(s0, H, lam, t, precession=True):
    """Noise-free spin in a field H along z: Eq. (11)'s map for s_z over a time t
    with the precession added (azimuth turns by -H t)."""
    tau = lam * H * t
    sz0 = s0[2]
    sz = (np.sinh(tau) + sz0 * np.cosh(tau)) / (np.cosh(tau) + sz0 * np.sinh(tau))
    sp = np.sqrt(1 - sz**2)
    psi = np.arctan2(s0[1], s0[0]) - (H * t if precession else 0.0)
    return np.array([sp * np.cos(psi), sp * np.sin(psi), sz])


def _single_spin_run(orc, method, dt, t, lam, H, s0, precession=True):
    g = orc.geom((1, 1, 1))
    p = orc.Params(J=0.0, H=(0, 0, H), lam=lam, dt=dt, precession=precession)
    n = int(round(t / dt))
    return orc.step(g, p, s0.reshape(3, 1), n, method)[:, 0]


S0_150 = np.array([np.sin(np.radians(150)) * np.cos(0.3), np.sin(np.radians(150)) * np.sin(0.3),
                   np.cos(np.radians(150))])


def test_single_spin_closed_form_rk4(orc):
    """RK4 on a spin in H = z: agrees with the exact map and its error drops by
    ~16 per halving of dt (fourth order)."""
    H, lam, t = 1.0, 0.04, 10.0
    ex = _single_spin_exact(S0_150, H, lam, t)
    errs = [np.max(np.abs(_single_spin_run(orc, "rk4", dt, t, lam, H, S0_150) - ex))
            for dt in (0.2, 0.1, 0.05)]
    assert errs[2] < 1e-6
    for a, b in zip(errs, errs[1:]):
        assert 13 < a / b < 19


def test_single_spin_slow_equation(orc):
    """Slow equation: same s_z(t), azimuth constant."""
    H, lam, t = 1.0, 0.1, 10.0
    ex = _single_spin_exact(S0_150, H, lam, t, precession=False)
    got = _single_spin_run(orc, "rk4", 0.5, t, lam, H, S0_150, precession=False)
    np.testing.assert_allclose(got, ex, atol=1e-6)


@pytest.mark.parametrize("method,order,dts", [("heun", 2, (0.02, 0.01)), ("rk2mid", 2, (0.02, 0.01)),
                                              ("rk5b", 5, (0.2, 0.1))])
def test_integrator_orders(orc, method, order, dts):
    H, lam, t = 1.0, 0.04, 6.0
    ex = _single_spin_exact(S0_150, H, lam, t)
    e1, e2 = [np.max(np.abs(_single_spin_run(orc, method, dt, t, lam, H, S0_150) - ex)) for dt in dts]
    assert 0.75 * 2**order < e1 / e2 < 1.25 * 2**order


def test_rk4_and_rk5_converge_to_same_lattice_trajectory(orc):
    g = orc.geom((3, 2, 2))
    s0 = inputs.unit_spins(12, 11)
    p = orc.Params(J=1.0, H=(0, 0, 0.3), D=0.2, lam=0.05, dt=0.0025)
    a = orc.step(g, p, s0, 800, "rk4")
    b = orc.step(g, p, s0, 800, "rk5b")
    np.testing.assert_allclose(a, b, atol=1e-9)


# ------------------------------------------------------------------ P3 -----
def test_lambda0_conserves_total_spin(orc):
    """lambda = 0, isotropic exchange: S = sum s_i is a linear first integral,
    preserved by RK4 to rounding; with H and easy axis along z, S_z is."""
    g = orc.geom((3, 3, 3))
    s0 = inputs.unit_spins(27, 12)
    p = orc.Params(J=1.0, lam=0.0, dt=0.1)
    s = orc.step(g, p, s0, 500)
    np.testing.assert_allclose(s.sum(axis=1), s0.sum(axis=1), atol=1e-12)
    p = orc.Params(J=1.0, H=(0, 0, 0.7), D=0.5, e=(0, 0, 1), lam=0.0, dt=0.1)
    s = orc.step(g, p, s0, 500)
    assert abs(s[2].sum() - s0[2].sum()) < 1e-12
    assert abs(s[0].sum() - s0[0].sum()) > 1e-3   # S_x is not conserved with a field


def test_lambda0_energy_drift_fourth_order(orc):
    """lambda = 0: E is conserved only up to the integrator error; its drift must
    shrink at least like dt^4 (measured close to dt^5 for this flow)."""
    g = orc.geom((4, 4, 4))
    s0 = inputs.unit_spins(64, 13)
    p0 = orc.Params(J=1.0, H=(0, 0, 0.1), D=0.05, lam=0.0)
    E0 = orc.energy_parts(g, p0, s0).sum()
    drift = []
    for dt in (0.1, 0.05, 0.025):
        p = orc.Params(J=1.0, H=(0, 0, 0.1), D=0.05, lam=0.0, dt=dt)
        s = orc.step(g, p, s0, int(round(4.0 / dt)))
        drift.append(abs(orc.energy_parts(g, p, s).sum() - E0))
    for a, b in zip(drift, drift[1:]):
        assert 14 < a / b < 40


def test_zero_temperature_energy_decreases(orc):
    g = orc.geom((4, 3, 3))
    s = inputs.unit_spins(36, 14)
    p = orc.Params(J=1.0, H=(0, 0, 0.2), D=0.1, lam=0.1, T=0.0, dt=0.05, Dt=0.1)
    E = [orc.energy_parts(g, p, s).sum()]
    for _ in range(40):
        s, _, dev = orc.run(g, p, s, seed=1, n_pulses=1)
        E.append(orc.energy_parts(g, p, s).sum())
    assert np.all(np.diff(E) < 0)
    # T = 0 kick is a pure renormalisation
    s = s * 1.01
    sk, dev = orc.kick(g, p, s, 0.0, seed=1, r=0, k=3)
    np.testing.assert_allclose(np.linalg.norm(sk, axis=0), 1.0, atol=1e-15)
    np.testing.assert_allclose(sk, s / np.linalg.norm(s, axis=0), atol=1e-15)
    assert dev == pytest.approx(np.max(np.abs(np.linalg.norm(s, axis=0) - 1)), rel=1e-12)


# ------------------------------------------------------------------ rotation
def test_rotation_matches_scipy(orc):
    """Eq. (6) equals the rotation by the rotation vector phi (right-hand sense),
    as computed by scipy's independent Rotation class."""
    from scipy.spatial.transform import Rotation
    r = np.random.default_rng(3)
    for _ in range(200):
        s = r.standard_normal(3)
        ph = r.standard_normal(3) * r.choice([1e-6, 0.1, 1.0, 3.0])
        np.testing.assert_allclose(orc.rotate(s, ph), Rotation.from_rotvec(ph).apply(s),
                                   rtol=1e-12, atol=1e-13)
    s = np.array([0.3, -0.4, 0.5])
    assert np.array_equal(orc.rotate(s, np.zeros(3)), s)


# ------------------------------------------------------------------ P4 -----
def _f_decay(s2):
    """Exact per-pulse factor of <s> for isotropic Gaussian rotation vectors with
    per-component variance s2: <s'_z> = (1 + 2 <cos|phi|>)/3 for s = z and
    <cos|phi|> = (1 - s2) exp(-s2/2) (Maxwell-distributed |phi|)."""
    return (1 + 2 * (1 - s2) * np.exp(-s2 / 2)) / 3


def _g_decay(s2):
    """Per-pulse factor of <P2(s_z)> (l = 2 character of the rotation)."""
    return (1 + 2 * (1 - s2) * np.exp(-s2 / 2) + 2 * (1 - 4 * s2) * np.exp(-2 * s2)) / 5


def test_noise_only_decay_exact(orc):
    """J = H = D = 0: only kicks act.  From the ordered state <s_z> after k
    kicks is f(sigma^2)^k with sigma^2 = 2 lambda T Delta t, and <P2(s_z)> after
    one kick is g(sigma^2); the statistical error with 2^20 spins is ~3e-4."""
    g = orc.geom((128, 128, 64))
    N = 128 * 128 * 64
    p = orc.Params(J=0.0, lam=0.01, T=1.0, dt=0.25, Dt=10.0)
    s2 = 2 * p.lam * p.T * p.Dt
    s = np.zeros((3, N)); s[2] = 1
    s1, _ = orc.kick(g, p, s, p.T, seed=7, r=0, k=0)
    mz = s1[2].mean()
    se = s1[2].std() / np.sqrt(N)
    assert abs(mz - _f_decay(s2)) < 5 * se
    assert abs(mz - np.exp(-s2)) > 5 * se          # the discrete factor is not e^{-s2}
    P2 = (1.5 * s1[2]**2 - 0.5)
    assert abs(P2.mean() - _g_decay(s2)) < 5 * P2.std() / np.sqrt(N)
    s2k, _ = orc.kick(g, p, s1, p.T, seed=7, r=0, k=1)
    assert abs(s2k[2].mean() - _f_decay(s2)**2) < 5 * s2k[2].std() / np.sqrt(N)


def test_golden_noise_only_paper_values(orc):
    """Fig. 1 setting of Sec. III.A: lambda = 0.01, T = 1, delta t = 0.25,
    Delta t = 10; the paper prints phi_RMS = sqrt(Lambda_N Delta t) ~ 0.45 and
    states that the pulses reproduce m = m0 exp(-Lambda_N t) (Eq. (10)) well."""
    with open(os.path.join(GOLDEN, "noise_only_fig1.json")) as fh:
        gold = json.load(fh)
    g = orc.geom((40, 40, 40))
    N = 40**3
    p = orc.Params(J=0.0, lam=gold["lambda"], T=gold["T"], dt=gold["dt"], Dt=gold["Dt"])
    s = np.zeros((3, N)); s[2] = 1
    s, trace, _ = orc.run(g, p, s, seed=3, n_pulses=gold["n_pulses"], obs_every=1)
    mz = np.array([t["m"][2] for t in trace])
    # recover sigma^2 from the first pulse by inverting the exact factor
    from scipy.optimize import brentq
    s2 = brentq(lambda x: _f_decay(x) - mz[0], 1e-4, 1.0)
    assert abs(np.sqrt(s2) - gold["phi_rms"]) < gold["phi_rms_tol"]
    t = gold["Dt"] * np.arange(1, gold["n_pulses"] + 1)
    cont = np.exp(-2 * gold["lambda"] * gold["T"] * t)
    assert np.max(np.abs(mz - cont)) < gold["max_abs_dev_from_eq10"]


# ------------------------------------------------------------- equilibria --
def _time_average(trace, key, burn):
    v = np.array([key(t) for t in trace])[burn:]
    nb = 20
    bm = v[: len(v) // nb * nb].reshape(nb, -1).mean(axis=1)
    return v.mean(), bm.std(ddof=1) / np.sqrt(nb)


def test_langevin_single_spin_equilibrium(orc):
    """Independent spins (J = 0) in H = z at temperature T: <s_z> = L(H/T)
    (the exact result the paper compares against in Sec. III.A), here with
    Lambda_N Delta t = 0.02 so that the pulse bias is small."""
    g = orc.geom((16, 16, 16))
    p = orc.Params(J=0.0, H=(0, 0, 1.0), lam=0.1, T=1.0, dt=0.05, Dt=0.1)
    s = orc.init_random_sphere(g, seed=2)
    s, trace, _ = orc.run(g, p, s, seed=9, n_pulses=1500, obs_every=1)
    mean, err = _time_average(trace, lambda t: t["m"][2], burn=300)
    assert abs(mean - langevin(1.0)) < 4 * err + 0.004, (mean, err)


def test_uniaxial_single_spin_equilibrium(orc):
    """Independent uniaxial spins E = -D s_z^2: <s_z^2> equals the Boltzmann
    average computed by quadrature."""
    D, T = 1.0, 1.0
    num = integrate.quad(lambda x: x * x * np.exp(D / T * x * x), -1, 1)[0]
    den = integrate.quad(lambda x: np.exp(D / T * x * x), -1, 1)[0]
    g = orc.geom((16, 16, 16))
    p = orc.Params(J=0.0, D=D, e=(0, 0, 1), lam=0.1, T=T, dt=0.05, Dt=0.1)
    s = orc.init_random_sphere(g, seed=4)
    s, trace, _ = orc.run(g, p, s, seed=10, n_pulses=1500, obs_every=1)
    N = 16**3
    mean, err = _time_average(trace, lambda t: -t["E_anis"] / (N * D), burn=300)
    assert abs(mean - num / den) < 4 * err + 0.004, (mean, err, num / den)


def test_open_chain_bond_correlation(orc):
    """Open classical Heisenberg chain (free boundaries, H = D = 0):
    <s_i . s_{i+1}> = L(J/T) for every bond (textbook result)."""
    Nc = 4096
    g = orc.geom((Nc, 1, 1), "free")
    p = orc.Params(J=1.0, lam=0.1, T=1.0, dt=0.05, Dt=0.1)
    s = orc.init_random_sphere(g, seed=5)
    s, trace, _ = orc.run(g, p, s, seed=11, n_pulses=1500, obs_every=1)
    mean, err = _time_average(trace, lambda t: -t["E_exch"] / (Nc - 1), burn=300)
    assert abs(mean - langevin(1.0)) < 4 * err + 0.004, (mean, err)


# ------------------------------------------------------------------ P9/P10 --
def test_slow_equation_lambda_scaling(orc):
    """Precession dropped: (lambda, dt, Dt) and (lambda/c, c dt, c Dt) give the
    same map (same lambda dt and Lambda_N Delta t)."""
    g = orc.geom((4, 4, 3))
    s0 = inputs.unit_spins(48, 15)
    kw = dict(J=1.0, H=(0, 0, 0.2), D=0.1, T=0.8, precession=False)
    a, _, _ = orc.run(g, orc.Params(lam=0.02, dt=2.0, Dt=4.0, **kw), s0, seed=3, n_pulses=5)
    b, _, _ = orc.run(g, orc.Params(lam=0.08, dt=0.5, Dt=1.0, **kw), s0, seed=3, n_pulses=5)
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_schedule_identity(orc):
    """run(K) equals the manual step(n1) / kick(k) / step(n2) sequence and the
    split K1 + (K - K1) continuation (the counter-based stream is stateless)."""
    g = orc.geom((3, 4, 5))
    s0 = inputs.unit_spins(60, 16)
    p = orc.Params(J=1.0, H=(0, 0, 0.1), D=0.05, lam=0.01, T=1.0, dt=0.1, Dt=0.5)
    full, _, _ = orc.run(g, p, s0, seed=21, r=3, first_pulse=10, n_pulses=4)
    s = s0.copy()
    for k in range(10, 14):
        s = orc.step(g, p, s, 2)
        s, _ = orc.kick(g, p, s, p.T, seed=21, r=3, k=k)
        s = orc.step(g, p, s, 3)
    assert np.array_equal(s, full)
    a, _, _ = orc.run(g, p, s0, seed=21, r=3, first_pulse=10, n_pulses=1)
    b, _, _ = orc.run(g, p, a, seed=21, r=3, first_pulse=11, n_pulses=3)
    assert np.array_equal(b, full)
    with pytest.raises(ValueError):
        orc.run(g, orc.Params(dt=0.3, Dt=1.0), s0, seed=1)


# ------------------------------------------------------------------ P12 ----
@pytest.mark.parametrize("precession", [True, False])
def test_adjoint_finite_differences(orc, precession):
    """Gradients of L = E(s_T) + m_z(s_T) w.r.t. H, J, D_i and s_0 agree with
    central finite differences of the forward run."""
    shape = (3, 4, 2)
    N = 24
    g = orc.geom(shape)
    D_site, e_site = inputs.site_anisotropy(N, 17)
    s0 = inputs.near_ordered_spins(N, 18)
    base = dict(J=1.0, H=(0.05, -0.02, 0.2), lam=0.05, T=0.5, dt=0.1, Dt=0.4, precession=precession)
    wm = (0.0, 0.0, 1.0)
    kw = dict(seed=4, r=0, first_pulse=0, n_pulses=2, wE=1.0, wm=wm)
    p = orc.Params(D_site=D_site, e_site=e_site, **base)
    res = orc.adjoint(g, p, s0, **kw)

    def L(**over):
        b = dict(base); d = D_site.copy(); s = s0.copy()
        if "H" in over:
            b["H"] = over["H"]
        if "J" in over:
            b["J"] = over["J"]
        if "D" in over:
            d = over["D"]
        if "s" in over:
            s = over["s"]
        pp = orc.Params(D_site=d, e_site=e_site, **b)
        sT, _, _ = orc.run(g, pp, s, seed=4, n_pulses=2)
        o = orc.observables(g, pp, sT)
        return o["E_total"] + o["m"][2]

    assert res["loss"] == pytest.approx(L(), rel=1e-14)
    eps = 1e-6
    for c in range(3):
        Hp = list(base["H"]); Hp[c] += eps
        Hm = list(base["H"]); Hm[c] -= eps
        fd = (L(H=tuple(Hp)) - L(H=tuple(Hm))) / (2 * eps)
        assert abs(fd - res["g_H"][c]) < 1e-6 * max(1, abs(fd))
    fd = (L(J=1.0 + eps) - L(J=1.0 - eps)) / (2 * eps)
    assert abs(fd - res["g_J"]) < 1e-6 * max(1, abs(fd))
    for i in (0, 7, 23):
        dp = D_site.copy(); dp[i] += eps
        dm = D_site.copy(); dm[i] -= eps
        fd = (L(D=dp) - L(D=dm)) / (2 * eps)
        assert abs(fd - res["g_D"][i]) < 1e-6 * max(1, abs(fd))
    v = inputs.unit_spins(N, 19)
    fd = (L(s=s0 + eps * v) - L(s=s0 - eps * v)) / (2 * eps)
    assert abs(fd - np.sum(res["g_s0"] * v)) < 1e-6 * max(1, abs(fd))


def test_adjoint_uniform_D(orc):
    """Uniform D: the returned g_D is dL/dD (sum over sites)."""
    g = orc.geom((3, 3, 3))
    s0 = inputs.near_ordered_spins(27, 20)
    base = dict(J=1.0, H=(0, 0, 0.2), e=(0, 0, 1), lam=0.05, T=0.5, dt=0.1, Dt=0.4)
    res = orc.adjoint(g, orc.Params(D=0.1, **base), s0, seed=2, n_pulses=2, wE=1.0, wm=(0, 0, 1))

    def L(D):
        pp = orc.Params(D=D, **base)
        sT, _, _ = orc.run(g, pp, s0, seed=2, n_pulses=2)
        o = orc.observables(g, pp, sT)
        return o["E_total"] + o["m"][2]
    eps = 1e-6
    fd = (L(0.1 + eps) - L(0.1 - eps)) / (2 * eps)
    assert abs(fd - res["g_D"]) < 1e-6 * max(1, abs(fd))


@pytest.mark.parametrize("precession", [True, False])
def test_adjoint_with_final_state_cotangent(orc, precession):
    """A loss that the caller computes from s_T itself enters the adjoint as
    its cotangent c = dL/ds_T.  For L = <c, s_T> + m_z(s_T) with a fixed
    random c, the gradients w.r.t. s_0, H, J and D_i agree with central finite
    differences of the forward run, and c alone (wE = 0, wm = 0) is linear:
    the gradients of c1 + c2 are the sums of those of c1 and c2."""
    shape = (3, 2, 3)
    N = 18
    g = orc.geom(shape, "free")
    D_site, e_site = inputs.site_anisotropy(N, 31)
    s0 = inputs.unit_spins(N, 32)
    c = inputs.rng(33).standard_normal((3, N))
    base = dict(J=0.9, H=(0.1, 0.0, -0.3), lam=0.04, T=0.6, dt=0.1, Dt=0.3, precession=precession)
    kw = dict(seed=7, r=1, first_pulse=3, n_pulses=2)
    p = orc.Params(D_site=D_site, e_site=e_site, **base)
    res = orc.adjoint(g, p, s0, wE=0.0, wm=(0.0, 0.0, 1.0), cot=c, **kw)

    def L(**over):
        b = dict(base)
        for k in ("H", "J"):
            if k in over:
                b[k] = over[k]
        pp = orc.Params(D_site=over.get("D", D_site), e_site=e_site, **b)
        sT, _, _ = orc.run(g, pp, over.get("s", s0), **kw)
        return float(np.sum(c * sT)) + orc.observables(g, pp, sT)["m"][2]

    assert res["loss"] == pytest.approx(L(), rel=1e-13)
    eps = 1e-6
    for comp in range(3):
        Hp = list(base["H"]); Hp[comp] += eps
        Hm = list(base["H"]); Hm[comp] -= eps
        fd = (L(H=tuple(Hp)) - L(H=tuple(Hm))) / (2 * eps)
        assert abs(fd - res["g_H"][comp]) < 1e-6 * max(1, abs(fd))
    fd = (L(J=0.9 + eps) - L(J=0.9 - eps)) / (2 * eps)
    assert abs(fd - res["g_J"]) < 1e-6 * max(1, abs(fd))
    for i in (0, 9, 17):
        dp = D_site.copy(); dp[i] += eps
        dm = D_site.copy(); dm[i] -= eps
        fd = (L(D=dp) - L(D=dm)) / (2 * eps)
        assert abs(fd - res["g_D"][i]) < 1e-6 * max(1, abs(fd))
    for seed in (34, 35):
        v = inputs.unit_spins(N, seed)
        fd = (L(s=s0 + eps * v) - L(s=s0 - eps * v)) / (2 * eps)
        assert abs(fd - np.sum(res["g_s0"] * v)) < 1e-6 * max(1, abs(fd))
    # linearity in the cotangent
    c2 = inputs.rng(36).standard_normal((3, N))
    r1 = orc.adjoint(g, p, s0, wE=0.0, cot=c, **kw)
    r2 = orc.adjoint(g, p, s0, wE=0.0, cot=c2, **kw)
    r12 = orc.adjoint(g, p, s0, wE=0.0, cot=c + c2, **kw)
    np.testing.assert_allclose(r12["g_s0"], r1["g_s0"] + r2["g_s0"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r12["g_D"], r1["g_D"] + r2["g_D"], rtol=1e-10, atol=1e-12)
    assert r12["g_J"] == pytest.approx(r1["g_J"] + r2["g_J"], rel=1e-10, abs=1e-12)
