"""FP64 CPU oracle for the pulse-noise Landau-Lifshitz-Langevin hot path.

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or calls
anything here; only the test suite, the smoke check and the benchmark's CPU
baseline leg do.  The arithmetic lives in ``lll_oracle.c`` (plain C, FP64,
built with ``-O2 -fno-fast-math -ffp-contract=off``); this module only marshals
numpy arrays through ctypes.

Array convention: a spin state is a float64 array of shape (3, N) with the
site index i = x + Lx*(y + Ly*z) (component-major, as in the paper's Appendix).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lll_oracle.c")
_LIB = os.path.join(_HERE, "liblll_oracle.so")
# the same source built with OpenMP: used only to time the oracle on all host
# cores (its site loops are independent, so it computes identical results)
_LIB_OMP = os.path.join(_HERE, "liblll_oracle_omp.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved), single-threaded and,
    for the all-cores timing, with OpenMP."""
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp"
            subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, out)
    return _LIB


class Geom(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("Lz", C.c_int32), ("bc", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [
        ("J", C.c_double), ("H", C.c_double * 3), ("D", C.c_double), ("e", C.c_double * 3),
        ("D_site", C.c_void_p), ("e_site", C.c_void_p),
        ("lam", C.c_double), ("T", C.c_double), ("dt", C.c_double), ("Dt", C.c_double),
        ("precession", C.c_int32), ("pad_", C.c_int32),
    ]


class Obs(C.Structure):
    _fields_ = [("E_total", C.c_double), ("E_exch", C.c_double), ("E_zeeman", C.c_double),
                ("E_anis", C.c_double), ("m", C.c_double * 3), ("max_norm_dev", C.c_double)]

    def as_dict(self):
        return {"E_total": self.E_total, "E_exch": self.E_exch, "E_zeeman": self.E_zeeman,
                "E_anis": self.E_anis, "m": tuple(self.m), "max_norm_dev": self.max_norm_dev}


@dataclass
class Params:
    """Physical and numerical parameters (units gamma = mu_0 = k_B = 1)."""
    J: float = 1.0
    H: Sequence[float] = (0.0, 0.0, 0.0)
    D: float = 0.0
    e: Sequence[float] = (0.0, 0.0, 1.0)
    lam: float = 0.01
    T: float = 1.0
    dt: float = 0.1
    Dt: float = 1.0
    precession: bool = True
    D_site: Optional[np.ndarray] = None   # (N,)
    e_site: Optional[np.ndarray] = None   # (3, N)
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _Params:
        p = _Params()
        p.J = self.J
        p.H[:] = list(map(float, self.H))
        p.D = self.D
        p.e[:] = list(map(float, self.e))
        self._keep = []
        if self.D_site is not None:
            a = np.ascontiguousarray(self.D_site, dtype=np.float64)
            self._keep.append(a)
            p.D_site = a.ctypes.data
        if self.e_site is not None:
            a = np.ascontiguousarray(self.e_site, dtype=np.float64)
            self._keep.append(a)
            p.e_site = a.ctypes.data
        p.lam = self.lam
        p.T = self.T
        p.dt = self.dt
        p.Dt = self.Dt
        p.precession = 1 if self.precession else 0
        return p


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _bind(C.CDLL(_LIB))
    return _lib


def lib_omp():
    """The OpenMP build (all-cores timing only; OMP_NUM_THREADS sets its threads)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP):
            build(force=True)
        _lib_omp = _bind(C.CDLL(_LIB_OMP))
    return _lib_omp


def _bind(L):
    """Sets the argument and result types of the oracle's C functions."""
    L.orc_threads.restype = C.c_int
    dp = C.POINTER(C.c_double)
    u32p = C.POINTER(C.c_uint32)
    G = C.POINTER(Geom)
    P = C.POINTER(_Params)
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_philox_stream.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32,
                                    C.c_uint32, C.c_uint32, u32p]
    L.orc_u01.argtypes = [C.c_uint32]
    L.orc_u01.restype = C.c_double
    L.orc_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, dp]
    L.orc_init_random_sphere.argtypes = [G, C.c_uint64, C.c_uint32, dp]
    L.orc_init_direction.argtypes = [G, dp, dp]
    for nm in ("orc_heff", "orc_rhs"):
        getattr(L, nm).argtypes = [G, P, dp, dp]
    L.orc_energy_parts.argtypes = [G, P, dp, dp]
    for nm in ("orc_step_rk4", "orc_step_heun", "orc_step_rk2mid", "orc_step_rk5b"):
        getattr(L, nm).argtypes = [G, P, dp, C.c_int64]
    L.orc_rotate.argtypes = [dp, dp, dp]
    L.orc_kick.argtypes = [G, P, C.c_double, C.c_uint64, C.c_uint32, C.c_uint64, dp]
    L.orc_kick.restype = C.c_double
    L.orc_kick_indexed.argtypes = [G, P, C.c_double, C.c_uint64, C.c_uint32, C.c_uint64, u32p, dp]
    L.orc_kick_indexed.restype = C.c_double
    L.orc_observables.argtypes = [G, P, dp, C.POINTER(Obs)]
    L.orc_steps_per_interval.argtypes = [P]
    L.orc_steps_per_interval.restype = C.c_int64
    L.orc_run.argtypes = [G, P, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64, dp, C.c_int32,
                          dp, C.POINTER(Obs)]
    L.orc_run.restype = C.c_double
    L.orc_adjoint.argtypes = [G, P, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64, dp, dp,
                              C.c_double, dp, dp, dp, dp, dp, dp, dp]
    L.orc_adjoint.restype = C.c_int
    L.orc_escape_time.argtypes = [C.c_double] * 6 + [C.c_int32, C.c_int32, C.c_uint64,
                                                      C.c_uint32, C.c_uint32, C.c_int64]
    L.orc_escape_time.restype = C.c_double
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _state(s, N):
    a = np.ascontiguousarray(s, dtype=np.float64).reshape(3, N).copy()
    return a


def geom(shape, bc: str = "periodic") -> Geom:
    Lx, Ly, Lz = shape
    return Geom(int(Lx), int(Ly), int(Lz), 0 if bc == "periodic" else 1)


def nsites(g: Geom) -> int:
    return g.Lx * g.Ly * g.Lz


# ---------------------------------------------------------------- RNG ------
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def philox_stream(seed: int, i0: int, n: int, c1: int, c2: int, c3: int) -> np.ndarray:
    out = np.zeros((n, 4), dtype=np.uint32)
    lib().orc_philox_stream(C.c_uint64(seed), i0, n, c1, c2, c3,
                            out.ctypes.data_as(C.POINTER(C.c_uint32)))
    return out


def u01(w: int) -> float:
    return lib().orc_u01(int(w) & 0xFFFFFFFF)


def gauss3(seed, i, k, r, tag) -> np.ndarray:
    G = np.zeros(3)
    lib().orc_gauss3(C.c_uint64(seed), i, k, r, tag, _dp(G))
    return G


# ------------------------------------------------------------- state -------
def init_random_sphere(g: Geom, seed: int, r: int = 0) -> np.ndarray:
    s = np.zeros((3, nsites(g)))
    lib().orc_init_random_sphere(C.byref(g), C.c_uint64(seed), r, _dp(s))
    return s


def init_direction(g: Geom, d) -> np.ndarray:
    s = np.zeros((3, nsites(g)))
    dd = np.asarray(d, dtype=np.float64)
    lib().orc_init_direction(C.byref(g), _dp(dd), _dp(s))
    return s


def heff(g: Geom, p: Params, s) -> np.ndarray:
    N = nsites(g)
    s = _state(s, N)
    h = np.zeros((3, N))
    pc = p.c()
    lib().orc_heff(C.byref(g), C.byref(pc), _dp(s), _dp(h))
    return h


def rhs(g: Geom, p: Params, s) -> np.ndarray:
    N = nsites(g)
    s = _state(s, N)
    f = np.zeros((3, N))
    pc = p.c()
    lib().orc_rhs(C.byref(g), C.byref(pc), _dp(s), _dp(f))
    return f


def energy_parts(g: Geom, p: Params, s) -> np.ndarray:
    N = nsites(g)
    s = _state(s, N)
    out = np.zeros(3)
    pc = p.c()
    lib().orc_energy_parts(C.byref(g), C.byref(pc), _dp(s), _dp(out))
    return out


def threads(all_cores: bool = True) -> int:
    """Threads the oracle's parallel loops use (the OpenMP build's, or 1)."""
    return int((lib_omp() if all_cores else lib()).orc_threads())


def step(g: Geom, p: Params, s, n_steps: int = 1, method: str = "rk4",
         all_cores: bool = False) -> np.ndarray:
    """n_steps steps of the integrator; all_cores runs the OpenMP build (the
    same results, used to time the oracle on every host core)."""
    N = nsites(g)
    s = _state(s, N)
    pc = p.c()
    fn = {"rk4": "orc_step_rk4", "heun": "orc_step_heun", "rk2mid": "orc_step_rk2mid",
          "rk5b": "orc_step_rk5b"}[method]
    getattr(lib_omp() if all_cores else lib(), fn)(C.byref(g), C.byref(pc), _dp(s), int(n_steps))
    return s


def rotate(s3, phi3) -> np.ndarray:
    a = np.ascontiguousarray(s3, dtype=np.float64)
    b = np.ascontiguousarray(phi3, dtype=np.float64)
    o = np.zeros(3)
    lib().orc_rotate(_dp(a), _dp(b), _dp(o))
    return o


def kick(g: Geom, p: Params, s, T: float, seed: int, r: int, k: int):
    N = nsites(g)
    s = _state(s, N)
    pc = p.c()
    dev = lib().orc_kick(C.byref(g), C.byref(pc), float(T), C.c_uint64(seed), r,
                         C.c_uint64(k), _dp(s))
    return s, dev


def kick_indexed(g: Geom, p: Params, s, T: float, seed: int, r: int, k: int, site_id):
    """Kick of a cut-out whose site j draws its normals from counter site_id[j]."""
    N = nsites(g)
    s = _state(s, N)
    ids = np.ascontiguousarray(site_id, dtype=np.uint32)
    pc = p.c()
    dev = lib().orc_kick_indexed(C.byref(g), C.byref(pc), float(T), C.c_uint64(seed), r,
                                 C.c_uint64(k), ids.ctypes.data_as(C.POINTER(C.c_uint32)), _dp(s))
    return s, dev


def observables(g: Geom, p: Params, s) -> dict:
    N = nsites(g)
    s = _state(s, N)
    pc = p.c()
    o = Obs()
    lib().orc_observables(C.byref(g), C.byref(pc), _dp(s), C.byref(o))
    return o.as_dict()


def steps_per_interval(p: Params) -> int:
    pc = p.c()
    return int(lib().orc_steps_per_interval(C.byref(pc)))


def run(g: Geom, p: Params, s, seed: int, r: int = 0, first_pulse: int = 0, n_pulses: int = 1,
        T_per_pulse=None, obs_every: int = 0):
    """Runs the schedule; returns (state, trace list of dicts, max kick deviation)."""
    N = nsites(g)
    s = _state(s, N)
    pc = p.c()
    nm = (n_pulses // obs_every) if obs_every > 0 else 0
    trace = (Obs * max(nm, 1))()
    Tp = None
    if T_per_pulse is not None:
        Tp = np.ascontiguousarray(T_per_pulse, dtype=np.float64)
    dev = lib().orc_run(C.byref(g), C.byref(pc), C.c_uint64(seed), r, C.c_uint64(first_pulse),
                        int(n_pulses), _dp(Tp) if Tp is not None else None, int(obs_every),
                        _dp(s), trace)
    if dev < 0:
        raise ValueError("invalid schedule: Dt/dt must be a positive integer")
    return s, [trace[i].as_dict() for i in range(nm)], dev


def adjoint(g: Geom, p: Params, s0, seed: int, r: int = 0, first_pulse: int = 0,
            n_pulses: int = 1, T_per_pulse=None, wE: float = 1.0, wm=(0.0, 0.0, 0.0), cot=None):
    """Loss L = <cot, s_T> + wE*E(s_T) + wm.m(s_T) and its gradients (dict);
    cot: optional (3, N) cotangent of the final state."""
    N = nsites(g)
    s0 = _state(s0, N)
    pc = p.c()
    wm_a = np.asarray(wm, dtype=np.float64)
    loss = np.zeros(1)
    gs0 = np.zeros((3, N))
    gH = np.zeros(3)
    gJ = np.zeros(1)
    gD = np.zeros(N if p.D_site is not None else 1)
    Tp = None
    if T_per_pulse is not None:
        Tp = np.ascontiguousarray(T_per_pulse, dtype=np.float64)
    ct = _state(cot, N) if cot is not None else None
    rc = lib().orc_adjoint(C.byref(g), C.byref(pc), C.c_uint64(seed), r, C.c_uint64(first_pulse),
                           int(n_pulses), _dp(Tp) if Tp is not None else None, _dp(s0), float(wE),
                           _dp(wm_a), _dp(ct) if ct is not None else None, _dp(loss), _dp(gs0),
                           _dp(gH), _dp(gJ), _dp(gD))
    if rc != 0:
        raise ValueError(f"orc_adjoint failed: {rc}")
    return {"loss": float(loss[0]), "g_s0": gs0, "g_H": gH, "g_J": float(gJ[0]),
            "g_D": gD if p.D_site is not None else float(gD[0])}


# --------------------------------------------------------------------------
# Escape of a uniaxial spin in a transverse field (Sec. III.B)
# --------------------------------------------------------------------------
_METHOD = {"rk4": 0, "rk2mid": 1, "rk5b": 2}


def escape_time(D: float, H: float, lam: float, T: float, dt: float, Dt: float, run: int,
                seed: int = 0, r: int = 0, max_pulses: int = 10**6, method: str = "rk4",
                precession: bool = True) -> float:
    """First-passage time of one run (see orc_escape_time); -1 if none within
    max_pulses intervals."""
    return float(lib().orc_escape_time(D, H, lam, T, dt, Dt, 1 if precession else 0,
                                       _METHOD[method], C.c_uint64(seed), r, run,
                                       int(max_pulses)))


def escape_F(h: float) -> float:
    """F(h) of the low-damping escape rate (Sec. III.B), from the paper's
    one-dimensional form: the integral over u in [0, 1] of
    x_c/(1 - x_c^2 u^2) [u (2(1 - h) - x_c^2 u^2)^2 / sqrt(1 - u^2) + x_c sqrt(1 - u^2)],
    x_c = 2 sqrt(h (1 - h)), evaluated with u = sin v (which removes the
    endpoint singularity) by adaptive quadrature."""
    from scipy.integrate import quad
    xc = 2.0 * np.sqrt(h * (1.0 - h))

    def g(v):
        sv, cv = np.sin(v), np.cos(v)
        # du/sqrt(1-u^2) = dv, sqrt(1-u^2) du = cos^2 v dv
        return xc / (1.0 - xc * xc * sv * sv) * (sv * (2.0 * (1.0 - h) - xc * xc * sv * sv) ** 2
                                                 + xc * cv * cv)
    if h == 0.5:  # x_c = 1: 1/(1 - sin^2 v) cancels against the bracket
        def g(v):  # noqa: F811
            sv, cv = np.sin(v), np.cos(v)
            return sv * cv * cv + 1.0
    val, _ = quad(g, 0.0, np.pi / 2, epsabs=1e-13, epsrel=1e-12, limit=200)
    return float(val)


def escape_F_contour(h: float) -> float:
    """F(h) from its definition as a contour integral over the separatrix
    f(x, phi) = x^2 + 2h sqrt(1 - x^2) cos(phi) = 2h around one well (Sec.
    III.B), x = cos(theta): one half of the closed curve, phi(x) =
    arccos[(2h - x^2) / (2h sqrt(1 - x^2))] for x from 0 to x_c, counted twice
    (the other half is its mirror phi -> -phi), with the factor 1/2 of the
    definition; parametrised by the angle phi itself to avoid the endpoint
    singularities of dphi/dx."""
    from scipy.integrate import quad
    from scipy.optimize import brentq
    xc = 2.0 * np.sqrt(h * (1.0 - h))

    def x_of_phi(ph):
        # f(x, phi) = 2h on the branch x in [0, x_c]
        c = np.cos(ph)
        fun = lambda x: x * x + 2.0 * h * np.sqrt(max(1.0 - x * x, 0.0)) * c - 2.0 * h  # noqa: E731
        if ph == 0.0:
            return 0.0
        return brentq(fun, 1e-15, xc, xtol=1e-15, rtol=1e-15, maxiter=200)

    def integrand(ph):
        x = x_of_phi(ph)
        sq = np.sqrt(max(1.0 - x * x, 1e-300))
        fx = 2.0 * x - 2.0 * h * x * np.cos(ph) / sq
        fph = -2.0 * h * sq * np.sin(ph)
        # dx/dphi from f(x(phi), phi) = const: fx dx + fph dphi = 0
        dxdph = -fph / fx if fx != 0.0 else 0.0
        return (1.0 - x * x) * fx - fph / (1.0 - x * x) * dxdph
    val, _ = quad(integrand, 0.0, np.pi, epsabs=1e-11, epsrel=1e-10, limit=400)
    return float(abs(val))


def escape_rate_theory(D: float, H: float, lam: float, T: float, regime: str) -> float:
    """Escape rate of Sec. III.B: Gamma = omega_0/(2 pi) A exp(-sigma (1 - h)^2),
    sigma = D/T, omega_0 = 2 D sqrt(1 - h^2) (gamma = 1); A = 1 ("ID"),
    A = lambda sigma F(h) ("LD") or A_LD / (1 + A_LD) ("ILD")."""
    h = H / (2.0 * D)
    sigma = D / T
    w0 = 2.0 * D * np.sqrt(1.0 - h * h)
    if regime == "ID":
        A = 1.0
    else:
        ald = lam * sigma * escape_F(h)
        A = ald if regime == "LD" else ald / (1.0 + ald)
    return float(w0 / (2.0 * np.pi) * A * np.exp(-sigma * (1.0 - h) ** 2))
