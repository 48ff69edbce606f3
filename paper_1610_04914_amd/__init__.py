"""Python binding of liblll, the MI355X (gfx950) pulse-noise
Landau-Lifshitz-Langevin library (Garanin, arXiv:1610.04914).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblll.so``; PyTorch provides device memory and the HIP stream.  The
functions ``lll_*`` mirror the C ABI of ``include/lll.h`` one to one;
``Lattice`` and ``Batch`` are thin handles over them.  There is no CPU
fallback: importing works anywhere, but any call fails loudly when the
library or a GPU is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblll.so")

LLL_OK = 0
LLL_EINVAL, LLL_ENOMEM, LLL_EDEVICE, LLL_EUNSUPPORTED, LLL_ENONFINITE = -1, -2, -3, -4, -5
LLL_WARN_APPLICABILITY, LLL_WARN_NORM = 1, 2
LLL_FP64, LLL_FP32 = 0, 1
LLL_BC_PERIODIC, LLL_BC_FREE = 0, 1
LLL_INIT_RANDOM_SPHERE, LLL_INIT_DIRECTION, LLL_INIT_KEEP = 0, 1, 2


class LLLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"liblll status {status}: {msg}")
        self.status = status


class ApplicabilityWarning(UserWarning):
    """LLL_WARN_APPLICABILITY: Eq. (8)/(9) or the step-size rule is violated."""


class NormDriftWarning(UserWarning):
    """LLL_WARN_NORM: a measured state's | |s_i| - 1 | exceeds NORM_WARN_LEVEL."""


NORM_WARN_LEVEL = 0.5


class lll_params(C.Structure):
    _fields_ = [
        ("J", C.c_double), ("H", C.c_double * 3), ("D", C.c_double), ("e", C.c_double * 3),
        ("D_site", C.c_void_p), ("e_site", C.c_void_p),
        ("lambda_", C.c_double), ("T", C.c_double), ("dt", C.c_double), ("Dt", C.c_double),
        ("precession", C.c_int32), ("integrator", C.c_int32), ("seed", C.c_uint64),
        ("replica", C.c_uint32), ("reserved", C.c_int32),
    ]


class lll_obs(C.Structure):
    _fields_ = [("E_total", C.c_double), ("E_exch", C.c_double), ("E_zeeman", C.c_double),
                ("E_anis", C.c_double), ("m", C.c_double * 3), ("max_norm_dev", C.c_double)]

    def as_dict(self):
        return {"E_total": self.E_total, "E_exch": self.E_exch, "E_zeeman": self.E_zeeman,
                "E_anis": self.E_anis, "m": tuple(self.m), "max_norm_dev": self.max_norm_dev}


class lll_escape_params(C.Structure):
    _fields_ = [
        ("D", C.c_double), ("H", C.c_double), ("lambda_", C.c_double), ("T", C.c_double),
        ("dt", C.c_double), ("Dt", C.c_double), ("precession", C.c_int32),
        ("integrator", C.c_int32), ("seed", C.c_uint64), ("replica", C.c_uint32),
        ("reserved", C.c_int32),
    ]


class lll_replica_desc(C.Structure):
    _fields_ = [
        ("Lx", C.c_int32), ("Ly", C.c_int32), ("Lz", C.c_int32), ("bc", C.c_int32),
        ("J", C.c_double), ("H", C.c_double * 3), ("D", C.c_double), ("e", C.c_double * 3),
        ("lambda_", C.c_double), ("T", C.c_double),
        ("seed", C.c_uint64), ("replica", C.c_uint32), ("init", C.c_int32),
    ]


_lib = None
_P = C.c_void_p


def lib():
    """Loads liblll.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_1610_04914_amd.build")
    L = C.CDLL(LIB_PATH)
    pp = C.POINTER(lll_params)
    L.lll_init_lattice.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.POINTER(C.c_double), C.c_uint64, _P, _P, _P, _P, C.POINTER(_P)]
    L.lll_step_conservative.argtypes = [_P, pp, C.c_int64]
    L.lll_noise_pulse.argtypes = [_P, pp, C.c_uint64]
    L.lll_observables.argtypes = [_P, pp, C.POINTER(lll_obs)]
    L.lll_run.argtypes = [_P, pp, C.c_uint64, C.c_int64, C.POINTER(C.c_double), C.c_int32,
                          C.POINTER(lll_obs)]
    L.lll_get_state.argtypes = [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P)]
    L.lll_kick_norm_dev.argtypes = [_P, C.POINTER(C.c_double), C.c_int32]
    L.lll_accumulators.argtypes = [_P, C.POINTER(C.c_double), C.c_int32]
    L.lll_set_step_config.argtypes = [_P, C.c_int32, C.c_int32]
    L.lll_get_step_config.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lll_set_kick_fusion.argtypes = [_P, C.c_int32]
    L.lll_escape_times.argtypes = [C.POINTER(lll_escape_params), C.c_int64, C.c_int64, _P, _P]
    L.lll_kernel_timing.argtypes = [_P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.lll_step_variant_info.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
    L.lll_autotune.argtypes = [_P, pp, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lll_adjoint.argtypes = [_P, pp, C.c_uint64, C.c_int64, C.c_int32, C.c_double,
                              C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), _P, _P]
    L.lll_adjoint_forward.argtypes = [_P, pp, C.c_uint64, C.c_int64, C.c_int32, C.POINTER(_P)]
    L.lll_adjoint_backward.argtypes = [_P, _P, C.c_double, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), _P, _P]
    L.lll_tape_destroy.argtypes = [_P]
    L.lll_tape_destroy.restype = None
    L.lll_destroy.argtypes = [_P]
    L.lll_destroy.restype = None
    L.lll_batch_create.argtypes = [C.c_int32, C.POINTER(lll_replica_desc), C.c_int32, C.c_double,
                                   C.c_double, C.c_int32, _P, C.POINTER(_P)]
    L.lll_batch_run.argtypes = [_P, C.c_uint64, C.c_int64, C.c_int32, C.POINTER(lll_obs)]
    L.lll_batch_observables.argtypes = [_P, C.POINTER(lll_obs)]
    L.lll_batch_state.argtypes = [_P, C.c_int32, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P)]
    L.lll_batch_accumulators.argtypes = [_P, C.POINTER(C.c_double), C.c_int32]
    L.lll_batch_autotune.argtypes = [_P, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lll_batch_destroy.argtypes = [_P]
    L.lll_batch_destroy.restype = None
    L.lll_philox4x32_10.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_uint32, C.c_uint32,
                                    C.c_uint32, _P, _P]
    L.lll_observables_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                          pp, _P, _P, _P, _P, _P]
    L.lll_last_error.restype = C.c_char_p
    L.lll_version.restype = C.c_char_p
    _lib = L
    return L


def _check(status: int, what: str = "") -> int:
    if status < 0:
        raise LLLError(status, (lib().lll_last_error() or b"").decode() + (f" ({what})" if what else ""))
    if status > 0:
        cat = NormDriftWarning if status == LLL_WARN_NORM else ApplicabilityWarning
        warnings.warn((lib().lll_last_error() or b"").decode(), cat, stacklevel=3)
    return status


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("liblll needs a HIP GPU (torch.cuda.is_available() is False)")
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------- C ABI, same names --
def lll_init_lattice(Lx, Ly, Lz, bc, prec, mode, dir3, seed, sx, sy, sz, stream):
    h = _P()
    d = (C.c_double * 3)(*dir3) if dir3 is not None else None
    _check(lib().lll_init_lattice(Lx, Ly, Lz, bc, prec, mode, d, C.c_uint64(seed), sx, sy, sz,
                                  stream, C.byref(h)), "lll_init_lattice")
    return h


def lll_step_conservative(h, params: lll_params, n_steps: int):
    return _check(lib().lll_step_conservative(h, C.byref(params), int(n_steps)))


def lll_noise_pulse(h, params: lll_params, pulse_index: int):
    return _check(lib().lll_noise_pulse(h, C.byref(params), C.c_uint64(pulse_index)))


def lll_observables(h, params: lll_params) -> dict:
    o = lll_obs()
    _check(lib().lll_observables(h, C.byref(params), C.byref(o)))
    return o.as_dict()


def lll_run(h, params: lll_params, first_pulse: int, n_pulses: int, T_per_pulse=None,
            obs_every: int = 0, trace: bool = True, raw: bool = False):
    """trace=False: the measurements still run (running sums, last values on the
    device) but none is copied back; returns [].  raw=True: the trace as a
    numpy array [measurement][8] of the lll_obs fields in order (E_total,
    E_exch, E_zeeman, E_anis, m_x, m_y, m_z, max_norm_dev; obs_row_dict turns a
    row into the dict form), without building Python dicts."""
    nm = n_pulses // obs_every if obs_every > 0 and trace else 0
    tr = (lll_obs * max(nm, 1))()
    Tp = None
    if T_per_pulse is not None:
        Tp = (C.c_double * n_pulses)(*[float(v) for v in T_per_pulse])
    st = lib().lll_run(h, C.byref(params), C.c_uint64(first_pulse), int(n_pulses), Tp,
                       int(obs_every), tr if nm > 0 else None)
    _check(st, "lll_run")
    if raw:
        import numpy as np
        return np.frombuffer(tr, dtype=np.float64, count=8 * nm).reshape(nm, 8).copy()
    return [tr[i].as_dict() for i in range(nm)]


def obs_row_dict(row) -> dict:
    """The dict form (as lll_obs.as_dict) of one row of a raw trace."""
    return {"E_total": float(row[0]), "E_exch": float(row[1]), "E_zeeman": float(row[2]),
            "E_anis": float(row[3]), "m": (float(row[4]), float(row[5]), float(row[6])),
            "max_norm_dev": float(row[7])}


def lll_observables_noalloc(Lx, Ly, Lz, bc, prec, params: lll_params, sx, sy, sz, out_dev,
                            stream):
    """Observables of a caller-held state into the device array out_dev[8]
    without allocating (no synchronisation; see include/lll.h)."""
    return _check(lib().lll_observables_noalloc(Lx, Ly, Lz, bc, prec, C.byref(params), sx, sy, sz,
                                                out_dev, stream), "lll_observables_noalloc")


def lll_destroy(h):
    lib().lll_destroy(h)


def lll_philox4x32_10(seed: int, i0: int, n: int, c1: int, c2: int, c3: int, out_ptr, stream):
    return _check(lib().lll_philox4x32_10(C.c_uint64(seed), i0, int(n), c1, c2, c3,
                                          C.c_void_p(out_ptr), stream))


def lll_version() -> str:
    return lib().lll_version().decode()


# ------------------------------------------------------------ handles -------
@dataclass
class Params:
    """Parameters of the method (units gamma = mu_0 = k_B = 1)."""
    J: float = 1.0
    H: Sequence[float] = (0.0, 0.0, 0.0)
    D: float = 0.0
    e: Sequence[float] = (0.0, 0.0, 1.0)
    lam: float = 0.01
    T: float = 1.0
    dt: float = 0.1
    Dt: float = 1.0
    precession: bool = True
    integrator: str = "rk4"           # "rk4", "rk2mid" (midpoint) or "rk5b" (Butcher's RK5)
    seed: int = 0
    replica: int = 0                  # Philox counter word 2 of the kicks (batch replica index)
    D_site: Optional[object] = None   # device tensor [N] of the lattice dtype
    e_site: Optional[object] = None   # device tensor [3, N] of the lattice dtype

    def c(self) -> lll_params:
        p = lll_params()
        p.J = float(self.J)
        p.H[:] = [float(v) for v in self.H]
        p.D = float(self.D)
        p.e[:] = [float(v) for v in self.e]
        p.D_site = self.D_site.data_ptr() if self.D_site is not None else None
        p.e_site = self.e_site.data_ptr() if self.e_site is not None else None
        p.lambda_ = float(self.lam)
        p.T = float(self.T)
        p.dt = float(self.dt)
        p.Dt = float(self.Dt)
        p.precession = 1 if self.precession else 0
        p.integrator = _INTEGRATOR[self.integrator]
        p.seed = int(self.seed)
        p.replica = int(self.replica)
        p.reserved = 0
        return p


def check_site_arrays(p: "Params", N: int, dtype) -> None:
    """Raises before any launch unless p's per-site anisotropy arrays are
    device tensors of the lattice dtype, contiguous, with N entries (D_site)
    and 3N entries (e_site, x block then y block then z block), given
    together.  The library reads them through raw device pointers."""
    if (p.D_site is None) != (p.e_site is None):
        raise ValueError("D_site and e_site must be given together")
    for name, t, n in (("D_site", p.D_site, N), ("e_site", p.e_site, 3 * N)):
        if t is None:
            continue
        if not all(hasattr(t, a) for a in ("data_ptr", "is_cuda", "dtype", "is_contiguous")):
            raise TypeError(f"{name} must be a torch tensor")
        if not t.is_cuda:
            raise ValueError(f"{name} must live in device memory")
        if t.dtype != dtype:
            raise ValueError(f"{name} has dtype {t.dtype}; the lattice computes in {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != n:
            raise ValueError(f"{name} has {t.numel()} entries; {n} expected")


_PREC = {"fp64": LLL_FP64, "fp32": LLL_FP32}
_INTEGRATOR = {"rk4": 0, "rk2mid": 1, "rk5b": 2}
_BC = {"periodic": LLL_BC_PERIODIC, "free": LLL_BC_FREE}


class Lattice:
    """A lattice whose spins live in a torch tensor `state` of shape (3, N)
    (component-major, i = x + Lx*(y + Ly*z)) on the current HIP device."""

    def __init__(self, shape, bc: str = "periodic", precision: str = "fp32", init: str = "random",
                 direction=(0.0, 0.0, 1.0), seed: int = 0, state=None):
        torch = _torch()
        self.shape = tuple(int(v) for v in shape)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.precision = precision
        self.bc = bc
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        if state is None:
            state = torch.empty((3, self.N), dtype=self.dtype, device="cuda")
            mode = {"random": LLL_INIT_RANDOM_SPHERE, "direction": LLL_INIT_DIRECTION}[init]
        else:
            if state.dtype != self.dtype or tuple(state.shape) != (3, self.N) or not state.is_cuda:
                raise ValueError("state must be a (3, N) CUDA tensor of the lattice dtype")
            state = state.contiguous()
            mode = LLL_INIT_KEEP
        self.state = state
        ptrs = [C.c_void_p(state[c].data_ptr()) for c in range(3)]
        self.h = lll_init_lattice(*self.shape, _BC[bc], _PREC[precision], mode, direction, seed,
                                  *ptrs, _stream())

    def close(self):
        if getattr(self, "h", None):
            lll_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pc(self, p: Params) -> lll_params:
        check_site_arrays(p, self.N, self.dtype)
        return p.c()

    def step(self, p: Params, n_steps: int = 1):
        return lll_step_conservative(self.h, self._pc(p), n_steps)

    def pulse(self, p: Params, k: int):
        return lll_noise_pulse(self.h, self._pc(p), k)

    def observables(self, p: Params) -> dict:
        return lll_observables(self.h, self._pc(p))

    def run(self, p: Params, first_pulse: int = 0, n_pulses: int = 1, T_per_pulse=None,
            obs_every: int = 0, trace: bool = True, raw: bool = False):
        return lll_run(self.h, self._pc(p), first_pulse, n_pulses, T_per_pulse, obs_every, trace,
                       raw)

    def kick_norm_dev(self, reset: bool = False) -> float:
        v = C.c_double()
        _check(lib().lll_kick_norm_dev(self.h, C.byref(v), 1 if reset else 0))
        return v.value

    def accumulators(self, reset: bool = False):
        a = (C.c_double * 8)()
        _check(lib().lll_accumulators(self.h, a, 1 if reset else 0))
        return list(a)

    def set_step_config(self, variant: int, bz: int = 0):
        _check(lib().lll_set_step_config(self.h, variant, bz))

    def kernel_timing_start(self):
        """Start timing fused-step launches (events recorded by the dispatches)."""
        _check(lib().lll_kernel_timing(self.h, 1, None, None))

    def kernel_timing_stop(self):
        """Synchronise and return (mean kernel ms, launches timed)."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().lll_kernel_timing(self.h, 0, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_kick_fusion(self, fused: bool):
        """Kick as the fused step's epilogue (True) or as its own launch."""
        _check(lib().lll_set_kick_fusion(self.h, 1 if fused else 0))

    def step_config(self):
        v, b = C.c_int32(), C.c_int32()
        _check(lib().lll_get_step_config(self.h, C.byref(v), C.byref(b)))
        return v.value, b.value

    def autotune(self, p: Params, cache_path: Optional[str] = None):
        v, b = C.c_int32(), C.c_int32()
        _check(lib().lll_autotune(self.h, self._pc(p), cache_path.encode() if cache_path else None,
                                  C.byref(v), C.byref(b)))
        return v.value, b.value

    def adjoint(self, p: Params, first_pulse: int, n_pulses: int, ckpt_every: int = 10,
                wE: float = 1.0, wm=(0.0, 0.0, 0.0), want_g_s0: bool = False):
        """Loss L = wE E(s_T) + wm.m(s_T) of lll_run from the current state and
        its gradients w.r.t. H, J, D (per site when p.D_site is set) and s_0."""
        torch = _torch()
        loss = C.c_double()
        gH = (C.c_double * 3)()
        gJ = C.c_double()
        wmc = (C.c_double * 3)(*[float(v) for v in wm])
        if p.D_site is not None:
            gD = torch.zeros(self.N, dtype=torch.float64, device="cuda")
            gDp = C.c_void_p(gD.data_ptr())
        else:
            gDh = C.c_double()
            gD = None
            gDp = C.cast(C.byref(gDh), C.c_void_p)
        gs0 = torch.zeros((3, self.N), dtype=self.dtype, device="cuda") if want_g_s0 else None
        _check(lib().lll_adjoint(self.h, C.byref(self._pc(p)), C.c_uint64(first_pulse), int(n_pulses),
                                 int(ckpt_every), float(wE), wmc, C.byref(loss), gH, C.byref(gJ),
                                 gDp, C.c_void_p(gs0.data_ptr()) if gs0 is not None else None),
               "lll_adjoint")
        return {"loss": loss.value, "g_H": list(gH), "g_J": gJ.value,
                "g_D": gD if gD is not None else gDh.value, "g_s0": gs0}

    def adjoint_forward(self, p: Params, first_pulse: int, n_pulses: int,
                        ckpt_every: int = 10) -> "Tape":
        """Runs n_pulses intervals like run() (the state advances to s_T) and
        records the tape of lll_adjoint_forward for a later backward().
        ckpt_every = TAPE_FULL (0) keeps every step's stage inputs, so the
        backward recomputes nothing."""
        pc = self._pc(p)
        h = _P()
        _check(lib().lll_adjoint_forward(self.h, C.byref(pc), C.c_uint64(first_pulse),
                                         int(n_pulses), int(ckpt_every), C.byref(h)),
               "lll_adjoint_forward")
        return Tape(self, h, p)


TAPE_FULL = 0  # ckpt_every value of a tape that keeps every step's stage inputs


class Tape:
    """Tape of one forward pass (lll_adjoint_forward); backward() may be
    called any number of times.  Keeps the Params it was recorded with (and
    so the per-site tensors the library reads)."""

    def __init__(self, lat: Lattice, h, p: Params):
        self.lat = lat
        self.h = h
        self.p = p

    def backward(self, cot=None, wE: float = 0.0, wm=(0.0, 0.0, 0.0), want_g_s0: bool = True):
        """Gradients of L = <cot, s_T> + wE E(s_T) + wm.m(s_T): cot is an
        optional (3, N) device tensor of the lattice dtype.  Returns a dict
        with loss (the energy terms only), g_H, g_J, g_D (per site when the
        tape has D_site) and g_s0 (a (3, N) tensor, when asked for)."""
        torch = _torch()
        lat = self.lat
        cp = None
        if cot is not None:
            if (not cot.is_cuda or cot.dtype != lat.dtype or tuple(cot.shape) != (3, lat.N)
                    or not cot.is_contiguous()):
                raise ValueError("cot must be a contiguous (3, N) device tensor of the lattice dtype")
            cp = C.c_void_p(cot.data_ptr())
        loss = C.c_double()
        gH = (C.c_double * 3)()
        gJ = C.c_double()
        wmc = (C.c_double * 3)(*[float(v) for v in wm])
        if self.p.D_site is not None:
            gD = torch.zeros(lat.N, dtype=torch.float64, device="cuda")
            gDp = C.c_void_p(gD.data_ptr())
        else:
            gDh = C.c_double()
            gD = None
            gDp = C.cast(C.byref(gDh), C.c_void_p)
        gs0 = torch.zeros((3, lat.N), dtype=lat.dtype, device="cuda") if want_g_s0 else None
        _check(lib().lll_adjoint_backward(self.h, cp, float(wE), wmc, C.byref(loss), gH,
                                          C.byref(gJ), gDp,
                                          C.c_void_p(gs0.data_ptr()) if gs0 is not None else None),
               "lll_adjoint_backward")
        return {"loss": loss.value, "g_H": list(gH), "g_J": gJ.value,
                "g_D": gD if gD is not None else gDh.value, "g_s0": gs0}

    def close(self):
        if getattr(self, "h", None):
            lib().lll_tape_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params_with(base: Params, H, J, D, dtype) -> Params:
    from dataclasses import replace
    p = replace(base, H=tuple(float(v) for v in H.detach().cpu().tolist()),
                J=float(J.detach().cpu()))
    if D.dim() == 0:
        return replace(p, D=float(D.detach().cpu()), D_site=None)
    return replace(p, D_site=D.detach().to(dtype).contiguous())


def _param_grads(r, H, J, D, scale=None):
    torch = _torch()
    gH = torch.tensor(r["g_H"], dtype=H.dtype, device=H.device)
    gJ = torch.tensor(r["g_J"], dtype=J.dtype, device=J.device)
    if D.dim() == 0:
        gD = torch.tensor(r["g_D"], dtype=D.dtype, device=D.device)
    else:
        gD = r["g_D"].to(dtype=D.dtype, device=D.device)
    if scale is not None:
        gH, gJ, gD = gH * scale, gJ * scale, gD * scale
    return gH, gJ, gD


def _autograd_functions():
    torch = _torch()

    class LLLRun(torch.autograd.Function):
        """s_T = n_pulses intervals of the schedule from s_0 on lattice `lat`,
        differentiable in s_0 ((3, N), the lattice dtype), H (3-vector), J
        (scalar) and D (scalar uniform D, or an (N,) tensor of per-site D_i
        with base.e_site).  The forward records a tape (checkpoints every
        ckpt_every operations); the backward hands the incoming gradient of
        s_T to the library's reverse pass as its cotangent."""

        @staticmethod
        def forward(ctx, s0, H, J, D, lat, base, first_pulse, n_pulses, ckpt_every):
            p = _params_with(base, H, J, D, lat.dtype)
            lat.state.copy_(s0.detach())
            ctx.tape = lat.adjoint_forward(p, first_pulse, n_pulses, ckpt_every)
            ctx.save_for_backward(H, J, D)
            return lat.state.clone()

        @staticmethod
        def backward(ctx, g_sT):
            H, J, D = ctx.saved_tensors
            tape = ctx.tape
            r = tape.backward(cot=g_sT.to(tape.lat.dtype).contiguous(), want_g_s0=True)
            gH, gJ, gD = _param_grads(r, H, J, D)
            return (r["g_s0"], gH, gJ, gD, None, None, None, None, None)

    class LLLLoss(torch.autograd.Function):
        """L = wE * E(s_T) + wm . m(s_T) after n_pulses intervals from s_0, the
        lattice's state before the call (the forward advances it to s_T).
        Differentiable in s_0, H, J and D as LLLRun.  The forward records the
        tape; the backward only recomputes and reverses."""

        @staticmethod
        def forward(ctx, s0, H, J, D, lat, base, first_pulse, n_pulses, ckpt_every, wE, wm):
            p = _params_with(base, H, J, D, lat.dtype)
            lat.state.copy_(s0.detach())
            ctx.tape = lat.adjoint_forward(p, first_pulse, n_pulses, ckpt_every)
            o = lat.observables(p)
            val = wE * o["E_total"] + sum(w * m for w, m in zip(wm, o["m"]))
            ctx.w = (float(wE), tuple(float(v) for v in wm))
            ctx.save_for_backward(H, J, D)
            return torch.tensor(val, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            H, J, D = ctx.saved_tensors
            wE, wm = ctx.w
            r = ctx.tape.backward(wE=wE, wm=wm, want_g_s0=True)
            g = float(gout)
            gH, gJ, gD = _param_grads(r, H, J, D, g)
            return (r["g_s0"] * g, gH, gJ, gD, None, None, None, None, None, None, None)

    return LLLRun, LLLLoss


_FUNCS = None


def _funcs():
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _autograd_functions()
    return _FUNCS


def lll_run_diff(s0, H, J, D, lat: "Lattice", base: Params, first_pulse: int, n_pulses: int,
                 ckpt_every: int = 10):
    """Differentiable final state of a pulse-noise run (see LLLRun): any torch
    loss of the returned s_T backpropagates to s0, H, J and D."""
    return _funcs()[0].apply(s0, H, J, D, lat, base, first_pulse, n_pulses, ckpt_every)


def lll_loss(H, J, D, lat: "Lattice", base: Params, first_pulse: int, n_pulses: int,
             ckpt_every: int = 10, wE: float = 1.0, wm=(0.0, 0.0, 1.0), s0=None):
    """Differentiable loss wE E(s_T) + wm.m(s_T) of a pulse-noise run from s0
    (default: the lattice's current state; see LLLLoss)."""
    if s0 is None:
        s0 = lat.state.clone()
    return _funcs()[1].apply(s0, H, J, D, lat, base, first_pulse, n_pulses, ckpt_every, wE, wm)


def step_variant_info(precision: str, variant: int):
    a = (C.c_int32 * 4)()
    _check(lib().lll_step_variant_info(_PREC[precision], variant, a))
    return {"bx": a[0], "by": a[1], "threads": a[2], "lds_bytes": a[3]}


def step_variants(precision: str):
    out = [0]
    v = 1
    while True:
        a = (C.c_int32 * 4)()
        if lib().lll_step_variant_info(_PREC[precision], v, a) != 0:
            break
        out.append(v)
        v += 1
    return out


class Batch:
    """Many independent replicas advanced together (one captured graph per run)."""

    def __init__(self, replicas, precision: str = "fp32", dt: float = 0.1, Dt: float = 1.0,
                 precession: bool = True):
        _torch()
        n = len(replicas)
        arr = (lll_replica_desc * n)()
        self.shapes = []
        for i, r in enumerate(replicas):
            d = arr[i]
            d.Lx, d.Ly, d.Lz = r["L"]
            d.bc = _BC[r.get("bc", "periodic")]
            d.J = float(r.get("J", 1.0))
            d.H[:] = [float(v) for v in r.get("H", (0, 0, 0))]
            d.D = float(r.get("D", 0.0))
            d.e[:] = [float(v) for v in r.get("e", (0, 0, 1))]
            d.lambda_ = float(r["lam"])
            d.T = float(r["T"])
            d.seed = int(r["seed"])
            d.replica = int(r.get("replica", i))
            d.init = LLL_INIT_DIRECTION if r.get("init", "random") == "direction" else LLL_INIT_RANDOM_SPHERE
            self.shapes.append(tuple(r["L"]))
        self.n = n
        self.precision = precision
        h = _P()
        _check(lib().lll_batch_create(n, arr, _PREC[precision], float(dt), float(Dt),
                                      1 if precession else 0, _stream(), C.byref(h)),
               "lll_batch_create")
        self.h = h

    def run(self, first_pulse: int, n_pulses: int, obs_every: int = 0, trace: bool = True,
            raw: bool = False):
        """trace=False: measurements run on the device (running sums) without
        copying a trace back; returns [].  raw=True: the trace as a numpy array
        [measurement][replica][8] of the lll_obs fields in order (E_total,
        E_exch, E_zeeman, E_anis, m_x, m_y, m_z, max_norm_dev), without
        building Python dicts."""
        nm = n_pulses // obs_every if obs_every > 0 and trace else 0
        tr = (lll_obs * max(nm * self.n, 1))()
        _check(lib().lll_batch_run(self.h, C.c_uint64(first_pulse), int(n_pulses), int(obs_every),
                                   tr if nm > 0 else None), "lll_batch_run")
        if raw:
            import numpy as np
            a = np.frombuffer(tr, dtype=np.float64, count=8 * nm * self.n)
            return a.reshape(nm, self.n, 8).copy()
        return [[tr[m * self.n + r].as_dict() for r in range(self.n)] for m in range(nm)]

    def observables(self):
        o = (lll_obs * self.n)()
        _check(lib().lll_batch_observables(self.h, o))
        return [o[r].as_dict() for r in range(self.n)]

    def state(self, r: int):
        """Copy of replica r's state as a (3, N) torch tensor."""
        torch = _torch()
        px, py, pz = _P(), _P(), _P()
        _check(lib().lll_batch_state(self.h, r, C.byref(px), C.byref(py), C.byref(pz)))
        Lx, Ly, Lz = self.shapes[r]
        N = Lx * Ly * Lz
        dt = torch.float64 if self.precision == "fp64" else torch.float32
        es = 8 if self.precision == "fp64" else 4
        out = torch.empty((3, N), dtype=dt, device="cuda")
        torch.cuda.current_stream().synchronize()
        hipMemcpy = _hip_memcpy()
        for c, p in enumerate((px, py, pz)):
            _hip_check(hipMemcpy(C.c_void_p(out[c].data_ptr()), p, C.c_size_t(N * es), 3))
        return out

    def autotune(self, cache_path: Optional[str] = None):
        v, b = C.c_int32(), C.c_int32()
        _check(lib().lll_batch_autotune(self.h, cache_path.encode() if cache_path else None,
                                        C.byref(v), C.byref(b)))
        return v.value, b.value

    def accumulators(self, reset: bool = False):
        a = (C.c_double * (8 * self.n))()
        _check(lib().lll_batch_accumulators(self.h, a, 1 if reset else 0))
        return [list(a[8 * r: 8 * r + 8]) for r in range(self.n)]

    def close(self):
        if getattr(self, "h", None):
            lib().lll_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _hip_memcpy():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip.hipMemcpy


def _hip_check(rc: int):
    if rc != 0:
        raise LLLError(LLL_EDEVICE, f"hipMemcpy failed with {rc}")


def escape_times(D: float, H: float, lam: float, T: float, dt: float, Dt: float, n_runs: int,
                 seed: int = 0, replica: int = 0, max_pulses: int = 10**6,
                 integrator: str = "rk4", precession: bool = True):
    """First-passage times of n_runs spins of the escape problem (Sec. III.B)
    as a float64 CUDA tensor; -1 marks runs that did not escape within
    max_pulses intervals (lll_escape_times)."""
    torch = _torch()
    p = lll_escape_params()
    p.D, p.H, p.lambda_, p.T, p.dt, p.Dt = map(float, (D, H, lam, T, dt, Dt))
    p.precession = 1 if precession else 0
    p.integrator = _INTEGRATOR[integrator]
    p.seed = int(seed)
    p.replica = int(replica)
    p.reserved = 0
    out = torch.empty(int(n_runs), dtype=torch.float64, device="cuda")
    _check(lib().lll_escape_times(C.byref(p), int(n_runs), int(max_pulses),
                                  C.c_void_p(out.data_ptr()) if n_runs > 0 else None, _stream()),
           "lll_escape_times")
    return out
