"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/lll.h, its structs have the layout the
Python binding marshals, and argument validation that happens before any
device call returns the documented status codes."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lll.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lll_status|void|const char\s*\*)\s*(lll_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def P():
    import paper_1610_04914_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("liblll.so is not built (run __graft_entry__.build())")
    P.lib()
    return P


def test_header_declares_the_boundary():
    names = declared_functions()
    for req in ("lll_init_lattice", "lll_step_conservative", "lll_noise_pulse", "lll_observables",
                "lll_run", "lll_destroy", "lll_last_error", "lll_batch_create", "lll_batch_run",
                "lll_adjoint", "lll_autotune", "lll_philox4x32_10"):
        assert req in names


def test_library_exports_every_declared_symbol(P):
    L = P.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(ln.split()[-1] for ln in out.splitlines() if ln.strip())
    assert set(declared_functions()) <= exported


def test_struct_layout_matches_binding(P):
    """sizeof/offsetof of the public structs as gcc sees include/lll.h equal
    what the ctypes binding uses."""
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "lll.h"
#define F(T, m) printf("%s.%s %zu\n", #T, #m, offsetof(T, m));
int main(void) {
  printf("lll_params %zu\nlll_obs %zu\nlll_replica_desc %zu\n", sizeof(lll_params), sizeof(lll_obs),
         sizeof(lll_replica_desc));
  F(lll_params, D_site) F(lll_params, lambda) F(lll_params, precession) F(lll_params, seed)
  F(lll_params, replica)
  F(lll_obs, m) F(lll_obs, max_norm_dev)
  F(lll_replica_desc, lambda) F(lll_replica_desc, seed) F(lll_replica_desc, replica)
  F(lll_replica_desc, init)
  printf("lll_escape_params %zu\n", sizeof(lll_escape_params));
  F(lll_escape_params, precession) F(lll_escape_params, seed) F(lll_escape_params, replica)
  return 0;
}
"""
    d = tempfile.mkdtemp()
    cfile = os.path.join(d, "layout.c")
    exe = os.path.join(d, "layout")
    open(cfile, "w").write(src)
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), "-o", exe, cfile])
    lines = dict(ln.rsplit(" ", 1) for ln in subprocess.check_output([exe], text=True).splitlines())
    lay = {k: int(v) for k, v in lines.items()}
    assert lay["lll_params"] == C.sizeof(P.lll_params)
    assert lay["lll_obs"] == C.sizeof(P.lll_obs)
    assert lay["lll_replica_desc"] == C.sizeof(P.lll_replica_desc)
    assert lay["lll_params.D_site"] == P.lll_params.D_site.offset
    assert lay["lll_params.lambda"] == P.lll_params.lambda_.offset
    assert lay["lll_params.replica"] == P.lll_params.replica.offset
    assert lay["lll_params.precession"] == P.lll_params.precession.offset
    assert lay["lll_params.seed"] == P.lll_params.seed.offset
    assert lay["lll_obs.m"] == P.lll_obs.m.offset
    assert lay["lll_obs.max_norm_dev"] == P.lll_obs.max_norm_dev.offset
    assert lay["lll_replica_desc.lambda"] == P.lll_replica_desc.lambda_.offset
    assert lay["lll_replica_desc.seed"] == P.lll_replica_desc.seed.offset
    assert lay["lll_replica_desc.replica"] == P.lll_replica_desc.replica.offset
    assert lay["lll_replica_desc.init"] == P.lll_replica_desc.init.offset
    assert lay["lll_escape_params"] == C.sizeof(P.lll_escape_params)
    for f in ("precession", "seed", "replica"):
        assert lay["lll_escape_params." + f] == getattr(P.lll_escape_params, f).offset


def test_validation_before_device_use(P):
    L = P.lib()
    h = C.c_void_p()
    st = L.lll_init_lattice(0, 4, 4, 0, 1, 0, None, 0, None, None, None, None, C.byref(h))
    assert st == P.LLL_EINVAL and b"sizes" in L.lll_last_error()
    st = L.lll_init_lattice(4, 4, 4, 7, 1, 0, None, 0, None, None, None, None, C.byref(h))
    assert st == P.LLL_EINVAL
    st = L.lll_init_lattice(4, 4, 4, 0, 9, 0, None, 0, None, None, None, None, C.byref(h))
    assert st == P.LLL_EINVAL
    # more than 2^31 - 1 sites, including products that overflow 64 bits
    for shape in ((2048, 2048, 512), (46341, 46341, 1), (2**31 - 1, 2, 1),
                  (2**21, 2**21, 2**21), (2**31 - 1, 2**31 - 1, 2**31 - 1)):
        st = L.lll_init_lattice(*shape, 0, 1, 0, None, 0, None, None, None, None, C.byref(h))
        assert st == P.LLL_EINVAL and b"2^31-1" in L.lll_last_error()
    st = L.lll_init_lattice(4, 4, 4, 0, 1, 0, None, 0, C.c_void_p(16), None, None, None, C.byref(h))
    assert st == P.LLL_EINVAL and b"all three" in L.lll_last_error()
    st = L.lll_init_lattice(4, 4, 4, 0, 1, P.LLL_INIT_KEEP, None, 0, None, None, None, None, C.byref(h))
    assert st == P.LLL_EINVAL
    st = L.lll_init_lattice(4, 4, 4, 0, 1, P.LLL_INIT_DIRECTION, None, 0, None, None, None, None,
                            C.byref(h))
    assert st == P.LLL_EINVAL
    assert L.lll_init_lattice(4, 4, 4, 0, 1, 0, None, 0, None, None, None, None, None) == P.LLL_EINVAL
    assert L.lll_step_conservative(None, None, 1) == P.LLL_EINVAL
    assert L.lll_run(None, None, 0, 1, None, 0, None) == P.LLL_EINVAL
    assert L.lll_philox4x32_10(0, 0, -1, 0, 0, 0, None, None) == P.LLL_EINVAL
    assert L.lll_philox4x32_10(0, 0, 0, 0, 0, 0, None, None) == P.LLL_OK
    assert L.lll_batch_create(0, None, 1, 0.1, 1.0, 1, None, C.byref(h)) == P.LLL_EINVAL
    desc = (P.lll_replica_desc * 1)()
    desc[0].Lx = desc[0].Ly = desc[0].Lz = 4
    desc[0].lambda_ = 0.01
    desc[0].T = 1.0
    assert L.lll_batch_create(1, desc, 1, 0.3, 1.0, 1, None, C.byref(h)) == P.LLL_EINVAL
    assert b"not a positive integer" in L.lll_last_error()
    big = (P.lll_replica_desc * 2)()
    for d in big:
        d.Lx = d.Ly = d.Lz = 2**21  # 2^63 sites each
        d.lambda_ = 0.01
        d.T = 1.0
    big[0].Lx = big[0].Ly = big[0].Lz = 4
    assert L.lll_batch_create(2, big, 1, 0.1, 1.0, 1, None, C.byref(h)) == P.LLL_EINVAL
    assert b"replica 1" in L.lll_last_error()
    for d in big:
        d.Lx, d.Ly, d.Lz = 1024, 1024, 1024  # 2^30 each, 2^31 in all
    assert L.lll_batch_create(2, big, 1, 0.1, 1.0, 1, None, C.byref(h)) == P.LLL_EINVAL
    assert b"too many sites" in L.lll_last_error()



def test_null_handles_rejected(P):
    """Every entry point that takes a lattice, batch or tape handle returns
    LLL_EINVAL with a message for a NULL handle, before any device call; the
    destroy calls accept NULL."""
    L = P.lib()
    o = P.lll_obs()
    d = (C.c_double * 8)()
    i1, i2 = C.c_int32(), C.c_int32()
    v = C.c_void_p()
    i64 = C.c_int64()
    wm = (C.c_double * 3)()
    calls = {
        "lll_noise_pulse": lambda: L.lll_noise_pulse(None, None, 0),
        "lll_observables": lambda: L.lll_observables(None, None, C.byref(o)),
        "lll_get_state": lambda: L.lll_get_state(None, C.byref(v), C.byref(v), C.byref(v)),
        "lll_kick_norm_dev": lambda: L.lll_kick_norm_dev(None, d, 0),
        "lll_accumulators": lambda: L.lll_accumulators(None, d, 0),
        "lll_set_step_config": lambda: L.lll_set_step_config(None, 1, 0),
        "lll_get_step_config": lambda: L.lll_get_step_config(None, C.byref(i1), C.byref(i2)),
        "lll_set_kick_fusion": lambda: L.lll_set_kick_fusion(None, 1),
        "lll_kernel_timing": lambda: L.lll_kernel_timing(None, 1, d, C.byref(i64)),
        "lll_autotune": lambda: L.lll_autotune(None, None, None, C.byref(i1), C.byref(i2)),
        "lll_adjoint_forward": lambda: L.lll_adjoint_forward(None, None, 0, 1, 10, C.byref(v)),
        "lll_adjoint_backward": lambda: L.lll_adjoint_backward(None, None, 1.0, wm, d, d, d,
                                                               d, None),
        "lll_batch_run": lambda: L.lll_batch_run(None, 0, 1, 0, None),
        "lll_batch_observables": lambda: L.lll_batch_observables(None, C.byref(o)),
        "lll_batch_state": lambda: L.lll_batch_state(None, 0, C.byref(v), C.byref(v), C.byref(v)),
        "lll_batch_accumulators": lambda: L.lll_batch_accumulators(None, d, 0),
        "lll_batch_autotune": lambda: L.lll_batch_autotune(None, None, C.byref(i1), C.byref(i2)),
        "lll_escape_times": lambda: L.lll_escape_times(None, 1, 1, None, None),
    }
    for name, call in calls.items():
        assert call() == P.LLL_EINVAL, name
        assert L.lll_last_error(), name
    L.lll_destroy(None)
    L.lll_batch_destroy(None)
    L.lll_tape_destroy(None)



def test_raw_trace_rows_follow_the_record_layout(P):
    """A raw trace row (numpy view of the lll_obs records) converts to the same
    dict as the record itself."""
    import numpy as np
    recs = (P.lll_obs * 2)()
    for k, r in enumerate(recs):
        r.E_total, r.E_exch, r.E_zeeman, r.E_anis = 1.0 + k, 2.0 + k, 3.0 + k, 4.0 + k
        r.m[0], r.m[1], r.m[2] = 5.0 + k, 6.0 + k, 7.0 + k
        r.max_norm_dev = 8.0 + k
    rows = np.frombuffer(recs, dtype=np.float64, count=16).reshape(2, 8)
    for k in range(2):
        assert P.obs_row_dict(rows[k]) == recs[k].as_dict()


def test_variant_table(P):
    for prec in ("fp32", "fp64"):
        vs = P.step_variants(prec)
        assert vs[0] == 0 and len(vs) >= 3
        for v in vs[1:]:
            info = P.step_variant_info(prec, v)
            es = 8 if prec == "fp64" else 4
            bx, by = info["bx"], info["by"]
            r = sum(((bx + 2 * q) | 1) * (by + 2 * q) for q in range(1, 5))
            assert info["lds_bytes"] == 6 * es * r
            assert info["lds_bytes"] <= 160 * 1024
            assert info["threads"] % 64 == 0 and info["threads"] <= 1024


def test_binding_fails_loudly_without_gpu(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        P.Lattice((4, 4, 4))


def test_binding_fails_loudly_without_the_library(tmp_path):
    """No CPU fallback: with liblll.so absent every entry point raises."""
    import subprocess
    import sys
    code = (
        "import paper_1610_04914_amd as P\n"
        f"P.LIB_PATH = {str(tmp_path / 'missing.so')!r}\n"
        "for f in (P.lib, lambda: P.Lattice((8, 8, 8)), lambda: P.step_variants('fp32')):\n"
        "    try:\n"
        "        f()\n"
        "    except (ImportError, RuntimeError):\n"
        "        continue\n"
        "    raise SystemExit('did not raise')\n"
        "print('ok')\n")
    root = __import__("os").path.dirname(__import__("os").path.dirname(__file__))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_status_codes_and_constants_match_header(P):
    """Every lll_status value and the norm-warning threshold as the binding
    spells them are the header's."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    enum = re.search(r"typedef enum \{(.*?)\} lll_status;", txt, re.S).group(1)
    vals = dict((k, int(v)) for k, v in re.findall(r"(LLL_\w+)\s*=\s*(-?\d+)", enum))
    assert len(vals) >= 8
    for k, v in vals.items():
        assert getattr(P, k) == v, k
    lvl = float(re.search(r"#define LLL_NORM_WARN_LEVEL\s+([0-9.eE+-]+)", txt).group(1))
    assert P.NORM_WARN_LEVEL == lvl
    full = int(re.search(r"#define LLL_TAPE_FULL\s+(\d+)", txt).group(1))
    assert P.TAPE_FULL == full


def test_site_arrays_rejected_before_any_launch():
    """Per-site anisotropy arrays reach the kernels as raw device pointers, so
    the binding refuses host tensors, a dtype other than the lattice's,
    non-contiguous views, wrong sizes and a lone D_site before any call."""
    import torch

    import paper_1610_04914_amd as P
    N = 24
    ok = dict(dtype=torch.float32)
    D = torch.ones(N, **ok)
    e = torch.zeros(3 * N, **ok)
    with pytest.raises(ValueError, match="device memory"):
        P.check_site_arrays(P.Params(D_site=D, e_site=e), N, torch.float32)
    with pytest.raises(ValueError, match="together"):
        P.check_site_arrays(P.Params(D_site=D), N, torch.float32)
    with pytest.raises(TypeError):
        P.check_site_arrays(P.Params(D_site=[1.0] * N, e_site=[0.0] * 3 * N), N, torch.float32)

    class FakeDev:
        """Quacks like a device tensor so the remaining checks are reached on a
        host without a GPU."""
        def __init__(self, t, contiguous=True):
            self.t, self.c = t, contiguous
            self.is_cuda = True
            self.dtype = t.dtype

        def data_ptr(self):
            return self.t.data_ptr()

        def is_contiguous(self):
            return self.c

        def numel(self):
            return self.t.numel()

    P.check_site_arrays(P.Params(D_site=FakeDev(D), e_site=FakeDev(e)), N, torch.float32)
    with pytest.raises(ValueError, match="dtype"):
        P.check_site_arrays(P.Params(D_site=FakeDev(D), e_site=FakeDev(e)), N, torch.float64)
    with pytest.raises(ValueError, match="contiguous"):
        P.check_site_arrays(P.Params(D_site=FakeDev(D, False), e_site=FakeDev(e)), N,
                            torch.float32)
    with pytest.raises(ValueError, match="entries"):
        P.check_site_arrays(P.Params(D_site=FakeDev(D), e_site=FakeDev(e[:N])), N, torch.float32)
    with pytest.raises(ValueError, match="entries"):
        P.check_site_arrays(P.Params(D_site=FakeDev(D[:5]), e_site=FakeDev(e)), N, torch.float32)
