"""Benchmark of the pulse-noise LLL hot path on one MI355X.

Workload (headline): 128^3 simple-cubic lattice, periodic boundaries, J = 1,
H = (0, 0, 0.1), uniaxial D = 0.05 along z, lambda = 0.01, T = 1.0, RK4 with
dt = 0.2, pulses every Dt = 2.0 (n = 10 steps per interval), fp32 state with
fp64 reductions, random-sphere initial state from seed 0, observables measured
after every interval.  One benchmark "step" is one interval of the schedule
(n1 = 5 RK4 steps, kick, n2 = 5 RK4 steps, fp64 observables); the default
timed region is the workload's full 2000 pulses (20000 RK4 steps).

Metric: spin-steps/s = sites x RK4 steps / s (kicks and reductions are inside
the timed region but are not counted as steps).  The JSON line also carries the
roofline of the dominant kernel (the fused RK4 step: VALU-bound, with its HBM
fraction alongside), the batched and adjoint ratios and the 256^3 overdamped
run ("extras", skipped with --no-extras), and the FP64 oracle timed on a
bounded sample on the host ("cpu_baseline").

Prints ONE JSON line.  --gpus above 1 is rejected: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SHAPE = (128, 128, 128)
PHYS = dict(J=1.0, H=(0.0, 0.0, 0.1), D=0.05, e=(0.0, 0.0, 1.0), lam=0.01, T=1.0, dt=0.2, Dt=2.0,
            precession=True, seed=0)
HBM_PEAK_GBS = 8000.0
BYTES_PER_SPIN_STEP = {"fp32": 24, "fp64": 48}
# Arithmetic per spin and RK4 step (precessional equation, uniaxial z
# anisotropy), counted per stage: neighbour sum 15, h = cJ n + cH 6, anisotropy
# 2, s x h 9, h - lam (s x h) 6, s x (...) 9, next stage input 6, accumulator 6.
FLOPS_PER_SPIN_STEP = 4 * 59
# Vector ALU peak for the instruction forms this library issues: 256 CUs x 4 SIMDs
# x 16 lanes x 2 flop (FMA) x 2.4 GHz.  The same for fp32 and fp64, because packed
# fp32 (which doubles the fp32 rate to 157.3 TFLOP/s) is disabled in the build.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
METRIC = "spin-steps/s (RK4, 128^3 sc, fp32) + % HBM roofline; batched & adjoint ratios"
TUNE_CACHE = os.path.join(ROOT, "paper_1610_04914_amd", "tune_cache.txt")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rk4_fused_128c_fp32_traffic.md")
TRAFFIC_FILE_256 = os.path.join(ROOT, "profiles", "rk4_fused_256c_fp32_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1610_04914_amd", "csrc", f)
                  for f in ("kern_fused.hpp", "lll_device.hpp")]


def kernel_hash() -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def configure_lattice(lat, prec: str, shape, p=None) -> tuple:
    """Step configuration used by the benchmark: the committed tuning table
    entry for this lattice (and physics p, default the headline's) when there is
    one, else an autotune run."""
    import paper_1610_04914_amd as P
    if p is None:
        p = P.Params(**PHYS)
    return lat.autotune(p, cache_path=TUNE_CACHE)


def measured_traffic(path: str = None):
    """Bytes per launch of the fused step between L2 and the memory fabric
    (calibrated FETCH_SIZE + WRITE_SIZE) from a committed rocprofv3 counter
    summary, or None when it is missing or was taken on other kernel sources.
    At 128^3 the reads include what the 256 MB Infinity Cache serves; at 256^3
    (two 201 MB state copies) they are close to HBM traffic."""
    path = path or TRAFFIC_FILE
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    mh = re.search(r"kernel_sources_hash:\s*(\w+)", txt)
    mb = re.search(r"l2_fabric_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not mh or not mb or mh.group(1) != kernel_hash():
        return None
    return float(mb.group(1))


def cpu_baseline(steps: int = 10, steps_all_cores: int = 40):
    """The FP64 oracle on a bounded sample of the same workload (RK4 steps of
    the 128^3 lattice): its OpenMP build on every core this process may use
    (the reported value), and the single-threaded build the tests use."""
    import numpy as np
    import oracle as orc
    g = orc.geom(SHAPE)
    p = orc.Params(J=PHYS["J"], H=PHYS["H"], D=PHYS["D"], e=PHYS["e"], lam=PHYS["lam"], T=PHYS["T"],
                   dt=PHYS["dt"], Dt=PHYS["Dt"], precession=True)
    s = orc.init_random_sphere(g, 0)
    N = int(np.prod(SHAPE))
    host = host_info()
    # the OpenMP runtime reads this when it starts; a value already set is kept
    os.environ.setdefault("OMP_NUM_THREADS", str(host["affinity_cores"] or 1))
    cores = orc.threads(all_cores=True)
    orc.step(g, p, s, 1)  # warm-up (page in)
    t0 = time.perf_counter()
    orc.step(g, p, s, steps)
    el1 = time.perf_counter() - t0
    orc.step(g, p, s, 1, all_cores=True)
    t0 = time.perf_counter()
    orc.step(g, p, s, steps_all_cores, all_cores=True)
    eln = time.perf_counter() - t0
    return {"value": N * steps_all_cores / eln, "unit": "spin-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps_all_cores} RK4 steps of the 128^3 fp64 lattice ({eln:.1f} s, "
                      f"OpenMP build on {cores} host threads)",
            "single_thread": {"value": N * steps / el1, "cores": 1,
                              "sample": f"{steps} RK4 steps ({el1:.1f} s, one host thread)"},
            "host": host}


def host_info() -> dict:
    """CPU model and the number of cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count()
    return {"cpu_model": model, "affinity_cores": n}


def _prepare_timing(lat):
    """Creates the library's dispatch events for kernel timing ahead of time:
    made inside a timed stretch they would leave the GPU idle long enough for
    its clock to drop (measured: a 10 ms pause cost 15% of the next 6 ms)."""
    lat.kernel_timing_start()
    lat.kernel_timing_stop()


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


# Pulses of the batched accuracy runs (--acc-pulses).  Near T_c the |m| series
# stay correlated over thousands of pulses: with 5000 the blocking analysis
# converged for 4 of 96 replicas and the error bars were lower bounds; 20000
# (about 100 s for both batches) gives converged errors for a quarter of them.
ACC_PULSES = 20000


def extra_batched(n_pulses: int = 500, n_seq: int = 100, n_acc: int = 0, burn: int = 1000):
    """Uneven-replica workload: 32 each of 24^3, 48^3, 64^3, T uniform in
    [0.3, 2], lambda log-uniform in [0.005, 0.05], J = 1, H = 0, dt = 0.1,
    Dt = 1.0, random-sphere starts, per-replica noise keys.

    Throughput (random starts): the fp32 batch over n_pulses, and the plain
    fp64 single-lattice path on the same replicas one after another over n_seq
    pulses (each lattice keyed with its replica's seed and index, so it draws
    the same noise as the batch).  The batch captures its schedule as a graph
    on the first call of a given length and measurement spacing and replays it
    for any first pulse (a long run in equal chunks); the timed call is such a
    replay, and the first call of that length, capture included, is reported
    beside it.  Both paths measure every interval on the device (observables
    and running sums) without copying a per-interval trace to Python, whose
    conversion alone would take 0.08 s of a 0.9 s batch call.

    Accuracy: fp32 and fp64 batches from the same start and noise over n_acc
    pulses; per replica, the time averages of E/N and |m| after `burn` pulses
    are compared against their combined standard errors (from each series'
    integrated autocorrelation time); the signed mean of the differences over
    replicas shows any fp32 bias.  The fp64 batch follows the fp64
    single-lattice path's trajectory (same keys, same arithmetic).  The
    accuracy runs start ordered along +z so that the series are stationary
    after the burn-in."""
    import numpy as np
    import paper_1610_04914_amd as P
    from tests import inputs
    n_acc = n_acc or ACC_PULSES
    reps = inputs.batch_replicas(seed=0)
    descs = [dict(r, J=1.0) for r in reps]
    sites = sum(int(np.prod(r["L"])) for r in reps)
    B = P.Batch(descs, precision="fp32", dt=0.1, Dt=1.0)
    B.autotune(cache_path=TUNE_CACHE)
    el_first, _ = _timed(lambda: B.run(first_pulse=10**6, n_pulses=n_pulses, obs_every=1,
                                       trace=False))
    el_b, _ = _timed(lambda: B.run(first_pulse=10, n_pulses=n_pulses, obs_every=1, trace=False))
    B.close()

    B0 = P.Batch(descs, precision="fp64", dt=0.1, Dt=1.0)
    lats = []
    for i, r in enumerate(reps):
        lat = P.Lattice(r["L"], precision="fp64", state=B0.state(i))
        lats.append((lat, P.Params(J=1.0, lam=r["lam"], T=r["T"], dt=0.1, Dt=1.0, seed=r["seed"],
                                   replica=r["replica"])))
    B0.close()
    for lat, p in lats:
        lat.run(p, first_pulse=0, n_pulses=2)

    def run_seq():
        return [lat.run(p, first_pulse=2, n_pulses=n_seq, obs_every=1, trace=False)
                for lat, p in lats]
    el_s, _ = _timed(run_seq)
    for lat, _ in lats:
        lat.close()

    def series(prec):
        # ordered starts (+z): below T_c a random start keeps coarsening far
        # beyond the run, so time averages would not be stationary
        A = P.Batch([dict(d, init="direction") for d in descs], precision=prec, dt=0.1, Dt=1.0)
        tr = A.run(first_pulse=0, n_pulses=n_acc, obs_every=1, raw=True)  # [m][r][8]
        A.close()
        e = tr[:, :, 0].T
        mag = np.linalg.norm(tr[:, :, 4:7], axis=2).T
        N = np.array([float(np.prod(r["L"])) for r in reps])
        return e / N[:, None], mag

    def mean_sem(x):
        """Mean after burn-in and its standard error by blocking (Flyvbjerg and
        Petersen, J. Chem. Phys. 91, 461 (1989)): the series is averaged in
        blocks of 1, 2, 4, ... samples, the naive error of the block means is
        taken at each level, and the largest over the levels that keep at
        least 16 blocks is used (the plateau, or its conservative side when
        the correlation time is not much shorter than the run)."""
        x = x[:, burn:]
        means, sems = x.mean(1), np.zeros(x.shape[0])
        conv = np.zeros(x.shape[0], dtype=bool)
        for r in range(x.shape[0]):
            b = x[r].copy()
            errs = []
            while b.size >= 16:
                errs.append((float(np.std(b, ddof=1) / np.sqrt(b.size)), b.size))
                m = b.size // 2
                b = 0.5 * (b[:2 * m:2] + b[1:2 * m:2])
            sems[r] = max(e for e, _ in errs)
            # plateau: the last two levels agree within the statistical error
            # of the last one, e / sqrt(2 (n_blocks - 1))
            (e1, _), (e2, n2) = errs[-2], errs[-1]
            conv[r] = abs(e2 - e1) <= e2 / np.sqrt(2 * (n2 - 1)) or sems[r] == 0.0
        return means, sems, conv

    e32, m32 = series("fp32")
    e64, m64 = series("fp64")
    zs, cv = {}, {}
    for name, a, b in (("E_per_site", e32, e64), ("abs_m", m32, m64)):
        ma, sa, ca = mean_sem(a)
        mb, sb, cb = mean_sem(b)
        zs[name] = (ma - mb) / np.sqrt(sa**2 + sb**2 + 1e-300)
        cv[name] = ca & cb
    # For independent normal z, P(|z| < 2) = 0.9545: 96 replicas give 91.6
    # within 2 sigma with a binomial standard deviation of 2.0.
    nrep = len(reps)
    hotT = np.array([r["T"] > 1.0 for r in reps])
    expect2 = 0.9545 * nrep
    sd2 = math.sqrt(nrep * 0.9545 * 0.0455)
    rate_b = sites * 10 * n_pulses / el_b
    rate_s = sites * 10 * n_seq / el_s
    return {"workload": "96 replicas (32 x 24^3, 48^3, 64^3), fp32 batch vs fp64 single-lattice path",
            "batched_fp32_spin_steps_per_s": rate_b,
            "batched_fp32_first_call_spin_steps_per_s": sites * 10 * n_pulses / el_first,
            "batched_alg_hbm_frac": rate_b * BYTES_PER_SPIN_STEP["fp32"] / (HBM_PEAK_GBS * 1e9),
            "sequential_fp64_spin_steps_per_s": rate_s,
            "speedup": rate_b / rate_s,
            "pulses_timed": {"batch": n_pulses, "sequential": n_seq},
            "accuracy": {"pulses": n_acc, "burn_in": burn, "replicas": nrep,
                         "error_bars": "blocking analysis, largest block error with >= 16 blocks",
                         "expected_within_2sigma": [expect2, sd2],
                         **{k: {"within_2sigma": int(np.sum(np.abs(z) < 2.0)),
                                "within_3sigma": int(np.sum(np.abs(z) < 3.0)),
                                "mean_signed_z": float(z.mean()),
                                "max_abs_z": float(np.abs(z).max()),
                                "blocking_converged": int(cv[k].sum()),
                                "converged_within_2sigma": int(np.sum(np.abs(z[cv[k]]) < 2.0)),
                                "converged_expected_within_2sigma": [
                                    0.9545 * int(cv[k].sum()),
                                    math.sqrt(int(cv[k].sum()) * 0.9545 * 0.0455)],
                                # sign test (no error bars needed): under no fp32
                                # bias the count of positive z is Binomial(n, 1/2)
                                "positive_z": int(np.sum(z > 0)),
                                "positive_z_T_above_1": int(np.sum(z[hotT] > 0)),
                                "replicas_T_above_1": int(hotT.sum()),
                                "sign_test_p": _binom_two_sided(int(np.sum(z > 0)), nrep),
                                "sign_test_p_T_above_1": _binom_two_sided(
                                    int(np.sum(z[hotT] > 0)), int(hotT.sum()))}
                            for k, z in zs.items()},
                         "per_replica_T_lambda_zE_zm_converged": [
                             [float(r["T"]), float(r["lam"]), float(zs["E_per_site"][i]),
                              float(zs["abs_m"][i]), int(cv["E_per_site"][i]),
                              int(cv["abs_m"][i])] for i, r in enumerate(reps)]}}


def _binom_two_sided(k: int, n: int) -> float:
    """Two-sided exact binomial p-value of k successes in n trials at p = 1/2."""
    if n == 0:
        return 1.0
    pk = [math.comb(n, j) / 2.0**n for j in range(n + 1)]
    return float(min(1.0, sum(q for q in pk if q <= pk[k] * (1 + 1e-12))))


def extra_adjoint():
    """Adjoint workload (32^3, per-site anisotropy, 3 intervals of 100 steps):
    (forward with checkpoints + backward with recompute) / plain forward, and
    the same with a full tape (the forward keeps every step's stage inputs,
    4 states per step, and the backward recomputes nothing)."""
    import numpy as np
    import torch
    import paper_1610_04914_amd as P
    from tests import inputs
    N = 32**3
    D, e = inputs.site_anisotropy(N, 4)
    out = {}
    for prec in ("fp64", "fp32"):
        dt_ = torch.float64 if prec == "fp64" else torch.float32
        Dt_ = torch.tensor(D, dtype=dt_, device="cuda")
        et = torch.tensor(e, dtype=dt_, device="cuda")
        p = P.Params(J=1.0, H=(0, 0, 0.2), lam=0.01, T=0.5, dt=0.1, Dt=10.0, D_site=Dt_, e_site=et,
                     seed=0)
        lat = P.Lattice((32, 32, 32), precision=prec, init="direction", direction=(0, 0, 1))
        variant, bz = lat.autotune(p, cache_path=TUNE_CACHE)
        s0 = lat.state.clone()
        lat.run(p, 0, 3)
        lat.state.copy_(s0)
        el_f, _ = _timed(lambda: (lat.run(p, 0, 3), lat.observables(p)))
        lat.state.copy_(s0)
        lat.adjoint(p, 0, 3, ckpt_every=10, wE=1.0, wm=(0, 0, 1))
        el_a, _ = _timed(lambda: lat.adjoint(p, 0, 3, ckpt_every=10, wE=1.0, wm=(0, 0, 1)))
        lat.adjoint(p, 0, 3, ckpt_every=P.TAPE_FULL, wE=1.0, wm=(0, 0, 1))
        el_t, _ = _timed(lambda: lat.adjoint(p, 0, 3, ckpt_every=P.TAPE_FULL, wE=1.0,
                                             wm=(0, 0, 1)))
        nops = 3 * (100 + 1)
        out[prec] = {"forward_s": el_f, "adjoint_s": el_a, "ratio": el_a / el_f,
                     "full_tape_adjoint_s": el_t, "full_tape_ratio": el_t / el_f,
                     "full_tape_bytes": 3 * N * lat.state.element_size() * (4 * nops + 1),
                     "step_variant": variant, "bz": bz}
        lat.close()
    return out


def extra_overdamped(n_pulses: int = 5000):
    """256^3, fp32, slow equation, J = 1, D = 0.02 z, lambda = 0.1, dt = Dt = 0.4
    (pulse every step), T ramp 2.0 -> 0.5."""
    import numpy as np
    import paper_1610_04914_amd as P
    lat = P.Lattice((256, 256, 256), precision="fp32", init="random", seed=0)
    p = P.Params(J=1.0, D=0.02, e=(0, 0, 1), lam=0.1, T=2.0, dt=0.4, Dt=0.4,
                 precession=False, seed=0)
    lat.autotune(p, cache_path=TUNE_CACHE)
    Ts = list(2.0 - 1.5 * np.arange(n_pulses) / (n_pulses - 1))
    lat.run(p, 0, 10, T_per_pulse=Ts[:10])
    el, tr = _timed(lambda: lat.run(p, 0, n_pulses, T_per_pulse=Ts, obs_every=100))
    N = lat.N
    lat.close()
    return {"workload": "256^3 fp32 slow equation, T ramp 2.0->0.5", "pulses": n_pulses,
            "spin_steps_per_s": N * n_pulses / el,
            "hbm_frac_alg": N * n_pulses * 24 / el / (HBM_PEAK_GBS * 1e9),
            "final_abs_m": float(np.linalg.norm(tr[-1]["m"]))}


def extra_max_lattice(n_pulses: int = 10):
    """The largest lattice the library accepts, 1024 x 1024 x 2047 (2.15e9
    sites, 25.8 GB per fp32 state copy), headline physics, fp32, observables
    every interval.  Step variant 1 (32 x 16 tiles) with the z-chunk chosen by
    a short sweep (three intervals each, measurements on the device); then
    n_pulses intervals timed with their trace."""
    import paper_1610_04914_amd as P
    lat = P.Lattice((1024, 1024, 2047), precision="fp32", init="random", seed=0)
    p = P.Params(**PHYS)
    n = int(round(PHYS["Dt"] / PHYS["dt"]))
    sweep = {}
    for bz in (128, 256, 512, 1024, 2047):
        lat.set_step_config(1, bz)
        lat.run(p, 10**6, 1, obs_every=1, trace=False)
        el, _ = _timed(lambda: lat.run(p, 10**6 + 1, 3, obs_every=1, trace=False))
        sweep[bz] = lat.N * n * 3 / el
    best = max(sweep, key=sweep.get)
    lat.set_step_config(1, best)
    el, tr = _timed(lambda: lat.run(p, 0, n_pulses, obs_every=1))
    rate = lat.N * n * n_pulses / el
    N = lat.N
    lat.close()
    return {"workload": "1024x1024x2047 (2.15e9 sites), headline physics, fp32, obs every interval",
            "sites": N, "pulses": n_pulses, "bz": best, "spin_steps_per_s": rate,
            "alg_hbm_frac": rate * BYTES_PER_SPIN_STEP["fp32"] / (HBM_PEAK_GBS * 1e9),
            "bz_sweep_spin_steps_per_s": sweep, "final_E_per_site": tr[-1]["E_total"] / N}


def extra_integrators(n_pulses: int = 50):
    """The headline lattice and physics (128^3 fp32, precession, dt = 0.2,
    Dt = 2) stepped with each integrator of the Appendix: classical RK4 (one
    fused launch per step), RK2 midpoint (two steps per fused launch) and
    Butcher's RK5 (two fused launches per step: stages 1-4, stages 5-6).
    Spin-steps/s over n_pulses intervals with observables, the mean kernel
    time of the fused step launches of an even run of steps (RK4: one step,
    RK2: two steps), and each method's time per step relative to RK4's."""
    import torch
    import paper_1610_04914_amd as P
    out = {}
    for method in ("rk4", "rk2mid", "rk5b"):
        p = P.Params(**dict(PHYS, integrator=method))
        lat = P.Lattice(SHAPE, precision="fp32", init="random", seed=0)
        lat.autotune(p, cache_path=TUNE_CACHE)
        _prepare_timing(lat)
        lat.run(p, first_pulse=0, n_pulses=3, obs_every=1)
        el, _ = _timed(lambda: lat.run(p, first_pulse=3, n_pulses=n_pulses, obs_every=1))
        n = int(round(PHYS["Dt"] / PHYS["dt"]))
        rec = {"spin_steps_per_s": lat.N * n * n_pulses / el, "pulses": n_pulses}
        if method != "rk5b":
            lat.kernel_timing_start()
            lat.step(p, 40)
            ms, nt = lat.kernel_timing_stop()
            steps_per_launch = 2 if method == "rk2mid" else 1
            rec["fused_launch_us"] = ms * 1e3
            rec["steps_per_launch"] = steps_per_launch
            rec["launches_timed"] = nt
        out[method] = rec
        lat.close()
    torch.cuda.synchronize()
    for method in ("rk2mid", "rk5b"):
        out[method]["step_time_vs_rk4"] = (out["rk4"]["spin_steps_per_s"] /
                                           out[method]["spin_steps_per_s"])
    return out


def extra_escape(n_runs: int = 65536):
    """Thermally activated escape of a uniaxial spin in a transverse field
    (D = 1, H = 1, h = 1/2; the paper's reference set dt = 1/6, Dt = 1 with
    Butcher's RK5): per damping lambda and barrier sigma (1 - h)^2 with
    sigma = D/T, n_runs independent spins on the GPU, capped at three
    theoretical mean first-passage times; Gamma = escaped runs / total time
    at risk (censored exponential estimate), compared with the
    intermediate-damping rate (A = 1) and the interpolated rate with F(1/2)
    from the paper's one-dimensional formula (1.904) and from its contour
    definition (4/3)."""
    import numpy as np
    import torch
    import paper_1610_04914_amd as P
    import oracle as orc
    D, H, dt, Dt = 1.0, 1.0, 1.0 / 6.0, 1.0
    n = int(round(Dt / dt))
    f17, fc = orc.escape_F(0.5), 4.0 / 3.0
    rows = []
    tot_steps, tot_s = 0.0, 0.0
    for sigma in (10.0, 16.0):
        T = D / sigma
        g_id = orc.escape_rate_theory(D, H, 0.1, T, "ID")
        for lam in (0.1, 0.03, 0.01, 0.003, 0.001):
            g_th = orc.escape_rate_theory(D, H, lam, T, "ILD")
            maxp = int(3.0 / (g_th * Dt)) + 10
            el, tt = _timed(lambda: P.escape_times(D, H, lam, T, dt, Dt, n_runs, seed=1,
                                                   max_pulses=maxp, integrator="rk5b"))
            t = tt.cpu().numpy()
            esc = t > 0
            risk = float(np.where(esc, t, maxp * Dt).sum())
            g = float(esc.sum()) / risk
            a17 = lam * sigma * f17
            ac = lam * sigma * fc
            tot_steps += risk / dt
            tot_s += el
            rows.append({"sigma": sigma, "lambda": lam, "escaped": float(esc.mean()), "gamma": g,
                         "gamma_over_ID": g / g_id,
                         "gamma_over_ILD_F1.904": g / (g_id * a17 / (1 + a17)),
                         "gamma_over_ILD_F4/3": g / (g_id * ac / (1 + ac)),
                         "seconds": el})
    torch.cuda.synchronize()
    return {"workload": f"{n_runs} runs per point, h = 1/2, RK5 dt = 1/6, Dt = 1",
            "single_spin_steps_per_s": tot_steps / tot_s, "points": rows}


def extra_precision(L: int = 64, intervals: int = 4):
    """Error of the GPU path against the FP64 oracle for every observable:
    the headline physics on an L^3 lattice, fp32 and fp64 state; each
    interval (10 RK4 steps with the kick) is run by the GPU and by the oracle
    started from the GPU's state before it, and the largest error over the
    intervals is reported: spin components (absolute; spins are unit
    vectors), energies and magnetisation components (relative to the total
    energy per site and to 1), and the norm deviation (absolute)."""
    import numpy as np
    import torch
    import paper_1610_04914_amd as P
    import oracle as orc
    shape = (L, L, L)
    g = orc.geom(shape)
    op = orc.Params(J=PHYS["J"], H=PHYS["H"], D=PHYS["D"], e=PHYS["e"], lam=PHYS["lam"], T=PHYS["T"],
                    dt=PHYS["dt"], Dt=PHYS["Dt"], precession=True)
    gp = P.Params(**PHYS)
    N = float(L**3)
    out = {"workload": f"{L}^3, headline physics, {intervals} intervals of 10 RK4 steps"}
    for prec in ("fp32", "fp64"):
        lat = P.Lattice(shape, precision=prec, init="random", seed=0)
        err = {k: 0.0 for k in ("state", "E_total", "E_exch", "E_zeeman", "E_anis", "m",
                                "max_norm_dev")}
        for q in range(intervals):
            torch.cuda.synchronize()
            s0 = lat.state.double().cpu().numpy()
            tr = lat.run(gp, first_pulse=q, n_pulses=1, obs_every=1)[0]
            s1 = lat.state.double().cpu().numpy()
            want, otr, _ = orc.run(g, op, s0, seed=PHYS["seed"], first_pulse=q, n_pulses=1,
                                   obs_every=1)
            o = otr[0]
            err["state"] = max(err["state"], float(np.max(np.abs(s1 - want))))
            scale = abs(o["E_total"]) / N
            for k in ("E_total", "E_exch", "E_zeeman", "E_anis"):
                err[k] = max(err[k], abs(tr[k] - o[k]) / N / scale)
            err["m"] = max(err["m"], float(np.max(np.abs(np.array(tr["m"]) - np.array(o["m"])))))
            err["max_norm_dev"] = max(err["max_norm_dev"], abs(tr["max_norm_dev"] - o["max_norm_dev"]))
        out[prec] = err
        lat.close()
    return out


def extra_headline_variants(lat, p, n_pulses: int = 400, repeats: int = 5):
    """The headline lattice after its timed run: `repeats` runs of `n_pulses`
    intervals with the observables measured every interval (as timed above) and
    with them measured once at the end only; median and range of each."""
    import torch
    n = int(round(PHYS["Dt"] / PHYS["dt"]))
    out = {}
    q = 10**6
    for name, every in (("obs_every_interval", 1), ("obs_at_end_only", 0)):
        rates = []
        for _ in range(repeats):
            def go():
                lat.run(p, first_pulse=q, n_pulses=n_pulses, obs_every=every)
                if every == 0:
                    lat.observables(p)
            el, _ = _timed(go)
            rates.append(lat.N * n * n_pulses / el)
        rates.sort()
        out[name] = {"spin_steps_per_s_median": rates[len(rates) // 2], "min": rates[0],
                     "max": rates[-1], "repeats": repeats, "intervals_each": n_pulses}
    torch.cuda.synchronize()
    return out


def extra_headline_256(n_pulses: int = 100):
    """The headline physics on 256^3 (fp32, 201 MB per state copy, so the two
    copies a step reads and writes exceed the 256 MB Infinity Cache): rate, and
    the fused step's mean duration from dispatch events as algorithmic HBM
    bandwidth."""
    import torch
    import paper_1610_04914_amd as P
    shape = (256, 256, 256)
    p = P.Params(**PHYS)
    lat = P.Lattice(shape, precision="fp32", init="random", seed=0)
    variant, bz = configure_lattice(lat, "fp32", shape)
    n = int(round(PHYS["Dt"] / PHYS["dt"]))
    _prepare_timing(lat)
    lat.run(p, first_pulse=0, n_pulses=20, obs_every=1)
    lat.kernel_timing_start()
    el, _ = _timed(lambda: lat.run(p, first_pulse=20, n_pulses=n_pulses, obs_every=1))
    ms, nt = lat.kernel_timing_stop()
    N = lat.N
    lat.close()
    torch.cuda.synchronize()
    gbs = BYTES_PER_SPIN_STEP["fp32"] * N / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    alg = BYTES_PER_SPIN_STEP["fp32"] * N
    meas = measured_traffic(TRAFFIC_FILE_256)
    return {"workload": "256^3, headline physics, fp32, obs every interval",
            "spin_steps_per_s": N * n * n_pulses / el, "step_variant": variant, "bz": bz,
            "fused_launch_us": ms * 1e3, "launches_timed": nt,
            "alg_hbm_gbs": gbs, "alg_hbm_frac": gbs / HBM_PEAK_GBS,
            "alg_bytes_per_launch": alg, "l2_fabric_bytes_per_launch": meas,
            "measured_over_algorithmic": meas / alg if meas else None}


def extra_headline_fp64(n_pulses: int = 300):
    """The headline workload in fp64 (128^3, the same physics and schedule,
    observables every interval): rate, and the fused step's mean duration
    from dispatch events with its algorithmic bandwidth (48 B per spin-step)."""
    import torch
    import paper_1610_04914_amd as P
    p = P.Params(**PHYS)
    lat = P.Lattice(SHAPE, precision="fp64", init="random", seed=0)
    variant, bz = configure_lattice(lat, "fp64", SHAPE)
    n = int(round(PHYS["Dt"] / PHYS["dt"]))
    _prepare_timing(lat)
    lat.run(p, first_pulse=0, n_pulses=50, obs_every=1)
    lat.kernel_timing_start()
    el, _ = _timed(lambda: lat.run(p, first_pulse=50, n_pulses=n_pulses, obs_every=1))
    ms, nt = lat.kernel_timing_stop()
    N = lat.N
    lat.close()
    torch.cuda.synchronize()
    gbs = BYTES_PER_SPIN_STEP["fp64"] * N / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"workload": "128^3, headline physics, fp64, obs every interval",
            "spin_steps_per_s": N * n * n_pulses / el, "intervals": n_pulses,
            "step_variant": variant, "bz": bz, "fused_launch_us": ms * 1e3,
            "launches_timed": nt, "alg_hbm_gbs": gbs, "alg_hbm_frac": gbs / HBM_PEAK_GBS}


def extra_config_16():
    """The small-lattice configuration in full: 16^3 periodic, J = 1, H = D = 0,
    lambda = 0.01, T = 1, fp64, RK4 dt = 0.1, a pulse every Dt = 1 (10 steps),
    1000 pulses from a random start (seed 0), observables every interval; on
    the GPU and with the FP64 oracle on one host thread (the same work; the
    trajectories part ways after a few intervals, as chaotic ones do, so only
    the final energies' magnitude is comparable).  Latency-bound on the GPU:
    4096 sites are 16 workgroups of the fused step."""
    import numpy as np
    import paper_1610_04914_amd as P
    import oracle as orc
    shape = (16, 16, 16)
    kw = dict(J=1.0, H=(0.0, 0.0, 0.0), D=0.0, e=(0.0, 0.0, 1.0), lam=0.01, T=1.0, dt=0.1, Dt=1.0)
    n_pulses = 1000
    lat = P.Lattice(shape, precision="fp64", init="random", seed=0)
    s0 = lat.state.double().cpu().numpy()
    variant, bz = configure_lattice(lat, "fp64", shape, P.Params(seed=0, **kw))
    lat.run(P.Params(seed=0, **kw), first_pulse=0, n_pulses=20)  # first launches
    lat.state.copy_(lat.state.new_tensor(s0))
    el_g, tr = _timed(lambda: lat.run(P.Params(seed=0, **kw), first_pulse=0, n_pulses=n_pulses,
                                      obs_every=1))
    lat.close()
    t0 = time.perf_counter()
    _, otr, _ = orc.run(orc.geom(shape), orc.Params(**kw), s0, seed=0, n_pulses=n_pulses,
                        obs_every=n_pulses)
    el_c = time.perf_counter() - t0
    N = int(np.prod(shape))
    steps = 10 * n_pulses
    return {"workload": "16^3 fp64, 1000 pulses of 10 RK4 steps", "step_variant": variant, "bz": bz,
            "gpu_spin_steps_per_s": N * steps / el_g,
            "oracle_spin_steps_per_s": N * steps / el_c, "oracle_seconds": el_c,
            "gpu_final_E_per_site": tr[-1]["E_total"] / N,
            "oracle_final_E_per_site": otr[-1]["E_total"] / N}


def extra_temperatures(n_pulses: int = 1000, tail: int = 500):
    """The headline workload at the three temperatures of its specification
    (T = 0.5, 1.0, 1.4; fp32, random start, seed 0): rate, and the time averages
    of E/N and |m| over the last `tail` intervals."""
    import torch
    import paper_1610_04914_amd as P
    out = {}
    for T in (0.5, 1.0, 1.4):
        p = P.Params(**dict(PHYS, T=T))
        lat = P.Lattice(SHAPE, precision="fp32", init="random", seed=0)
        configure_lattice(lat, "fp32", SHAPE)
        n = int(round(PHYS["Dt"] / PHYS["dt"]))
        el, tr = _timed(lambda: lat.run(p, first_pulse=0, n_pulses=n_pulses, obs_every=1))
        last = tr[-tail:]
        N = lat.N
        out[f"T={T}"] = {
            "spin_steps_per_s": N * n * n_pulses / el,
            "E_per_site": sum(o["E_total"] for o in last) / (len(last) * N),
            "abs_m": sum(math.sqrt(sum(c * c for c in o["m"])) for o in last) / len(last),
            "intervals": n_pulses, "averaged_over": tail}
        lat.close()
    torch.cuda.synchronize()
    return out


def _progress(name, fn):
    """Runs one extra workload and reports its wall time on stderr."""
    t0 = time.perf_counter()
    r = fn()
    print(f"extra {name}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return r


EXTRAS = {"temperatures": extra_temperatures, "headline_256": extra_headline_256,
          "headline_fp64": extra_headline_fp64,
          "config_16": extra_config_16, "batched": extra_batched, "adjoint": extra_adjoint,
          "overdamped_256": extra_overdamped, "max_lattice": extra_max_lattice,
          "integrators": extra_integrators,
          "escape": extra_escape, "precision": extra_precision}


def main():
    global ACC_PULSES
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed intervals (pulses)")
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--no-settle", dest="settle", action="store_false",
                    help="skip the untimed run of the timed length before a short warm-up")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-steps-all-cores", type=int, default=40)
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="skip the batched, adjoint and 256^3 overdamped workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--acc-pulses", type=int, default=ACC_PULSES,
                    help="pulses of the batched accuracy runs (fp32 and fp64 batches)")
    ap.add_argument("--extra", default=None, metavar="NAME",
                    help="only run the named extra workload (one of: " + ", ".join(EXTRAS) +
                         ") and print its JSON")
    args = ap.parse_args()
    ACC_PULSES = args.acc_pulses
    if args.extra is not None:
        if args.extra not in EXTRAS:
            ap.error(f"unknown extra {args.extra!r}")
        import warnings
        import paper_1610_04914_amd as P
        warnings.simplefilter("ignore", P.ApplicabilityWarning)
        print(json.dumps({args.extra: EXTRAS[args.extra]()}))
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * 2**20 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is "
              "not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1610_04914_amd as P

    prec = args.precision
    p = P.Params(**PHYS)
    lat = P.Lattice(SHAPE, precision=prec, init="random", seed=0)
    variant, bz = configure_lattice(lat, prec, SHAPE)
    N = lat.N
    n = int(round(PHYS["Dt"] / PHYS["dt"]))

    import warnings
    warnings.simplefilter("ignore", P.ApplicabilityWarning)
    # Settling: in a fresh process the first run with as many intervals in flight
    # as the timed one is about 7% slower than later runs of the same length
    # (measured; shorter runs before it, even for a second, do not remove the
    # effect).  Unless the warm-up is already that long, one untimed run of the
    # timed length (pulse indices outside the timed range) precedes the warm-up.
    # A short warm-up is then extended by untimed runs until about a second of
    # GPU work has passed: after a few milliseconds of work the step kernel
    # still runs about 8% slower than in steady state (measured: 20 timed
    # intervals after a 5-interval warm-up gave 0.350 ms per interval, 200
    # after 20 gave 0.309).
    # Host set-up that the timed region needs (the library's dispatch events)
    # is done here: the GPU's clock drops within milliseconds of idling
    # (measured: 20 intervals started 10 ms after the previous work ran at
    # 5.9e10 spin-steps/s, back to back at 6.9e10), so nothing but the
    # synchronisation separates the warm-up from the timed run.
    _prepare_timing(lat)
    if args.settle and args.warmup < args.steps:
        lat.run(p, first_pulse=10**7, n_pulses=args.steps, obs_every=1)
        torch.cuda.synchronize()
    if args.settle:
        t_end = time.perf_counter() + 1.0
        q = 0
        while time.perf_counter() < t_end:
            lat.run(p, first_pulse=2 * 10**7 + q, n_pulses=100, obs_every=1, trace=False)
            torch.cuda.synchronize()
            q += 100
    lat.run(p, first_pulse=0, n_pulses=args.warmup, obs_every=1, raw=True)
    torch.cuda.synchronize()
    # Dominant kernel: the fused RK4 step.  Its mean duration comes from event
    # pairs that a sample of the timed region's step launches record at their
    # own dispatch (start and end of the kernel, as a kernel trace sees them).
    lat.kernel_timing_start()
    # The timed region is the wall time between two synchronisations (timing
    # events recorded on the stream around it would add about 40 us of their
    # own to it).  The trace comes back to the host inside it; its records
    # become Python dicts after it.
    t0 = time.perf_counter()
    trace = lat.run(p, first_pulse=args.warmup, n_pulses=args.steps, obs_every=1, raw=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms, n_timed = lat.kernel_timing_stop()
    spin_steps = N * n * args.steps
    value = spin_steps / elapsed
    alg_bytes = BYTES_PER_SPIN_STEP[prec] * N
    alg_flops = FLOPS_PER_SPIN_STEP * N
    achieved_gbs = alg_bytes / (step_ms * 1e-3) / 1e9 if step_ms > 0 else 0.0
    achieved_tf = alg_flops / (step_ms * 1e-3) / 1e12 if step_ms > 0 else 0.0
    traffic = measured_traffic() if prec == "fp32" else None

    out = {
        "metric": METRIC if prec == "fp32" else "spin-steps/s (RK4, 128^3 sc, fp64)",
        "value": value,
        "unit": "spin-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic (random-sphere initial state, Philox noise)",
        "config": {"workload": "128^3 sc PBC, J=1, H=(0,0,0.1), D=0.05 z, lambda=0.01, T=1.0, "
                               "RK4 dt=0.2, Dt=2.0 (n=10), obs every interval",
                   "sites": N, "rk4_steps_per_interval": n, "intervals": args.steps,
                   "step_variant": variant, "bz": bz, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": ALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / ALU_PEAK_TFLOPS,
                     "traffic": traffic,
                     "traffic_kind": "L2<->fabric bytes per launch (FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated); at 128^3 reads served by the Infinity "
                                     "Cache are included (256^3 figure in extras.headline_256)",
                     "kernel": "rk4_fused_kernel",
                     "alg_flops_per_launch": alg_flops,
                     "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": step_ms, "launches_timed": n_timed,
                     "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved_gbs / HBM_PEAK_GBS}},
        "final_obs": P.obs_row_dict(trace[len(trace) - 1]) if len(trace) else None,
    }
    if args.extras:
        out["extras"] = {"headline_variants": extra_headline_variants(lat, p),
                         **{name: _progress(name, fn) for name, fn in EXTRAS.items()}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, args.cpu_steps_all_cores)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
