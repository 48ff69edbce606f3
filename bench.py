"""Benchmark of the pulse-noise LLL hot path on one MI355X.

Workload (headline): 128^3 simple-cubic lattice, periodic boundaries, J = 1,
H = (0, 0, 0.1), uniaxial D = 0.05 along z, lambda = 0.01, T = 1.0, RK4 with
dt = 0.2, pulses every Dt = 2.0 (n = 10 steps per interval), fp32 state with
fp64 reductions, random-sphere initial state from seed 0, observables measured
after every interval.  One benchmark "step" is one interval of the schedule
(n1 = 5 RK4 steps, kick, n2 = 5 RK4 steps, fp64 observables); the default
timed region is the workload's full 2000 pulses (20000 RK4 steps).

Metric: spin-steps/s = sites x RK4 steps / s (kicks and reductions are inside
the timed region but are not counted as steps).

Prints ONE JSON line.  --gpus above 1 is rejected: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
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
TUNE_CACHE = os.path.join(ROOT, "paper_1610_04914_amd", "tune_cache.txt")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rk4_fused_128c_fp32_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1610_04914_amd", "csrc", f)
                  for f in ("kern_fused.hpp", "lll_device.hpp")]


def kernel_hash() -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def configure_lattice(lat, prec: str, shape) -> tuple:
    """Step configuration used by the benchmark: the committed tuning table
    entry for this lattice when there is one, else an autotune run."""
    import paper_1610_04914_amd as P
    p = P.Params(**PHYS)
    return lat.autotune(p, cache_path=TUNE_CACHE)


def measured_traffic():
    """HBM bytes per launch of the fused step from the committed rocprofv3
    counter summary, or None when it is missing or was taken on other kernel
    sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    mh = re.search(r"kernel_sources_hash:\s*(\w+)", txt)
    mb = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not mh or not mb or mh.group(1) != kernel_hash():
        return None
    return float(mb.group(1))


def cpu_baseline(steps: int = 4):
    """The FP64 oracle (single-threaded C) on a bounded sample of the same
    workload: `steps` RK4 steps of the 128^3 lattice."""
    import numpy as np
    import oracle as orc
    g = orc.geom(SHAPE)
    p = orc.Params(J=PHYS["J"], H=PHYS["H"], D=PHYS["D"], e=PHYS["e"], lam=PHYS["lam"], T=PHYS["T"],
                   dt=PHYS["dt"], Dt=PHYS["Dt"], precession=True)
    s = orc.init_random_sphere(g, 0)
    orc.step(g, p, s, 1)  # warm-up (page in)
    t0 = time.perf_counter()
    orc.step(g, p, s, steps)
    el = time.perf_counter() - t0
    N = int(np.prod(SHAPE))
    return {"value": N * steps / el, "unit": "spin-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} RK4 steps of the 128^3 fp64 lattice ({el:.1f} s, one host thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed intervals (pulses)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
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
              "not part of this build", file=sys.stderr)
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
    lat.run(p, first_pulse=0, n_pulses=args.warmup, obs_every=1)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    trace = lat.run(p, first_pulse=args.warmup, n_pulses=args.steps, obs_every=1)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    elapsed = max(wall, ev_ms / 1e3)
    spin_steps = N * n * args.steps
    value = spin_steps / elapsed

    # Dominant kernel: the fused RK4 step.  Average launch duration from HIP
    # events around back-to-back steps on the library's stream.
    reps = 200
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    lat.step(p, 2)
    k0.record(stream)
    lat.step(p, reps)
    k1.record(stream)
    torch.cuda.synchronize()
    step_ms = k0.elapsed_time(k1) / reps
    alg_bytes = BYTES_PER_SPIN_STEP[prec] * N
    achieved = alg_bytes / (step_ms * 1e-3) / 1e9
    traffic = measured_traffic() if prec == "fp32" else None

    out = {
        "metric": "spin-steps/s (RK4, 128^3 sc, fp32)" if prec == "fp32" else "spin-steps/s (RK4, 128^3 sc, fp64)",
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
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "rk4_fused_kernel",
                     "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": step_ms},
        "final_obs": trace[-1] if trace else None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
