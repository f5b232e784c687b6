"""Benchmark of the M2M + moving-prior step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2|3|4]

A step is one pass of the whole hot path over every particle: force of
change, leapfrog push, deposit into the observables, time smoothing,
residuals and chi^2, and (every 25 correction steps) the moving priors.
Inputs are synthetic and seeded (``workloads``); targets are the library's
own measurement of a realization of the target distribution function.

Prints one JSON line with the throughput (particle-steps/s, particles
resident in HBM), the roofline of the fused step kernel (HIP-event timing of
its launches; algorithmic bytes: 60 per particle-step in FP32) and a CPU
baseline (the FP64 oracle on the host cores, bounded sample).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# launch shape (threads per block, particles per lane, tiles per CU) of the
# fused step kernel per workload, as chosen by paper_1202_2355_amd.autotune
LAUNCH = {1: (256, 1, 4), 2: (256, 4, 4), 3: (256, 4, 4), 4: (256, 4, 4), 5: (256, 4, 4)}

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BYTES_PER_PSTEP = {"f32": 60, "f64": 120}   # read x, v, u, uhat; write x, v, u
KERNEL_SOURCES = ("paper_1202_2355_amd/csrc/m2m_kernels.hip",)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name: str, n_particles: int):
    """HBM bytes per particle-step of the fused kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(workload_name)
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    return e["bytes_per_launch"] / float(n_particles)


def make_fit_and_targets(wl, Fit, dtype="f32"):
    from workloads import make_targets
    tp = wl.target_particles()
    tfit = Fit(wl.potential, wl.layout, wl.params, tp, dtype=dtype)
    T = make_targets(lambda V, S: tfit.observe(V, S), wl)
    tfit.close()
    del tp
    ic = wl.initial_particles()
    fit = Fit(wl.potential, wl.layout, wl.params, ic, dtype=dtype)
    fit.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    return fit


def cpu_baseline(wl, seconds: float):
    """The FP64 oracle on this host's cores over a bounded sample of the same
    workload (its own targets, measured by the oracle)."""
    from oracle import oracle as O
    from workloads import make_targets
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    tp = wl.target_particles(n=1 << 20)
    ones = np.ones(tp["x"].size)
    T = make_targets(lambda V, S: O.deposit(tp, ones, wl.layout, V_p=V, sigma_p=S, nthreads=cores),
                     wl)
    n = min(wl.N, 1_000_000)
    ic = wl.initial_particles(n=n)
    f = O.OracleFit(wl.potential, wl.layout, wl.params, ic, T["Y"], T["sigma"], T["V_p"],
                    T["sigma_p"], nthreads=cores)
    t0 = time.perf_counter()
    f.step(1)
    t1 = time.perf_counter() - t0
    k = max(1, min(200, int(seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    f.step(k)
    dt = time.perf_counter() - t0
    return {"value": n * k / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} particles of {wl.name}, {k} steps after 1 untimed step "
                      f"(FP64, OpenMP, targets from a 2^20-particle target realization)"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2, 3])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the M2M path here is a "
              "single-GPU build", file=sys.stderr)
        return 2

    import torch
    from paper_1202_2355_amd import _abi
    from paper_1202_2355_amd.fit import Fit
    from workloads import workload

    wl = workload(args.workload)
    dtype = wl.state
    _abi.m2m_set_launch(*LAUNCH[args.workload])
    print(f"[bench] {wl.name}: N={wl.N} J={wl.J} dtype={dtype} launch={LAUNCH[args.workload]}",
          file=sys.stderr, flush=True)
    fit = make_fit_and_targets(wl, Fit, dtype)
    fit.step(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record()
    fit.step(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1)
    ob = fit.observables()
    print(f"[bench] timed {args.steps} steps: {ms:.3f} ms (wall {1e3 * t_wall:.3f} ms), "
          f"chi2/J {ob['chi2'] / wl.J:.4f}", file=sys.stderr, flush=True)
    ms_step, ms_fin = fit.profile_step(50)
    bpp = BYTES_PER_PSTEP[dtype]
    achieved = bpp * wl.N / (ms_step * 1e-3) / 1e9
    tb = measured_traffic(wl.name, wl.N)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (tb * wl.N if tb is not None else None),
            "kernel": "k_step (fused force of change + push + deposit)",
            "kernel_ms": ms_step, "finalize_ms": ms_fin,
            "bytes_per_particle_step": bpp}
    fit.close()
    value = wl.N * args.steps / (ms * 1e-3)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.cpu_seconds)
    out = {
        "metric": "particle-steps/sec (push+deposit+weight update) at 1 GPU",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl.name, "particles": wl.N, "observables": wl.J,
                   "kinematics": wl.layout["kin"], "prior_grid": [wl.params["n_E"], wl.params["n_x"]],
                   "prior_every": wl.params["prior_every"], "state": dtype,
                   "launch": list(LAUNCH[args.workload])},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
