"""Benchmark of the M2M + moving-prior step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 1|2|3|4|5]

A step is one pass of the whole hot path over every particle: force of
change, leapfrog push, deposit into the observables, time smoothing,
residuals and chi^2, and (every 25 correction steps) the moving priors.
Inputs are synthetic and seeded (``workloads``); targets are the library's
own measurement of a realization of the target distribution function.

The default workload is the batch of 64 fits of uneven size (Sigma N about
3.6e7 particles, 1.2 GB of FP32 state: far beyond the 256 MB memory-side
cache), stepped by one fused step kernel and one finalize per step. Prints
one JSON line with the whole-step throughput (particle-steps/s, particles
resident in HBM), the roofline of the fused step kernel (HIP-event timing of
its launches on the batch stream; algorithmic bytes: 60 per particle-step in
FP32) beside the whole step's, the same fits stepped one launch per fit, and
a CPU baseline (the FP64 oracle on the host cores, bounded sample).
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

SERVE_N_MIN = 100_000   # smallest fit of the serving trace (errors floored at its noise)
METRIC = "particle-steps/sec (push+deposit+weight update) at 1 GPU; p50/p99 fit latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
GRAPH_STEPS = 32               # steps per captured graph of one fit in the library
BYTES_PER_PSTEP = {"f32": 60, "f64": 120}   # read x, v, u, uhat; write x, v, u
# the sources of the step kernel (the kernel the counters are taken on): its
# code, its launchers, the device helpers and structures it uses
KERNEL_SOURCES = tuple(f"paper_1202_2355_amd/csrc/{f}" for f in (
    "m2m_device.h", "m2m_step.h", "m2m_step_f32d.hip", "m2m_step_f32f.hip", "m2m_step_f64.hip",
    "m2m_internal.h"))
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
    # the same oracle on one thread, over a tenth of the particles for about a
    # third of the time
    n1 = max(1, n // 10)
    f1 = O.OracleFit(wl.potential, wl.layout, wl.params, {key: v[:n1] for key, v in ic.items()},
                     T["Y"], T["sigma"], T["V_p"], T["sigma_p"], nthreads=1)
    t0 = time.perf_counter()
    f1.step(1)
    t1 = time.perf_counter() - t0
    k1 = max(1, min(200, int(seconds / 3 / max(t1, 1e-6))))
    t0 = time.perf_counter()
    f1.step(k1)
    dt1 = time.perf_counter() - t0
    return {"value": n * k / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} particles of {wl.name}, {k} steps after 1 untimed step "
                      f"(FP64, OpenMP, targets from a 2^20-particle target realization)",
            "value_1_thread": n1 * k1 / dt1,
            "sample_1_thread": f"the first {n1} of those particles, {k1} steps after 1 untimed step, "
                               f"one thread"}


PREWARM_MS = 300.0  # device copies before the warm-up steps


def prewarm_device(torch, ms: float = PREWARM_MS) -> str:
    """Keep the GPU streaming memory (256 MiB device copies) for about `ms`
    milliseconds. Input generation leaves it nearly idle for seconds, and
    its clocks then take tens of milliseconds of load to come back: the
    first ~20 steps after an idle second run ~10 % slower than the steps of
    any fit of hundreds of steps. The copies touch no fit; the W warm-up
    steps and the K timed steps follow as usual."""
    src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t0 = time.perf_counter()
    n = 0
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(20):
            dst.copy_(src)
        n += 20
        torch.cuda.synchronize()
    del src, dst
    return f"{n} device copies of 256 MiB ({ms:.0f} ms) before the warm-up steps"


def cpu_baseline_batch(fits_wl, seconds: float, n_cap: int = 1 << 18):
    """The FP64 oracle on this host's cores over the first fits of the batch
    (each fit's own potential and targets, at most n_cap of its particles),
    run one after another as a CPU would run them: total particle-steps over
    total time."""
    from oracle import oracle as O
    from workloads import make_targets
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    work, spent, used, nsum, ksum = 0.0, 0.0, 0, 0, 0
    for wl in fits_wl:
        if spent >= seconds:
            break
        tp = wl.target_particles(n=1 << 16)
        ones = np.ones(tp["x"].size)
        T = make_targets(lambda V, S: O.deposit(tp, ones, wl.layout, V_p=V, sigma_p=S,
                                                nthreads=cores), wl)
        n = min(wl.N, n_cap)
        ic = wl.initial_particles(n=n)
        f = O.OracleFit(wl.potential, wl.layout, wl.params, ic, T["Y"], T["sigma"], T["V_p"],
                        T["sigma_p"], nthreads=cores)
        t0 = time.perf_counter()
        f.step(1)
        t1 = time.perf_counter() - t0
        k = max(1, min(100, int(seconds / 4 / max(t1, 1e-6))))
        t0 = time.perf_counter()
        f.step(k)
        dt = time.perf_counter() - t0
        work += n * k
        spent += dt
        used += 1
        nsum += n
        ksum += k
    return {"value": work / spent, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"the first {used} fits of the batch ({nsum} particles: each fit's first "
                      f"min(N, {n_cap}) particles, its own potential and targets), "
                      f"{ksum} steps in all after one untimed step per fit, run one fit after "
                      f"another with all cores (FP64, OpenMP); total particle-steps over total "
                      f"time"}


def run_batch(args, Fit, torch, _abi):
    """Workload 4: 64 fits of uneven size stepping as one batch, against the
    same fits stepped one launch per fit."""
    from paper_1202_2355_amd.batch import Batch
    from workloads import make_targets
    from workloads.configs import batch_fits
    from workloads.device import om_model_device
    fits_wl = batch_fits(args.fits)
    from paper_1202_2355_amd import tuning
    fits = []
    t0 = time.perf_counter()
    # each context takes the tuned parameters of a single fit of its size at
    # creation (the comparator steps them one launch per fit); the batch
    # takes the batch class's at its rebuild
    for wl in fits_wl:
        tuning.use("single", "f32", wl.layout, wl.N)
        ic = om_model_device(wl.N, wl.potential, float("inf"), seed=wl.seed * 10 + 1)
        tp = om_model_device(wl.n_target, wl.potential, wl.target_ra, seed=wl.seed * 10 + 2)
        tf = Fit(wl.potential, wl.layout, wl.params, tp, dtype="f32")
        T = make_targets(lambda V, S: tf.observe(V, S), wl)
        tf.close()
        f = Fit(wl.potential, wl.layout, wl.params, ic, dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        fits.append(f)
        del ic, tp
    ntot = sum(f.n for f in fits)
    print(f"[bench] batch of {len(fits)} fits, {ntot} particles, inputs in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    tuned = tuning.use("batch", "f32", fits_wl[0].layout)
    if args.groups is not None:
        _abi.m2m_set_batch_groups(args.groups)
        tuned["groups"] = args.groups
    b = Batch(max_fits=len(fits))
    for f in fits:
        assert b.admit(f, args.warmup + args.steps + 40)
    prewarm = prewarm_device(torch)
    b.run(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    b.run(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    assert b.particles() == ntot
    ms_step, ms_fin = b.profile(32)
    for f in list(fits):
        b.cancel(f)
    # comparator: the same fits, each stepped by its own launches
    k_alone = max(4, args.steps // 10)
    ev0.record()
    for _ in range(k_alone):
        for f in fits:
            f.step(1)
    ev1.record()
    torch.cuda.synchronize()
    ms_alone = ev0.elapsed_time(ev1) / k_alone
    b.close()
    for f in fits:
        f.close()
    cpu = None if args.no_cpu_baseline else cpu_baseline_batch(fits_wl, args.cpu_seconds)
    return {"name": f"batch{len(fits)}_gh", "N": ntot, "J": fits_wl[0].J, "ms": ms,
            "ms_step": ms_step, "ms_fin": ms_fin, "dtype": "f32", "layout": fits_wl[0].layout,
            "params": fits_wl[0].params, "fits": len(fits), "cpu": cpu, "tuned": tuned,
            "prewarm": prewarm,
            "comparator": {"kind": "the same fits, one step kernel and one finalize launch per fit",
                           "value": ntot / (ms_alone * 1e-3), "unit": "particle-steps/s",
                           "ms_per_step": ms_alone, "steps": k_alone}}


SERVE_RATE = 20.0  # requests per second of the serving trace


def run_serve(args, torch, rate=SERVE_RATE):
    """Workload 5: a Poisson trace of fit requests through the continuous-
    batching server; throughput and p50/p99 latency. At another arrival rate
    the same requests arrive at times scaled by SERVE_RATE / rate."""
    from paper_1202_2355_amd.fit import Fit
    from paper_1202_2355_amd.serve import Request, Server
    from workloads import add_noise, floor_model_noise, workload
    from workloads.configs import serve_trace
    from workloads.device import om_model_device, plummer_jeans_device
    base = workload(3)
    tp = om_model_device(1 << 22, base.potential, base.target_ra, seed=base.seed * 10 + 2)
    tf = Fit(base.potential, base.layout, base.params, tp, dtype=args.state)
    Y_true = tf.observe()
    tf.close()
    del tp
    levels = (0.01, 0.02, 0.05)
    datasets = []
    for k, s in enumerate(levels):
        Y, sig = add_noise(Y_true, base.layout, s, np.random.Generator(np.random.Philox(key=50 + k)))
        datasets.append({"Y": Y, "sigma": floor_model_noise(Y_true, sig, SERVE_N_MIN)})
    arrival, wls = serve_trace(n_requests=args.requests, state=args.state)
    arrival = np.asarray(arrival) * (SERVE_RATE / rate)
    reqs = [Request(rid=k, arrival=float(arrival[k]), potential=w.potential, params=w.params,
                    layout=w.layout, n=w.N, steps=w.steps, dataset=levels.index(w.noise),
                    seed=w.seed) for k, w in enumerate(wls)]
    tdt = torch.float32 if args.state == "f32" else torch.float64
    model = lambda r: plummer_jeans_device(r.n, r.potential, r.seed, dtype=tdt)
    from paper_1202_2355_amd import tuning
    tuning.use("batch", args.state, base.layout)
    srv = Server(datasets, hbm_budget=int(args.hbm_gb * 2 ** 30), max_fits=args.max_fits,
                 steps_per_launch=args.steps_per_launch, dtype=args.state, initial_model=model,
                 preparers=args.preparers)
    # warm-up request (first graph capture, first allocations), not counted
    srv.run([Request(rid=-1, arrival=0.0, potential=base.potential, params=base.params,
                     layout=base.layout, n=100_000, steps=64, dataset=0, seed=1)])
    m = srv.run(reqs, realtime=True, log=sys.stderr)
    srv.close()
    return m


def static_mix(torch, steps=128):
    """The serving trace's first 64 requests admitted at once as one static
    batch (the saturation reference of the server): whole-step particle-
    steps/s over ``steps`` steps, after a device warm-up and 32 steps."""
    from paper_1202_2355_amd import tuning
    from paper_1202_2355_amd.autotune import losvd_mix_fits
    from paper_1202_2355_amd.batch import Batch
    from workloads import workload
    tuning.use("batch", "f32", workload(3).layout)
    fits, _, _ = losvd_mix_fits(64)
    n = sum(f.n for f in fits)
    b = Batch(max_fits=len(fits))
    for f in fits:
        if not b.admit(f, steps + 64):
            raise RuntimeError("static mix: admission failed")
    prewarm_device(torch)
    b.run(32)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.run(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for f in fits:
        b.cancel(f)
        f.close()
    b.close()
    return {"fits": len(fits), "particles": n, "us_per_step": 1e3 * ms,
            "particle_steps_per_s": n / (ms * 1e-3)}


def parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", type=int, default=4, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--fits", type=int, default=64, help="workload 4: number of fits")
    ap.add_argument("--groups", type=int, default=None, choices=[1, 2],
                    help="workload 4: step the batch as 1 or 2 overlapping groups "
                         "(default: the library's choice)")
    ap.add_argument("--requests", type=int, default=500, help="workload 5: trace length")
    ap.add_argument("--rate", type=float, default=SERVE_RATE,
                    help="workload 5: arrival rate of the trace (requests/s)")
    ap.add_argument("--interleave", type=int, default=None, choices=[-1, 0, 1],
                    help="workloads 1-3: tiles of the step kernel take contiguous ranges (0) or "
                         "interleaved chunks (1); default: the library's choice by state size")
    ap.add_argument("--state", default=None, choices=["f32", "f64"],
                    help="particle state of workloads 2, 3 and 5 (default: the workload's own, "
                         "FP32 for the serving trace)")
    ap.add_argument("--hbm-gb", type=float, default=96.0, help="workload 5: HBM budget")
    ap.add_argument("--steps-per-launch", type=int, default=64)
    ap.add_argument("--max-fits", type=int, default=64, help="workload 5: batch slots")
    ap.add_argument("--preparers", type=int, default=4,
                    help="workload 5: threads preparing requests side by side")
    ap.add_argument("--sweep", default="", metavar="RATES",
                    help="workload 5: also serve the same trace at these arrival rates "
                         "(comma-separated, requests/s): the saturation sweep")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB float32 device copy (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--smooth", action="store_true",
                    help="workloads 1-3: thin-plate GCV smoothing of the prior grid at refreshes")
    ap.add_argument("--alm", type=int, default=None, metavar="L",
                    help="workloads 1-3: spherical-harmonic density observables a_lm (l <= L) "
                         "on a 60-point radial mesh instead of the radial mass bins")
    ap.add_argument("--scf", type=int, default=None, metavar="L",
                    help="workloads 1-3: the stellar potential from the particles, a multipole "
                         "expansion (l <= L, 32 nodes on [0.02, 100]) instead of the Hernquist part")
    ap.add_argument("--deposit", default=None, choices=["f64", "f32c"],
                    help="workloads 1-3: the in-tile deposit mode instead of the tuned one")
    ap.add_argument("--scf-every", type=int, default=10,
                    help="with --scf: steps between rebuilds of the expansion")
    return ap


def main(argv=None):
    args = parser().parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the M2M path here is a "
              "single-GPU build", file=sys.stderr)
        return 2

    if args.workload == 5 and args.state is None:
        args.state = "f32"
    if args.workload == 5:
        # the preparing threads' streams get hardware queues of their own
        # instead of queueing behind the batch's enqueued runs (read when HIP
        # starts, i.e. before torch touches the GPU)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")
    import torch
    from paper_1202_2355_amd import _abi, tuning
    from paper_1202_2355_amd.fit import Fit
    from workloads import workload

    if args.workload == 5:
        m = run_serve(args, torch, rate=args.rate)
        ref = static_mix(torch) if args.sweep else None
        sweep = []
        for rate in [float(x) for x in args.sweep.split(",") if x.strip()]:
            ms = run_serve(args, torch, rate=rate)
            sweep.append({"arrival_rate_per_s": rate, "particle_steps_per_s": ms["particle_steps_per_s"],
                          "p50_s": ms["p50_latency_s"], "p99_s": ms["p99_latency_s"]})
            print(f"[bench] serve at {rate:g}/s: {ms['particle_steps_per_s']:.3e} particle-steps/s, "
                  f"p50 {ms['p50_latency_s']:.3f} s, p99 {ms['p99_latency_s']:.3f} s",
                  file=sys.stderr, flush=True)
        out = {"metric": METRIC,
               "value": m["particle_steps_per_s"], "unit": "particle-steps/s", "n_gpus": 1,
               "steps": None, "warmup": None, "ms_per_step": None, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": args.state, "data": "synthetic",
               "config": {"workload": "serve_losvd", "requests": m["requests"],
                          "arrival_rate_per_s": args.rate, "hbm_budget_gb": args.hbm_gb,
                          "steps_per_launch": args.steps_per_launch, "preparers": args.preparers,
                          "max_fits": args.max_fits,
                          "launch": tuning.current()},
               "latency": {"p50_s": m["p50_latency_s"], "p99_s": m["p99_latency_s"],
                           "mean_s": m["mean_latency_s"]},
               **({"sweep": sweep, "static_batch": ref} if sweep else {}),
               "roofline": None, "cpu_baseline": None}
        print(json.dumps(out), flush=True)
        return 0
    if args.workload == 4:
        r = run_batch(args, Fit, torch, _abi)
        bpp = BYTES_PER_PSTEP["f32"]
        ms_per_step = r["ms"] / args.steps
        achieved = bpp * r["N"] / (r["ms_step"] * 1e-3) / 1e9
        whole = bpp * r["N"] / (ms_per_step * 1e-3) / 1e9
        tb = measured_traffic(r["name"], r["N"])
        out = {"metric": METRIC,
               "value": r["N"] / (ms_per_step * 1e-3), "unit": "particle-steps/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": r["name"], "fits": r["fits"], "particles": r["N"],
                          "observables": r["J"], "kinematics": r["layout"]["kin"],
                          "prior_grid": [r["params"]["n_E"], r["params"]["n_x"]],
                          "prior_every": r["params"]["prior_every"], "state": "f32",
                          "launch": r["tuned"], "device_warmup": r["prewarm"]},
               "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                            "traffic": (tb * r["N"] if tb is not None else None),
                            "kernel": "k_step (fused force of change + push + deposit, all fits)",
                            "kernel_ms": r["ms_step"], "finalize_ms": r["ms_fin"],
                            "bytes_per_particle_step": bpp,
                            "whole_step_achieved": whole, "whole_step_frac": whole / HBM_PEAK_GBS},
               "comparator": r["comparator"],
               "cpu_baseline": r["cpu"]}
        print(json.dumps(out), flush=True)
        return 0
    wl = workload(args.workload)
    if args.alm is not None:
        from workloads import with_alm
        wl = with_alm(wl, n_mesh=60, l_max=args.alm)
    if args.smooth:
        wl = wl.with_(name=f"{wl.name}_smooth", params=dict(wl.params, smooth=1))
    if args.scf is not None:
        from workloads import with_scf
        wl = with_scf(wl, l_max=args.scf, n_nodes=32, r_min=0.02, r_max=100.0,
                      every=args.scf_every)
    if args.state:
        wl = wl.with_(name=f"{wl.name}_{args.state}" if args.state != wl.state else wl.name,
                      state=args.state)
    dtype = wl.state
    tuned = tuning.use("single", dtype, wl.layout, wl.N)
    if args.deposit:
        tuned = dict(tuned, deposit=args.deposit)
        tuning.apply(tuned)
    if args.interleave is not None:
        _abi.m2m_set_interleave(args.interleave)
        tuned = dict(tuned, interleave=args.interleave)
    print(f"[bench] {wl.name}: N={wl.N} J={wl.J} dtype={dtype} launch={tuned}",
          file=sys.stderr, flush=True)
    fit = make_fit_and_targets(wl, Fit, dtype)
    prewarm = prewarm_device(torch)
    fit.step(args.warmup)
    graph_note = None
    if args.steps >= GRAPH_STEPS and args.warmup < GRAPH_STEPS:
        # the library captures the fit's 32-step graph at its first use: do
        # that before the timed steps, not inside them
        fit.step(GRAPH_STEPS)
        graph_note = f"{GRAPH_STEPS} more untimed steps after the warm-up captured the step graph"
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
    if args.calibrate_copy:
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    bpp = BYTES_PER_PSTEP[dtype]
    achieved = bpp * wl.N / (ms_step * 1e-3) / 1e9
    tb = measured_traffic(wl.name, wl.N)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (tb * wl.N if tb is not None else None),
            "kernel": "k_step1 (fused force of change + push + deposit)",
            "kernel_ms": ms_step, "finalize_ms": ms_fin,
            "bytes_per_particle_step": bpp,
            "whole_step_achieved": bpp * wl.N / (ms / args.steps * 1e-3) / 1e9,
            "whole_step_frac": bpp * wl.N / (ms / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS}
    fit.close()
    value = wl.N * args.steps / (ms * 1e-3)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.cpu_seconds)
    out = {
        "metric": METRIC,
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": wl.name, "particles": wl.N, "observables": wl.J,
                   "kinematics": wl.layout["kin"], "prior_grid": [wl.params["n_E"], wl.params["n_x"]],
                   "prior_every": wl.params["prior_every"], "state": dtype,
                   "prior_smoothing": bool(wl.params.get("smooth", 0)),
                   "density": (f"alm l<={wl.layout['l_max']} on {wl.layout['n_r']} radii"
                               if wl.layout.get("dens") == "alm" else "radial bins"),
                   "stellar_potential": (
                       f"multipole l<={wl.params['scf_lmax']}, {wl.params['scf_nr']} nodes, "
                       f"rebuilt every {wl.params['scf_every']} steps"
                       if wl.params.get("scf_nr", 0) else "analytic"),
                   "launch": tuned, "device_warmup": prewarm,
                   **({"graph_capture": graph_note} if graph_note else {})},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
