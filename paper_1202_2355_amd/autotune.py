"""Launch-shape search for the fused step kernel.

The shape is (threads per block, tiles per compute unit): the tile count
sets how many blocks stream the particles (and how many partial rows the
finalize reduces), the block size sets the waves per CU that share one set
of LDS bins. The
search times whole M2M steps (step + finalize kernels, graph replays) on
fresh copies of the same particles and keeps the fastest shape.
"""

from __future__ import annotations

import itertools
import json
import sys
import time

import torch

from . import _abi as A
from .fit import Fit

BLOCKS = (256, 512, 1024)
TILES_PER_CU = (1, 2, 4, 8)


def time_shape(make_fit, shape, steps=40, warmup=16):
    A.m2m_set_launch(*shape)
    fit = make_fit()
    fit.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fit.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fit.close()
    return ms


def search(make_fit, blocks=BLOCKS, tiles=TILES_PER_CU, steps=40, log=sys.stderr, dtype="f32"):
    """Time every shape; returns (best shape, {shape: ms per step})."""
    before = A.m2m_get_launch()
    res = {}
    try:
        for b, t in itertools.product(blocks, tiles):
            if dtype == "f64" and b != 256:
                continue
            ms = time_shape(make_fit, (b, t), steps=steps)
            res[(b, t)] = ms
            if log:
                print(f"[autotune] block={b} tiles/cu={t}: {1e3 * ms:.2f} us/step",
                      file=log, flush=True)
    finally:
        A.m2m_set_launch(*before)
    best = min(res, key=res.get)
    return best, res


def time_batch_shape(fits, shape, steps=40, warmup=16):
    """Mean ms per batched step of ``fits`` with the step kernel in ``shape``."""
    from .batch import Batch
    A.m2m_set_launch(*shape)
    b = Batch(max_fits=len(fits))
    for f in fits:
        if not b.admit(f, warmup + steps + 8):
            raise RuntimeError("batch admission failed")
    b.run(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.run(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for f in fits:
        b.cancel(f)
    b.close()
    return ms


def search_batch(fits, blocks=BLOCKS, tiles=TILES_PER_CU + (6, 12), steps=40, log=sys.stderr):
    """Time every batch shape; returns (best shape, {shape: ms per step})."""
    before = A.m2m_get_launch()
    res = {}
    try:
        for b, t in itertools.product(blocks, tiles):
            ms = time_batch_shape(fits, (b, t), steps=steps)
            res[(b, t)] = ms
            if log:
                print(f"[autotune] batch block={b} tiles/cu={t}: {1e3 * ms:.2f} us/step",
                      file=log, flush=True)
    finally:
        A.m2m_set_launch(*before)
    best = min(res, key=res.get)
    return best, res


def main(argv=None):
    import argparse
    import os

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    from workloads import make_targets, workload

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.workload == 4:
        return main_batch(args)
    wl = workload(args.workload)
    t0 = time.time()
    tp = wl.target_particles(n=1 << 20)
    tf = Fit(wl.potential, wl.layout, wl.params, tp, dtype=wl.state)
    T = make_targets(lambda V, S: tf.observe(V, S), wl)
    tf.close()
    ic = wl.initial_particles()
    dev = {k: torch.as_tensor(v, dtype=torch.float32 if wl.state == "f32" else torch.float64,
                              device="cuda") for k, v in ic.items()}
    print(f"[autotune] {wl.name}: inputs ready in {time.time() - t0:.1f} s", file=sys.stderr,
          flush=True)

    def make_fit():
        f = Fit(wl.potential, wl.layout, wl.params, dev, dtype=wl.state)
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        return f

    best, res = search(make_fit, steps=args.steps, dtype=wl.state)
    out = {"workload": wl.name, "best": list(best), "us_per_step": 1e3 * res[best],
           "all": {f"{b},{t}": 1e3 * ms for (b, t), ms in res.items()}}
    print(json.dumps(out))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)


def main_batch(args):
    """The 64-fit batch of uneven sizes (device-drawn models and targets)."""
    from workloads import make_targets
    from workloads.configs import batch_fits
    from workloads.device import om_model_device
    t0 = time.time()
    fits = []
    for wl in batch_fits(64):
        ic = om_model_device(wl.N, wl.potential, float("inf"), seed=wl.seed * 10 + 1)
        tp = om_model_device(wl.n_target, wl.potential, wl.target_ra, seed=wl.seed * 10 + 2)
        tf = Fit(wl.potential, wl.layout, wl.params, tp, dtype="f32")
        T = make_targets(lambda V, S: tf.observe(V, S), wl)
        tf.close()
        f = Fit(wl.potential, wl.layout, wl.params, ic, dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        fits.append(f)
    print(f"[autotune] batch of {len(fits)} fits, {sum(f.n for f in fits)} particles: inputs "
          f"ready in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    best, res = search_batch(fits, steps=args.steps)
    out = {"workload": "batch64_gh", "best": list(best), "us_per_step": 1e3 * res[best],
           "all": {f"{b},{t}": 1e3 * ms for (b, t), ms in res.items()}}
    print(json.dumps(out))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)
    for f in fits:
        f.close()


if __name__ == "__main__":
    main()
