"""Continuous-batching server of M2M fit requests.

A request is a target data set plus a potential (the mass-to-light and halo
scans of the paper's applications, Sec. 6). The server draws the request's
initial particle model on the device, keeps its particles and weights
resident, and admits it into the running batch as soon as a slot and the
HBM budget allow (footprint: particle state plus the library workspace).
Each loop turn admits the requests prepared in the previous turn, enqueues
a number of batched steps on the batch stream, prepares the next waiting
requests on a setup stream while those steps run, then retires the fits
that finished and copies their weights to the host. Latency is measured from
a request's arrival to its weights being on the host.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A
from .batch import Batch
from .fit import Fit


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    potential: object       # workloads.Potential
    params: dict
    layout: dict
    n: int
    steps: int
    dataset: int            # index into the server's target data sets
    seed: int
    t_admit: float = float("nan")
    t_done: float = float("nan")
    it_admit: int = -1      # server loop iteration of admission / completion
    it_done: int = -1
    rejected: str = ""      # why the request was refused (empty: served)
    weights: np.ndarray | None = field(default=None, repr=False)


def footprint_bytes(req: Request, dtype: str) -> int:
    """HBM a request holds while it runs: its particle state and the library
    workspace (0 workspace bytes mark a request the library would refuse)."""
    sz = 8 if dtype == "f64" else 4
    return req.n * 8 * sz + A.m2m_workspace_bytes(req.layout, req.params, req.n, dtype)


def refusal(req: Request, dtype: str, budget: int) -> str:
    """Why a request can never be served under ``budget`` (empty if it can):
    a layout or parameters the library refuses, or a footprint larger than
    the whole budget, which no amount of waiting would free."""
    if A.m2m_workspace_bytes(req.layout, req.params, req.n, dtype) == 0:
        return "invalid layout, parameters or particle count"
    need = footprint_bytes(req, dtype)
    if need > budget:
        return f"footprint {need} bytes exceeds the HBM budget of {budget} bytes"
    return ""


class Server:
    def __init__(self, datasets, hbm_budget: int, max_fits: int = 64, steps_per_launch: int = 64,
                 dtype: str = "f32", keep_weights: bool = False, initial_model=None,
                 max_prepared: int = 4):
        """datasets: list of dicts with Y and sigma (and V_p, sigma_p for
        Gauss-Hermite layouts). initial_model(req) -> dict of device tensors.

        The batch runs on a stream of its own; new requests are prepared
        (initial model drawn, context created, targets set) on a second
        stream while the batch runs, and admitted at the next loop turn."""
        self.datasets = datasets
        self.budget = int(hbm_budget)
        self.max_fits = max_fits
        self.spl = steps_per_launch
        self.dtype = dtype
        self.keep = keep_weights
        self.initial_model = initial_model
        self.max_prepared = max_prepared
        self.stream = torch.cuda.Stream()
        self.setup = torch.cuda.Stream()
        self.batch = Batch(max_fits=max_fits, hbm_budget=self.budget, stream=self.stream)
        self.live = {}
        self.prepared = deque()

    def _prepared_bytes(self) -> int:
        return sum(footprint_bytes(r, self.dtype) for _, r in self.prepared)

    def _prepare(self, req: Request) -> bool:
        """Draw the request's model and create its context on the setup
        stream; False if the HBM budget does not allow it now."""
        need = footprint_bytes(req, self.dtype)
        if self.batch.footprint + self._prepared_bytes() + need > self.budget:
            return False
        with torch.cuda.stream(self.setup):
            parts = self.initial_model(req)
            fit = Fit(req.potential, req.layout, req.params, parts, dtype=self.dtype,
                      stream=self.setup)
            del parts
            d = self.datasets[req.dataset]
            fit.set_targets(d["Y"], d["sigma"], d.get("V_p"), d.get("sigma_p"))
        self.prepared.append((fit, req))
        return True

    def _admit(self, now: float, it: int) -> None:
        while self.prepared and self.batch.active < self.max_fits:
            fit, req = self.prepared[0]
            if not self.batch.admit(fit, req.steps):
                break
            self.prepared.popleft()
            req.t_admit = now
            req.it_admit = it
            self.live[id(fit)] = (fit, req)

    def run(self, requests, realtime: bool = True, log=None):
        """Serve ``requests`` (sorted by arrival). Returns the metrics dict."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = deque()
        done = []
        rejected = []
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else None
        sim_now = 0.0
        it = 0
        while pending or waiting or self.prepared or self.batch.active:
            it += 1
            now = clock() if realtime else sim_now
            while pending and pending[0].arrival <= now:
                req = pending.popleft()
                # a request that can never fit is refused at once, so that it
                # neither blocks the queue behind it nor keeps the loop alive
                why = refusal(req, self.dtype, self.budget)
                if why:
                    req.rejected = why
                    rejected.append(req)
                    if log:
                        print(f"[serve] refused request {req.rid}: {why}", file=log, flush=True)
                else:
                    waiting.append(req)
            self._admit(now, it)
            if self.batch.active:
                self.batch.run(self.spl)
            # while the batch runs: prepare the next requests
            while waiting and len(self.prepared) < self.max_prepared and self._prepare(waiting[0]):
                waiting.popleft()
            if self.batch.active:
                fin, _ = self.batch.poll()
                t = clock() if realtime else now
                for fit in fin:
                    _, req = self.live.pop(id(fit))
                    w = fit.weights()
                    req.t_done = clock() if realtime else t
                    req.it_done = it
                    if self.keep:
                        req.weights = w
                    fit.close()
                    done.append(req)
                if log and fin:
                    print(f"[serve] t={now:.3f}s done={len(done)} active={self.batch.active} "
                          f"prepared={len(self.prepared)} waiting={len(waiting)}", file=log,
                          flush=True)
            elif pending and not self.prepared:
                if realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
                else:
                    sim_now = pending[0].arrival
            if not realtime:
                sim_now = max(sim_now, now)
        makespan = (clock() if realtime else sim_now)
        lat = np.array([r.t_done - r.arrival for r in done])
        work = float(sum(r.n * r.steps for r in done))
        first = min(r.arrival for r in done) if done else 0.0
        last = max(r.t_done for r in done) if done else 0.0
        return {
            "requests": len(done),
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_latency_s": float(lat.mean()) if len(lat) else None,
            "particle_steps": work,
            "particle_steps_per_s": work / max(last - first, 1e-9),
            "makespan_s": makespan,
            "done": done,
            "rejected": rejected,
        }

    def close(self):
        for fit, _ in list(self.live.values()):
            try:
                self.batch.cancel(fit)
            except Exception:
                pass
            fit.close()
        self.live.clear()
        while self.prepared:
            self.prepared.popleft()[0].close()
        self.batch.close()
