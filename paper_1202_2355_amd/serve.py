"""Continuous-batching server of M2M fit requests.

A request is a target data set plus a potential (the mass-to-light and halo
scans of the paper's applications, Sec. 6). The server draws the request's
initial particle model on the device, keeps its particles and weights
resident, and admits it into the running batch as soon as a slot and the
HBM budget allow (footprint: particle state plus the library workspace).
The loop thread only admits, enqueues and polls. Each turn admits the
requests that are ready, enqueues a number of batched steps on the batch
stream, then waits only for the turn before (``Batch.poll_lagged``): the fits
that had finished by then leave the batch while the steps just enqueued keep
the GPU busy. Helper threads do the rest: preparing threads prepare waiting
requests (initial model drawn, context created, targets set, on a stream of
each thread's own) as far ahead as the HBM budget and ``max_prepared``
allow, and a finishing thread copies the weights of finished fits to the
host and closes them (the close waits for the steps that could still read
the fit). Latency is measured from
a request's arrival to its weights being on the host.
"""

from __future__ import annotations

import queue
import threading
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
                 max_prepared: int = 8, preparers: int = 4):
        """datasets: list of dicts with Y and sigma (and V_p, sigma_p for
        Gauss-Hermite layouts). initial_model(req) -> dict of device tensors
        (called on a preparing thread, under a stream of the request's own).
        At most ``max_prepared`` prepared requests wait for a slot.
        ``preparers`` threads prepare requests side by side: a preparation is
        a chain of small device steps, each waiting for room beside the
        running batch, so several chains keep up with the batch where one
        does not; with one, requests are admitted in arrival order. The
        preparations' streams should not share a hardware queue with the
        batch's streams, where they would wait behind whole enqueued runs:
        a process that serves sets GPU_MAX_HW_QUEUES (HIP's hardware queues
        per process, 4 by default) to 16 before HIP starts."""
        self.datasets = datasets
        self.budget = int(hbm_budget)
        self.max_fits = max_fits
        self.spl = steps_per_launch
        self.dtype = dtype
        self.keep = keep_weights
        self.initial_model = initial_model
        self.max_prepared = max_prepared
        self.preparers = max(1, int(preparers))
        self.stream = torch.cuda.Stream()
        self.batch = Batch(max_fits=max_fits, hbm_budget=self.budget, stream=self.stream)
        self.live = {}

    def _new_stream(self):
        """A stream for one preparing thread."""
        return torch.cuda.Stream()

    def _make(self, req: Request, st):
        """The request's fit, prepared on the preparing thread's stream ``st``
        (admission orders the batch after it on the device, without waiting
        on the host)."""
        with torch.cuda.stream(st):
            parts = self.initial_model(req)
            fit = Fit(req.potential, req.layout, req.params, parts, dtype=self.dtype, stream=st)
            del parts
            d = self.datasets[req.dataset]
            fit.set_targets(d["Y"], d["sigma"], d.get("V_p"), d.get("sigma_p"))
        return fit

    def run(self, requests, realtime: bool = True, log=None):
        """Serve ``requests`` (sorted by arrival). Returns the metrics dict.
        realtime = False: arrivals on a simulated clock that jumps to the next
        arrival when nothing runs (tests)."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        n_total = len(pending)
        todo, ready, finishing = queue.Queue(), queue.Queue(maxsize=self.max_prepared), queue.Queue()
        cond = threading.Condition()
        stop = threading.Event()
        held = [0]            # bytes of fits prepared, in the batch, or finishing
        errors, done, rejected = [], [], []
        t0 = time.perf_counter()
        sim = [0.0]
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: sim[0])

        def prepare():
            try:
                # one stream per preparing thread, made once: with the
                # hardware queues HIP gives a process, the few streams of the
                # server each get a queue of their own
                st = self._new_stream()
                while True:
                    req = todo.get()
                    if req is None:
                        return
                    need = footprint_bytes(req, self.dtype)
                    with cond:
                        while held[0] + need > self.budget and not stop.is_set():
                            cond.wait(0.05)
                        held[0] += need
                    if stop.is_set():
                        return
                    item = (self._make(req, st), req)
                    while True:
                        try:
                            ready.put(item, timeout=0.05)
                            break
                        except queue.Full:
                            if stop.is_set():
                                item[0].close()
                                return
            except BaseException as e:  # noqa: BLE001 - handed to the loop thread
                errors.append(e)
                stop.set()

        def finish():
            try:
                while True:
                    item = finishing.get()
                    if item is None:
                        return
                    fit, req = item
                    w = fit.weights()
                    req.t_done = clock()
                    if self.keep:
                        req.weights = w
                    fit.close()
                    with cond:
                        held[0] -= footprint_bytes(req, self.dtype)
                        cond.notify_all()
                    done.append(req)
            except BaseException as e:  # noqa: BLE001
                errors.append(e)
                stop.set()

        workers = [threading.Thread(target=prepare, daemon=True) for _ in range(self.preparers)]
        workers.append(threading.Thread(target=finish, daemon=True))
        for w in workers:
            w.start()
        front = deque()       # prepared fits taken from the queue, not yet admitted
        in_prep = 0           # requests handed to the preparing thread, not yet taken
        handed = 0            # fits handed back by the batch
        it = 0
        try:
            while handed + len(rejected) < n_total:
                if errors:
                    raise errors[0]
                it += 1
                now = clock()
                while pending and pending[0].arrival <= now:
                    req = pending.popleft()
                    # a request that can never fit is refused at once, so
                    # that it neither blocks the queue behind it nor keeps
                    # the loop alive
                    why = refusal(req, self.dtype, self.budget)
                    if why:
                        req.rejected = why
                        rejected.append(req)
                        if log:
                            print(f"[serve] refused request {req.rid}: {why}", file=log, flush=True)
                    else:
                        todo.put(req)
                        in_prep += 1
                # prepared fits for the free slots (the rest wait in the
                # bounded queue, which holds the preparing threads back)
                while self.batch.active + len(front) < self.max_fits:
                    try:
                        front.append(ready.get_nowait())
                        in_prep -= 1
                    except queue.Empty:
                        break
                while front and self.batch.active < self.max_fits:
                    fit, req = front[0]
                    if not self.batch.admit(fit, req.steps):
                        break
                    front.popleft()
                    req.t_admit = now
                    req.it_admit = it
                    self.live[id(fit)] = (fit, req)
                if self.batch.active:
                    self.batch.run(self.spl)
                    fin, _ = self.batch.poll_lagged()
                    for fit in fin:
                        _, req = self.live.pop(id(fit))
                        req.it_done = it
                        finishing.put((fit, req))
                        handed += 1
                    if log and fin:
                        print(f"[serve] t={now:.3f}s handed back {handed} active={self.batch.active} "
                              f"ready={len(front) + ready.qsize()} preparing={in_prep}", file=log,
                              flush=True)
                elif not front:
                    # nothing runs: wait for a prepared request, or move the
                    # clock to the next arrival
                    if in_prep:
                        try:
                            front.append(ready.get(timeout=0.05))
                            in_prep -= 1
                        except queue.Empty:
                            pass
                    elif pending:
                        if realtime:
                            time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
                        else:
                            sim[0] = pending[0].arrival
        finally:
            stop.set()
            for _ in range(self.preparers):
                todo.put(None)
            finishing.put(None)
            for w in workers:
                w.join()
            while front:
                front.popleft()[0].close()
            while True:
                try:
                    ready.get_nowait()[0].close()
                except queue.Empty:
                    break
        if errors:
            raise errors[0]
        makespan = clock()
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
        self.batch.close()
