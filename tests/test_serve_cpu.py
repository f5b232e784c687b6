"""Host-side admission rules of the serving loop, without a GPU: a request
whose footprint exceeds the whole HBM budget, or that the library refuses,
is rejected at once instead of blocking the queue behind it."""

from workloads import make_params, make_potential, workload


def _req(n, rid=0, **par):
    from paper_1202_2355_amd.serve import Request
    wl = workload(3)
    pot = make_potential(upsilon=1.0, M200=10.0, c=8.0)
    p = dict(make_params(pot, n_E=64, n_x=32), **par)
    return Request(rid=rid, arrival=0.0, potential=pot, params=p, layout=wl.layout, n=n,
                   steps=10, dataset=0, seed=0)


def test_footprint_counts_state_and_workspace():
    from paper_1202_2355_amd import _abi
    from paper_1202_2355_amd.serve import footprint_bytes
    r = _req(100_000)
    ws = _abi.m2m_workspace_bytes(r.layout, r.params, r.n, "f32")
    assert ws > 0
    assert footprint_bytes(r, "f32") == 32 * r.n + ws
    assert footprint_bytes(r, "f64") == 64 * r.n + _abi.m2m_workspace_bytes(
        r.layout, r.params, r.n, "f64")


def test_oversized_and_invalid_requests_are_refused():
    from paper_1202_2355_amd.serve import footprint_bytes, refusal
    small, big = _req(100_000, 0), _req(4_000_000, 1)
    budget = footprint_bytes(small, "f32") * 3
    assert refusal(small, "f32", budget) == ""
    assert "exceeds the HBM budget" in refusal(big, "f32", budget)
    # the same request fits a budget that holds it, however tight
    assert refusal(big, "f32", footprint_bytes(big, "f32")) == ""
    # parameters the library refuses (a grid too large to smooth)
    bad = _req(1000, 2, smooth=1, n_E=64, n_x=64)
    assert "invalid" in refusal(bad, "f32", 1 << 40)


# ---- the serving loop's host logic with a stand-in batch and fits -----------
import threading
import time

import numpy as np
import pytest


class _FakeFit:
    def __init__(self, req, log):
        self.req, self.log = req, log
        self.closed = False

    def weights(self):
        return np.full(self.req.n, 1.0 / self.req.n)

    def close(self):
        assert not self.closed
        self.closed = True
        self.log.append(("close", self.req.rid))


class _FakeBatch:
    """Steps every admitted fit by steps_per_launch per run; hands fits back
    one run after the run in which they finished (as m2m_batch_poll_lagged)."""

    def __init__(self, max_fits, budget, footprint):
        self.max_fits, self.budget, self.fp = max_fits, budget, footprint
        self.left, self.finished_in, self.runs = {}, {}, 0

    @property
    def active(self):
        return len(self.left)

    @property
    def footprint(self):
        return sum(self.fp(f.req) for f in self.left)

    def admit(self, fit, n):
        if self.active >= self.max_fits or self.footprint + self.fp(fit.req) > self.budget:
            return False
        self.left[fit] = n
        return True

    def run(self, spl):
        self.runs += 1
        for f in self.left:
            if self.left[f] > 0:
                self.left[f] = max(0, self.left[f] - spl)
                if self.left[f] == 0:
                    self.finished_in[f] = self.runs

    def poll_lagged(self):
        done = [f for f in self.left if f in self.finished_in and self.finished_in[f] <= self.runs - 1]
        for f in done:
            del self.left[f]
        return done, self.active


def _fake_server(budget, max_fits, preparers, fail_rid=None):
    from paper_1202_2355_amd.serve import Server, footprint_bytes
    log, lock = [], threading.Lock()
    srv = Server.__new__(Server)
    srv.datasets, srv.budget, srv.max_fits, srv.spl = [None], budget, max_fits, 16
    srv.dtype, srv.keep, srv.initial_model, srv.max_prepared = "f32", False, None, 3
    srv.preparers, srv.live = preparers, {}
    srv.batch = _FakeBatch(max_fits, budget, lambda r: footprint_bytes(r, "f32"))
    held = [0, 0]   # bytes of open fits, the most seen

    def make(req, st):
        if req.rid == fail_rid:
            raise RuntimeError("preparation failed")
        time.sleep(0.002)
        with lock:
            held[0] += footprint_bytes(req, "f32")
            held[1] = max(held[1], held[0])
        f = _FakeFit(req, log)
        orig = f.close

        def close():
            with lock:
                held[0] -= footprint_bytes(req, "f32")
            orig()
        f.close = close
        return f
    srv._new_stream = lambda: None
    srv._make = make
    return srv, log, held


def test_server_loop_serves_every_request_within_slots_and_budget():
    from paper_1202_2355_amd.serve import footprint_bytes
    reqs = [_req(n, rid=k) for k, n in enumerate(np.random.default_rng(3).integers(1e5, 2e6, 30))]
    for k, r in enumerate(reqs):
        r.steps = 16 * (1 + k % 5)
        r.arrival = 0.001 * k
    budget = 5 * max(footprint_bytes(r, "f32") for r in reqs)
    srv, log, held = _fake_server(budget, max_fits=4, preparers=3)
    m = srv.run(reqs, realtime=False)
    assert m["requests"] == 30 and not m["rejected"]
    assert held[1] <= budget and held[0] == 0
    assert sorted(r for kind, r in log if kind == "close") == list(range(30))
    done = m["done"]
    last = max(r.it_done for r in done)
    for t in range(1, last + 1):
        assert sum(r.it_admit <= t <= r.it_done for r in done) <= 4, t
    # a fit of s steps is handed back one run after the run that finished it
    for r in done:
        assert r.it_done - r.it_admit >= -(-r.steps // 16)


def test_server_loop_refuses_what_never_fits_and_keeps_serving():
    from paper_1202_2355_amd.serve import footprint_bytes
    small = [_req(100_000, rid=k) for k in range(4)]
    big = _req(4_000_000, rid=9)
    budget = 2 * footprint_bytes(small[0], "f32")
    srv, log, held = _fake_server(budget, max_fits=2, preparers=2)
    m = srv.run([small[0], big] + small[1:], realtime=False)
    assert [r.rid for r in m["rejected"]] == [9]
    assert sorted(r.rid for r in m["done"]) == [0, 1, 2, 3]


def test_server_loop_reports_a_failed_preparation():
    srv, log, held = _fake_server(1 << 40, max_fits=2, preparers=2, fail_rid=2)
    t = time.time()
    with pytest.raises(RuntimeError, match="preparation failed"):
        srv.run([_req(100_000, rid=k) for k in range(5)], realtime=False)
    assert time.time() - t < 30
