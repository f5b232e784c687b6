"""Continuous-batching server on the GPU: requests that arrive while others
run are admitted as slots free up (prepared ahead on a thread of their own),
their steps share the batched launches, and every result equals the same fit
run alone (same library, one context) and the FP64 oracle within the weight
tolerance of the FP32 path."""

import sys

import numpy as np
import pytest

from m2m_testlib import cast, oracle_targets, weight_errors
from workloads import make_params, make_potential, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_2355_amd import _abi
    _abi.lib()
    return torch.device("cuda:0")


def test_served_fits_equal_alone_and_oracle(oracle, gpu):
    from paper_1202_2355_amd.fit import Fit
    from paper_1202_2355_amd.serve import Request, Server
    wl = workload(2)
    T = oracle_targets(oracle, wl)
    data = [{"Y": T["Y"], "sigma": T["sigma"], "V_p": T["V_p"], "sigma_p": T["sigma_p"]}]
    # four requests, two slots: the last two wait and are admitted as the
    # first ones finish; two mass-to-light ratios and one dark halo
    spec = [(12_007, 40, 1.0, 0.0), (30_011, 24, 0.8, 0.0), (9_001, 32, 1.25, 10.0),
            (20_021, 16, 1.0, 0.0)]
    reqs, parts = [], {}
    for k, (n, steps, ups, m200) in enumerate(spec):
        pot = make_potential(upsilon=ups, M200=m200, c=8.0 if m200 > 0 else 0.0)
        par = make_params(pot, n_E=wl.params["n_E"], n_x=wl.params["n_x"])
        parts[k] = cast(wl.initial_particles(n=n, seed=60 + k), "f32")
        reqs.append(Request(rid=k, arrival=0.0, potential=pot, params=par, layout=wl.layout, n=n,
                            steps=steps, dataset=0, seed=60 + k))
    _say("serving", [(r.n, r.steps) for r in reqs])

    def model(req):
        return {key: torch.as_tensor(v, dtype=torch.float32, device="cuda")
                for key, v in parts[req.rid].items()}

    srv = Server(data, hbm_budget=1 << 30, max_fits=2, steps_per_launch=8, dtype="f32",
                 keep_weights=True, initial_model=model, preparers=1)
    m = srv.run(reqs, realtime=False)
    srv.close()
    assert m["requests"] == 4
    done = {r.rid: r for r in m["done"]}
    # never more than the two slots in use (a fit holds its slot from the
    # turn it is admitted to the turn it is handed back), so requests 2 and 3
    # could only start after a slot was freed
    for t in range(1, max(r.it_done for r in done.values()) + 1):
        assert sum(r.it_admit <= t <= r.it_done for r in done.values()) <= 2, t
    assert done[2].it_admit > min(done[0].it_done, done[1].it_done)
    for k, r in done.items():
        f = Fit(r.potential, r.layout, r.params, parts[k], dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        f.step(r.steps)
        w_alone = f.weights()
        f.close()
        np.testing.assert_allclose(r.weights, w_alone, rtol=1e-5)
        o = oracle.OracleFit(r.potential, r.layout, r.params, parts[k], T["Y"], T["sigma"],
                             T["V_p"], T["sigma_p"], track_flags=True, band=1e-5, nthreads=8)
        o.step(r.steps)
        u = np.asarray(r.weights, dtype=np.float64) * r.n / r.params["mass"]
        r2, rmax, rall, frac = weight_errors(u, o.arr["u"], o.flag)
        _say("served", k, "rel2", r2, "max(unflagged)", rmax, "flagged", frac)
        assert r2 <= 1e-4 and rmax <= 1e-4
