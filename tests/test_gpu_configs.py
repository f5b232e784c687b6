"""GPU parity at the benchmarked configurations (run on an MI355X), scaled
only in particle count and steps where the FP64 oracle must follow:

* the 8-million-particle LOSVD configuration (NFW + Hernquist, 2610
  observables, 64 x 32 prior grid) in its benchmark launch shape, over two
  in-step prior refreshes;
* the Gauss-Hermite configuration for 200 FP32 steps;
* the 64-fit batch: fits drawn as it draws them (own mass-to-light ratio
  and NFW concentration, uneven N), in its benchmark launch shape, each fit
  against the oracle and against itself run alone;
* the served LOSVD requests in NFW potentials, FP32 and FP64 state;
* the finalize hand-over in a batch where prior refreshes come every other
  step (and with the self-consistent potential rebuilt every other step):
  every fit's counters, chi^2 history and weights as when run alone.

Criteria as in the other parity tests: weights ||du||/||u|| <= 1e-4 and
max |du|/u <= 1e-4 over particles the oracle never saw near an edge (FP32
state), 1e-10 (FP64 state); chi^2 histories rtol 1e-4 (FP32), 1e-9 (FP64).
"""

import struct
import sys

import numpy as np
import pytest

from m2m_testlib import cast, oracle_targets, weight_errors
from workloads import floor_model_noise, make_targets, with_scf, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def Fit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_2355_amd import _abi
    _abi.lib()
    from paper_1202_2355_amd.fit import Fit
    return Fit


def _tuned(mode, wl):
    """The package's tuned launch parameters of the workload's class (as the
    benchmark runs it), restored on exit."""
    from paper_1202_2355_amd import tuning
    return tuning.tuned(mode, wl.state, wl.layout, wl.N)


def _counters(fit):
    """(kstep, tstep) of a fit from its checkpoint: correction steps and
    steps of any kind taken."""
    blob = fit.get_state()
    # header: magic, version (u32), n (i64), 8 x i32; then the fit state
    # starting with kstep, tstep (i64)
    return struct.unpack_from("<qq", blob, 48)


def _run_pair(oracle, Fit, wl, parts, T, dtype, band, nthreads=16):
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype)
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, T["Y"], T["sigma"], T["V_p"],
                         T["sigma_p"], track_flags=True, band=band, nthreads=nthreads)
    return f, o


def test_losvd_nfw_configuration_over_two_refreshes(oracle, Fit):
    """The LOSVD configuration (Hernquist + NFW potential, 50 radial bins +
    40 annuli x 64 velocity bins, 64 x 32 prior grid refreshed every 25
    steps) with 200 003 particles in its benchmark launch shape, 60 FP32
    steps: two in-step refreshes and their assignments."""
    wl = workload(3)
    n, steps = 200_003, 60
    T = oracle_targets(oracle, wl)
    parts = cast(wl.initial_particles(n=n, seed=301), "f32")
    with _tuned("single", wl) as shape:
        _say("losvd/nfw", n, steps, "launch", shape)
        f, o = _run_pair(oracle, Fit, wl, parts, T, "f32", 1e-5)
        f.step(steps)
        hist_g = f.chi2_history(steps)
        st = f.particles()
        ks = _counters(f)
        f.close()
    hist_o = o.step(steps)
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("losvd/nfw: rel2", r2, "max(unflagged)", rmax, "max(all)", rall, "flagged", frac)
    assert ks == (steps, steps)
    assert r2 <= 1e-4 and rmax <= 1e-4
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-4)
    # the priors of the second refresh: a cell's mean moves when a particle
    # near an edge is binned on the other side, so compare them as a whole:
    # almost every particle has the oracle's prior
    rel = np.abs(st["uh"] / o.arr["uhat"] - 1.0)
    _say("losvd/nfw priors: median", float(np.median(rel)), "fraction > 1e-4",
         float(np.mean(rel > 1e-4)))
    assert np.median(rel) < 1e-5 and np.mean(rel > 1e-4) < 0.02


def test_gauss_hermite_configuration_200_steps(oracle, Fit):
    """The Gauss-Hermite configuration (40 radial bins + 30 annuli x h1..h4,
    50 x 20 prior grid) at its full 10^6 particles in its benchmark launch
    shape: 200 FP32 steps, eight refreshes. (At 10^5 particles one particle
    binned on the other side of an edge moves the residual of a faint annulus
    enough to shift every particle of it by about 1e-4 over the run; the
    shift falls as 1/sqrt(N).)"""
    wl = workload(2)
    n, steps = wl.N, 200
    T = oracle_targets(oracle, wl)
    parts = cast(wl.initial_particles(n=n, seed=302), "f32")
    with _tuned("single", wl) as shape:
        _say("gh", n, steps, "launch", shape)
        f, o = _run_pair(oracle, Fit, wl, parts, T, "f32", 1e-5)
        f.step(steps)
        hist_g = f.chi2_history(steps)
        u = f.particles()["u"]
        f.close()
    hist_o = o.step(steps)
    r2, rmax, rall, frac = weight_errors(u, o.arr["u"], o.flag)
    _say("gh 200 steps: rel2", r2, "max(unflagged)", rmax, "max(all)", rall, "flagged", frac)
    assert r2 <= 1e-4 and rmax <= 1e-4
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-4)


def _batch_members(n_fits, scale, seed=4):
    """Fits drawn as the 64-fit batch draws them (the first n_fits of its
    draw), their particle counts divided by ``scale``."""
    from workloads.configs import batch_fits
    fits = batch_fits(n_fits=64, seed=seed)[:n_fits]
    return [wl.with_(N=max(64, int(wl.N // scale))) for wl in fits]


def test_batched_configuration_in_its_launch_shape(oracle, Fit):
    """Ten fits of the 64-fit batch (own mass-to-light ratio and NFW
    concentration, N from 4 100 to 130 000 after dividing by 16) in the
    batch's benchmark launch shape: each fit against the oracle and against
    the same fit run alone, 50 steps (two refreshes)."""
    from paper_1202_2355_amd.batch import Batch
    members = _batch_members(10, 16)
    full = _batch_members(10, 1)
    steps = 50
    data = []
    for wl in members:
        T = oracle_targets(oracle, wl, n_target=1 << 16)
        parts = cast(wl.initial_particles(), "f32")
        data.append((T, parts))
    alone = []
    for wl, wf, (T, parts) in zip(members, full, data):
        # alone: in the tuned shape of a single fit of the batch member's size
        with _tuned("single", wf):
            f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        f.step(steps)
        alone.append((f.particles()["u"], f.chi2_history(steps)))
        f.close()
    with _tuned("batch", members[0]) as shape:
        _say("batch", [wl.N for wl in members], "launch", shape)
        b = Batch(max_fits=len(members))
        fits = []
        for wl, (T, parts) in zip(members, data):
            f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f32")
            f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
            assert b.admit(f, steps)
            fits.append(f)
        done = b.run_to_completion(steps_per_launch=16, max_steps=10 * steps)
        assert len(done) == len(members)
        got = [(f.particles()["u"], f.chi2_history(steps), _counters(f)) for f in fits]
        for f in fits:
            f.close()
        b.close()
    for k, (wl, (T, parts)) in enumerate(zip(members, data)):
        u, hist, ks = got[k]
        assert ks == (steps, steps)
        np.testing.assert_allclose(u, alone[k][0], rtol=1e-5)
        np.testing.assert_allclose(hist, alone[k][1], rtol=1e-6)
        o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, T["Y"], T["sigma"],
                             T["V_p"], T["sigma_p"], track_flags=True, band=1e-5, nthreads=16)
        hist_o = o.step(steps)
        r2, rmax, rall, frac = weight_errors(u, o.arr["u"], o.flag)
        _say("batch fit", k, "N", wl.N, "upsilon", wl.potential.upsilon, "c", wl.potential.c,
             "rel2", r2, "max(unflagged)", rmax, "flagged", frac)
        assert r2 <= 1e-4 and rmax <= 1e-4
        np.testing.assert_allclose(hist, hist_o, rtol=1e-4)


def test_full_size_batch_across_a_refresh(oracle, Fit):
    """The benchmarked batch itself: all 64 fits at their full particle
    counts (3.6e7 in all, drawn on the device as the benchmark draws them),
    oracle targets, the batch's tuned launch, 26 steps (the first in-step
    prior refresh). Every fit ends with 26 steps taken and a finite chi^2;
    the smallest, the median and the largest fit match the oracle run alone
    from the same initial state (weights within 1e-4)."""
    from paper_1202_2355_amd.batch import Batch
    from workloads.configs import batch_fits
    from workloads.device import om_model_device
    steps = 26
    fits_wl = batch_fits(64)
    sizes = [wl.N for wl in fits_wl]
    order = sorted(range(len(fits_wl)), key=lambda k: sizes[k])
    sample = sorted({order[0], order[len(order) // 2], order[-1]})
    _say("full-size batch", sum(sizes), "particles; oracle on fits", [sizes[k] for k in sample])
    fits, Ts, ics = [], [], {}
    for k, wl in enumerate(fits_wl):
        T = oracle_targets(oracle, wl, n_target=1 << 15, nthreads=16)
        ic = om_model_device(wl.N, wl.potential, float("inf"), seed=wl.seed * 10 + 1)
        f = Fit(wl.potential, wl.layout, wl.params, ic, dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        if k in sample:
            st = f.particles()
            ics[k] = {q: st[q] for q in ("x", "y", "z", "vx", "vy", "vz")}
        del ic
        fits.append(f)
        Ts.append(T)
    with _tuned("batch", fits_wl[0]) as shape:
        _say("batch launch", shape)
        b = Batch(max_fits=len(fits))
        for f in fits:
            assert b.admit(f, steps)
        done = b.run_to_completion(steps_per_launch=16, max_steps=10 * steps)
        assert len(done) == len(fits)
        got = {}
        for k, f in enumerate(fits):
            assert _counters(f) == (steps, steps), k
            assert np.isfinite(f.observables()["chi2"]), k
            if k in sample:
                got[k] = f.particles()["u"]
        for f in fits:
            f.close()
        b.close()
    for k in sample:
        wl, T = fits_wl[k], Ts[k]
        o = oracle.OracleFit(wl.potential, wl.layout, wl.params, ics[k], T["Y"], T["sigma"],
                             T["V_p"], T["sigma_p"], track_flags=True, band=1e-5, nthreads=16)
        o.step(steps)
        r2, rmax, rall, frac = weight_errors(got[k], o.arr["u"], o.flag)
        _say("full-size batch fit", k, "N", wl.N, "rel2", r2, "max(unflagged)", rmax,
             "flagged", frac)
        assert r2 <= 1e-4 and rmax <= 1e-4


@pytest.mark.parametrize("scf", [False, True])
def test_batch_finalize_hand_over_with_frequent_refreshes(oracle, Fit, scf):
    """Sixteen LOSVD fits (41 observable and 32 cell finalize jobs each), the
    prior grid refreshed every other step (with the self-consistent
    potential also rebuilt every other step): each fit ends with the counters
    of its steps and the chi^2 history and weights of the same fit run
    alone. A finalize job that read a fit's counters after another job had
    ended its step would take the wrong refresh schedule."""
    from paper_1202_2355_amd.batch import Batch
    base = workload(3)
    if scf:
        base = with_scf(base, l_max=2, n_nodes=16, every=2)
    # a strong entropy term, so that a refresh taken at the wrong step shows
    # in the weights
    par = dict(base.params, prior_every=2, mu=1.0)
    wl = base.with_(params=par)
    sizes = [3_001 + 1_777 * k for k in range(16)]
    steps = 14
    _say("hand-over", "scf" if scf else "analytic", sizes)
    tp = wl.target_particles(n=1 << 16)
    ones = np.ones(tp["x"].size)
    T = make_targets(lambda V, S: oracle.deposit(tp, ones, wl.layout, V_p=V, sigma_p=S,
                                                 nthreads=16), wl)
    # errors no smaller than the particle noise of the smallest fit (as the
    # serving data sets), so that every fit stays finite
    T["sigma"] = floor_model_noise(T["Y_true"], T["sigma"], min(sizes))
    parts = [cast(wl.initial_particles(n=n, seed=400 + k), "f32") for k, n in enumerate(sizes)]
    alone = []
    for p in parts:
        f = Fit(wl.potential, wl.layout, wl.params, p, dtype="f32")
        f.set_targets(T["Y"], T["sigma"])
        f.step(steps)
        alone.append((f.particles()["u"], f.chi2_history(steps), _counters(f)))
        f.close()
    b = Batch(max_fits=16)
    fits = []
    for p in parts:
        f = Fit(wl.potential, wl.layout, wl.params, p, dtype="f32")
        f.set_targets(T["Y"], T["sigma"])
        assert b.admit(f, steps)
        fits.append(f)
    done = b.run_to_completion(steps_per_launch=4, max_steps=10 * steps)
    assert len(done) == 16
    for k, f in enumerate(fits):
        ks = _counters(f)
        assert ks == alone[k][2] == (steps, steps), (k, ks, alone[k][2])
        np.testing.assert_allclose(f.chi2_history(steps), alone[k][1], rtol=1e-6)
        np.testing.assert_allclose(f.particles()["u"], alone[k][0], rtol=1e-5)
        f.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_served_losvd_requests_in_nfw_potentials(oracle, Fit, dtype):
    """Four requests of the serving trace's kind (LOSVD layout of 2610
    observables, Hernquist + NFW potentials with their own mass-to-light
    ratio and concentration, noise 1-5 %), scaled to 9 000-30 000 particles
    and 40-60 steps, through the server with two slots, in FP32 and FP64
    particle state: each result against the oracle (and the later requests
    admitted as slots free up)."""
    from paper_1202_2355_amd.serve import Request, Server
    from workloads.configs import serve_trace
    _, trace = serve_trace(n_requests=4, rate=20.0, seed=5, state=dtype)
    spec = [(12_007, 60), (30_011, 40), (9_001, 52), (20_021, 44)]
    reqs, parts, data = [], {}, []
    for k, (wl, (n, steps)) in enumerate(zip(trace, spec)):
        T = oracle_targets(oracle, wl, n_target=1 << 17)
        # errors floored at the particle noise of the smallest request, as
        # the serving data sets are
        data.append({"Y": T["Y"], "sigma": floor_model_noise(T["Y_true"], T["sigma"], 9_001)})
        parts[k] = cast(wl.initial_particles(n=n, seed=500 + k), dtype)
        reqs.append(Request(rid=k, arrival=0.0, potential=wl.potential, params=wl.params,
                            layout=wl.layout, n=n, steps=steps, dataset=k, seed=500 + k))
    _say("serving losvd", dtype, [(r.n, r.steps) for r in reqs])
    tdt = torch.float32 if dtype == "f32" else torch.float64

    def model(req):
        return {key: torch.as_tensor(v, dtype=tdt, device="cuda") for key, v in parts[req.rid].items()}

    srv = Server(data, hbm_budget=1 << 30, max_fits=2, steps_per_launch=8, dtype=dtype,
                 keep_weights=True, initial_model=model, preparers=1)
    m = srv.run(reqs, realtime=False)
    srv.close()
    assert m["requests"] == 4 and not m["rejected"]
    done = {r.rid: r for r in m["done"]}
    for t in range(1, max(r.it_done for r in done.values()) + 1):
        assert sum(r.it_admit <= t <= r.it_done for r in done.values()) <= 2, t
    assert done[2].it_admit > min(done[0].it_done, done[1].it_done)
    for k, r in done.items():
        d = data[k]
        band = 1e-5 if dtype == "f32" else 1e-12
        o = oracle.OracleFit(r.potential, r.layout, r.params, parts[k], d["Y"], d["sigma"],
                             track_flags=True, band=band, nthreads=16)
        o.step(r.steps)
        u = np.asarray(r.weights, dtype=np.float64) * r.n / r.params["mass"]
        r2, rmax, rall, frac = weight_errors(u, o.arr["u"], o.flag)
        _say("served losvd", dtype, k, "rel2", r2, "max(unflagged)", rmax, "flagged", frac)
        tol = 1e-4 if dtype == "f32" else 1e-10
        assert r2 <= tol and rmax <= tol
