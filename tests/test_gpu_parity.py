"""GPU parity of the HIP path against the FP64 oracle (run on an MI355X).

Criteria
* observables of one state: |y_gpu - y_ora| <= rel * sum_i |w_i K_ij|
  + sum over particles within 4 float32 ulps of an edge of |w_i K_ij|,
  rel = 1e-5 for FP32 particle state, 1e-12 for FP64;
* weights after independent runs from the same initial state:
  ||u_gpu - u_ora|| / ||u_ora|| <= 1e-4 and max_i |u_gpu/u_ora - 1| <= 1e-4 for
  every particle the oracle never saw within 1e-5 r of an observable or cell
  edge (FP32); 1e-10 for FP64 state, whose only differences are summation
  order and last-bit differences of the elementary functions.
"""

import sys

import numpy as np
import pytest

from m2m_testlib import (BAND_F32, BAND_F64, assert_observables, assert_priors_within, cast,
                         oracle_targets, prior_bounds, random_weights, weight_errors)
from workloads import workload

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


@pytest.fixture(scope="module")
def Fit(gpu):
    from paper_1202_2355_amd.fit import Fit
    return Fit


def _gh_centres(n_R, seed=3):
    g = np.random.default_rng(seed)
    return g.uniform(-0.05, 0.05, n_R), g.uniform(0.25, 0.6, n_R)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("wlid", [1, 2, 3])
def test_observe_one_state(oracle, Fit, wlid, dtype):
    wl = workload(wlid)
    n = 50_003
    _say("observe", wl.name, dtype, n)
    parts = cast(wl.initial_particles(n=n, seed=100 + wlid), dtype)
    u = cast({"u": random_weights(n, 7)}, dtype)["u"]
    V, S = _gh_centres(wl.layout["n_R"])
    V, S = cast({"V": V, "S": S}, dtype).values()
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype, u=u)
    y = f.observe(V, S)
    band = BAND_F32 if dtype == "f32" else BAND_F64
    yo, ya, yb = oracle.deposit(parts, u, wl.layout, mass=wl.params["mass"], V_p=V, sigma_p=S,
                                band=band, nthreads=8, with_abs=True)
    worst = assert_observables(y, yo, ya, yb, 1e-5 if dtype == "f32" else 1e-12, wl.name)
    _say("observe", wl.name, dtype, "max |dy|/sum|wK| =", worst)
    f.close()


def _run_pair(oracle, Fit, wl, n, steps, dtype, band, seed=11):
    T = oracle_targets(oracle, wl)
    parts = cast(wl.initial_particles(n=n, seed=seed), dtype)
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype)
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, T["Y"], T["sigma"], T["V_p"],
                         T["sigma_p"], track_flags=True, band=band, nthreads=8)
    return T, parts, f, o


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_initial_residuals_and_one_step(oracle, Fit, dtype):
    wl = workload(2)
    n = 30_001
    _say("one step", wl.name, dtype, n)
    T, parts, f, o = _run_pair(oracle, Fit, wl, n, 1, dtype, 1e-5)
    ob0 = f.observables()
    rel = 1e-5 if dtype == "f32" else 1e-12
    np.testing.assert_allclose(ob0["ytilde"], o.ytilde, rtol=0, atol=1e-4 * np.abs(o.ytilde).max())
    assert ob0["chi2"] == pytest.approx(o.chi2, rel=1e-3 if dtype == "f32" else 1e-10)
    f.step(1)
    o.step(1)
    st = f.particles()
    ob1 = f.observables()
    # per-step observables: the oracle deposits the GPU's own state of step 1
    band = BAND_F32 if dtype == "f32" else BAND_F64
    yo, ya, yb = oracle.deposit(st, st["u"], wl.layout, mass=1.0, V_p=T["V_p"],
                                sigma_p=T["sigma_p"], band=band, nthreads=8, with_abs=True)
    assert_observables(ob1["y"], yo, ya, yb, rel, "step-1 deposit")
    r2, rmax, _, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("one step", dtype, "weights rel2", r2, "max", rmax, "flagged", frac)
    assert r2 <= (1e-6 if dtype == "f32" else 1e-13)
    assert rmax <= (1e-6 if dtype == "f32" else 1e-12)
    f.close()


@pytest.mark.parametrize("mode", ["f64", "f32c"])
def test_run_fp32_matches_oracle_200_steps(oracle, Fit, mode):
    """Workload 1 with FP32 particle state: weights after 200 steps, with
    FP64 and with compensated FP32 in-tile deposit sums."""
    from paper_1202_2355_amd import _abi
    wl = workload(1)
    n = 20_003
    _say("run fp32", wl.name, n, "deposit", mode)
    _abi.m2m_set_deposit_mode(mode)
    T, parts, f, o = _run_pair(oracle, Fit, wl, n, 200, "f32", 1e-5)
    _abi.m2m_set_deposit_mode("f64")
    f.step(200)
    hist_o = o.step(200)
    hist_g = f.chi2_history(200)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("run fp32 200 steps: rel2", r2, "max(unflagged)", rmax, "max(all)", rall, "flagged", frac)
    assert r2 <= 1e-4
    assert rmax <= 1e-4
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-4)
    f.close()


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_interleaved_tiles_match_oracle_and_contiguous_tiles(oracle, Fit, block):
    """Tiles of interleaved chunks (the mapping the library picks for single
    fits whose state exceeds the memory-side cache), forced on a fit of
    workload 2's layout at every block size (FP32 state, the one it is built
    for), one tile per compute unit, so that every tile takes several chunks
    and the last chunk is ragged: weights and the chi^2 history after 60
    steps (two prior refreshes) against the oracle, and the weights against
    the same fit with contiguous tiles (rounding order only)."""
    from paper_1202_2355_amd import _abi, tuning
    wl = workload(2)
    n = 600_011
    steps = 60
    _say("interleaved tiles, block", block, "n", n)
    before = tuning.current()
    u = {}
    try:
        tuning.apply(dict(before, block=block, tiles_per_cu=1))
        for il in (1, 0):
            _abi.m2m_set_interleave(il)
            T, parts, f, o = _run_pair(oracle, Fit, wl, n, steps, "f32", 1e-5)
            f.step(steps)
            hist_g = f.chi2_history(steps)
            u[il] = f.particles()["u"]
            f.close()
            if il == 1:
                hist_o = o.step(steps)
                r2, rmax, rall, frac = weight_errors(u[1], o.arr["u"], o.flag)
                _say("interleaved: rel2", r2, "max(unflagged)", rmax, "max(all)", rall,
                     "flagged", frac)
                assert r2 <= 1e-4 and rmax <= 1e-4
                np.testing.assert_allclose(hist_g, hist_o, rtol=1e-4)
    finally:
        _abi.m2m_set_interleave(-1)
        tuning.apply(before)
    np.testing.assert_allclose(u[1], u[0], rtol=1e-5)


@pytest.mark.parametrize("n", [1, 1_023, 70_001])
def test_interleaved_tiles_with_empty_tiles(oracle, Fit, n):
    """Interleaved tiles when the fit has fewer chunks than tiles (up to 256
    tiles of 1024 threads): most tiles take no particle and deposit nothing.
    One particle, one short chunk, and 69 chunks with a ragged last one, FP32
    state, workload 1's layout with a prior refresh every 4 steps and the
    fit's own initial observables as targets (5 % errors; a few particles
    against a full model's targets would overflow the weights): weights
    after 12 steps against the oracle."""
    from paper_1202_2355_amd import _abi, tuning
    wl = workload(1)
    wl = wl.with_(params=dict(wl.params, prior_every=4))
    parts = cast(wl.initial_particles(n=n, seed=12 + n), "f32")
    Y = oracle.deposit(parts, np.ones(n), wl.layout, mass=wl.params["mass"])
    sig = 0.05 * np.abs(Y) + 1e-3 * np.abs(Y).max() + 1e-12
    _say("interleaved tiles, empty tiles, n", n)
    before = tuning.current()
    try:
        tuning.apply(dict(before, block=1024, tiles_per_cu=1))
        _abi.m2m_set_interleave(1)
        f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f32")
    finally:
        _abi.m2m_set_interleave(-1)
        tuning.apply(before)
    f.set_targets(Y, sig)
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, Y, sig, None, None,
                         track_flags=True, band=1e-5, nthreads=8)
    f.step(12)
    o.step(12)
    st = f.particles()
    f.close()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("empty tiles: rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    assert r2 <= 1e-4 and rmax <= 1e-4


@pytest.mark.parametrize("case", ["alm_f32", "v2_f64"])
def test_interleave_request_on_fits_built_without_it(oracle, Fit, case):
    """Interleaving forced on fits whose step kernel is built with contiguous
    tiles only (a_lm density observables; FP64 state): the request is
    ignored and the fit matches the oracle as always (weights after 12 steps
    with three prior refreshes)."""
    from paper_1202_2355_amd import _abi, tuning
    from workloads import with_alm
    if case == "alm_f32":
        wl, dtype, n, band, tol = with_alm(workload(1), n_mesh=20, l_max=2), "f32", 30_011, 1e-5, 1e-4
    else:
        wl, dtype, n, band, tol = workload(1), "f64", 30_011, 1e-12, 1e-10
    wl = wl.with_(params=dict(wl.params, prior_every=4))
    parts = cast(wl.initial_particles(n=n, seed=14), dtype)
    Y = oracle.deposit(parts, np.ones(n), wl.layout, mass=wl.params["mass"])
    sig = 0.05 * np.abs(Y) + 1e-3 * np.abs(Y).max() + 1e-12
    _say("interleave requested on", case, n)
    before = tuning.current()
    try:
        tuning.apply(dict(before, block=1024, tiles_per_cu=1))
        _abi.m2m_set_interleave(1)
        f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype)
    finally:
        _abi.m2m_set_interleave(-1)
        tuning.apply(before)
    f.set_targets(Y, sig)
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, Y, sig, None, None,
                         track_flags=True, band=band, nthreads=8)
    f.step(12)
    o.step(12)
    st = f.particles()
    f.close()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say(case, "rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    assert r2 <= tol and rmax <= tol


def test_run_fp64_matches_oracle_200_steps(oracle, Fit):
    """Workload 1 as specified (FP64 particle state): weights after 200 steps."""
    wl = workload(1)
    n = 20_003
    _say("run fp64", wl.name, n)
    T, parts, f, o = _run_pair(oracle, Fit, wl, n, 200, "f64", 1e-12)
    f.step(200)
    o.step(200)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("run fp64 200 steps: rel2", r2, "max(unflagged)", rmax, "max(all)", rall, "flagged", frac)
    assert r2 <= 1e-10
    assert rmax <= 1e-10
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(st[k], o.arr[k], rtol=0, atol=1e-9)
    ob = f.observables()
    np.testing.assert_allclose(ob["ytilde"], o.ytilde, rtol=1e-10, atol=1e-15)
    assert ob["chi2"] == pytest.approx(o.chi2, rel=1e-9)
    f.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_prior_refresh_matches_oracle(oracle, Fit, dtype):
    wl = workload(3)
    n = 40_001
    _say("priors", wl.name, dtype, n)
    parts = cast(wl.initial_particles(n=n, seed=5), dtype)
    u = cast({"u": random_weights(n, 9, spread=0.5)}, dtype)["u"]
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype, u=u)
    f.update_priors()
    uh = f.particles()["uh"]
    f.close()
    from m2m_testlib import assert_priors_within, prior_bounds
    band = 1e-5 if dtype == "f32" else 1e-12
    o = _oracle_priors(oracle, wl, wl.params, parts, u, band)
    # every particle: its prior within the bounds that the particles near a
    # cell edge (either side) leave on its cell's mean
    lo, hi = prior_bounds(oracle, wl.potential, wl.params, parts, u, o.flag, band)
    np.testing.assert_allclose(o.arr["uhat"], np.clip(o.arr["uhat"], lo, hi), rtol=1e-13)
    unbounded = assert_priors_within(uh, lo, hi, 1e-6 if dtype == "f32" else 1e-13, "priors")
    _say("priors", dtype, "flagged", float((o.flag != 0).mean()), "unbounded", unbounded)
    assert unbounded < 1e-3


def test_batch_equals_alone(oracle, Fit):
    from paper_1202_2355_amd.batch import Batch
    wl = workload(2)
    T = oracle_targets(oracle, wl)
    sizes = [9_001, 33_333, 70_007]
    steps = [40, 25, 40]
    _say("batch vs alone", sizes, steps)
    alone = []
    parts = [cast(wl.initial_particles(n=n, seed=20 + k), "f32") for k, n in enumerate(sizes)]
    for k, n in enumerate(sizes):
        f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        f.step(steps[k])
        alone.append((f.particles()["u"], f.observables()))
        f.close()
    fits = []
    b = Batch(max_fits=8)
    for k, n in enumerate(sizes):
        f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        b.admit(f, steps[k])
        fits.append(f)
    done = b.run_to_completion(steps_per_launch=16)
    assert len(done) == 3
    for k, f in enumerate(fits):
        u = f.particles()["u"]
        ob = f.observables()
        # same tiles of FP64-reduced, compensated sums: the runs differ only by
        # the order of atomic adds, i.e. by last-bit roundings of FP32 state
        np.testing.assert_allclose(u, alone[k][0], rtol=1e-5)
        yt = alone[k][1]["ytilde"]
        assert np.abs(ob["ytilde"] - yt).max() <= 1e-6 * np.abs(yt).max()
        f.close()
    b.close()


def test_checkpoint_resume(oracle, Fit):
    wl = workload(2)
    T = oracle_targets(oracle, wl)
    n = 25_003
    _say("checkpoint", n)
    parts = cast(wl.initial_particles(n=n, seed=31), "f32")
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f32")
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    f.step(30)
    blob = f.get_state()
    mid = f.particles()
    f.step(30)
    end = f.particles()
    g = Fit(wl.potential, wl.layout, wl.params, {k: mid[k] for k in ("x", "y", "z", "vx", "vy", "vz")},
            dtype="f32", u=mid["u"], u_prior=mid["uh"])
    g.set_state(blob)
    g.step(30)
    end2 = g.particles()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(end2[k], end[k], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(end2["u"], end["u"], rtol=1e-5)
    yt, yt2 = f.observables()["ytilde"], g.observables()["ytilde"]
    assert np.abs(yt2 - yt).max() <= 1e-6 * np.abs(yt).max()
    assert g.chi2_history(60).size == 60   # history carried over: 30 + 30 steps
    f.close()
    g.close()


@pytest.mark.parametrize("mode", ["f32c", "f64"])
@pytest.mark.parametrize("n", [4_000_003, 200_001])
def test_compensated_deposit_is_exact_to_fp64_rounding(oracle, Fit, n, mode):
    """All particles in one radial bin: FP32 in-tile sums that carry their
    exact rounding errors (TwoSum on the LDS atomics), and FP64 in-tile sums,
    both give the FP64 sum of the FP32 contributions far below FP32
    accuracy."""
    from paper_1202_2355_amd import _abi
    from workloads import make_layout, make_params, make_potential
    _abi.m2m_set_deposit_mode(mode)
    pot = make_potential()
    g = np.random.default_rng(4)
    r = g.uniform(1.0, 2.0, n)
    parts = {"x": r, "y": np.zeros(n), "z": np.zeros(n), "vx": np.zeros(n), "vy": np.zeros(n),
             "vz": np.zeros(n)}
    parts = cast(parts, "f32")
    u = cast({"u": g.uniform(0.5, 1.5, n)}, "f32")["u"]
    lay = make_layout(1, 0.5, 4.0)
    par = make_params(pot)
    _say("compensated deposit", n)
    f = Fit(pot, lay, par, parts, dtype="f32", u=u)
    y = f.observe()[0]
    # the GPU forms each contribution in FP32 as float(u * float(1/N))
    w0 = np.float32(1.0 / n)
    contrib = (u.astype(np.float32) * w0).astype(np.float64)
    exact = np.sum(np.sort(contrib))
    rel = abs(y / exact - 1)
    _say("deposit", mode, "rel err", rel, "(one FP32 ulp", 2.0 ** -24, ")")
    f.close()
    _abi.m2m_set_deposit_mode("f64")
    assert rel < 1e-12


def test_invalid_arguments(Fit):
    from paper_1202_2355_amd._abi import M2M_EINVAL, M2M_ESTATE, M2MError
    wl = workload(1)
    parts = wl.initial_particles(n=1000)
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f32")
    with pytest.raises(M2MError) as e:
        f.step(1)
    assert e.value.status == M2M_ESTATE
    J = f.J
    for Y, S in [(np.ones(J), np.zeros(J)), (np.full(J, np.nan), np.ones(J)),
                 (np.ones(J - 1), np.ones(J - 1))]:
        with pytest.raises(M2MError) as e:
            f.set_targets(Y, S)
        assert e.value.status == M2M_EINVAL
    f.set_targets(np.ones(J), np.ones(J))
    f.step(2)
    assert np.isfinite(f.observables()["chi2"])
    f.close()


@pytest.mark.parametrize("wlid,steps", [(2, 10), (3, 3), (3, 26)])
def test_full_size_workloads(oracle, Fit, wlid, steps):
    """Workloads 2 and 3 at their full particle counts, in the launch shape
    the benchmark uses (workload 3: interleaved tiles): observables of the
    initial state and weights after a few steps against the oracle; for
    workload 3 also across its first in-step prior refresh (26 steps)."""
    from paper_1202_2355_amd import tuning
    wl = workload(wlid)
    T = oracle_targets(oracle, wl)
    parts = cast(wl.initial_particles(), "f32")
    # the library reads its launch settings when a context is made
    with tuning.tuned("single", wl.state, wl.layout, wl.N) as shape:
        _say("full size", wl.name, wl.N, "launch", shape)
        f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f32")
    y0 = f.observe(T["V_p"], T["sigma_p"])
    yo, ya, yb = oracle.deposit(parts, np.ones(wl.N), wl.layout, V_p=T["V_p"], sigma_p=T["sigma_p"],
                                band=BAND_F32, nthreads=16, with_abs=True)
    assert_observables(y0, yo, ya, yb, 1e-5, wl.name + " initial")
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, T["Y"], T["sigma"], T["V_p"],
                         T["sigma_p"], track_flags=True, band=1e-5, nthreads=16)
    f.step(steps)
    o.step(steps)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("full size", wl.name, "rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    f.close()
    assert r2 <= 1e-4 and rmax <= 1e-4


def test_fp32_vs_fp64_state_per_observable(oracle, Fit):
    """FP32 against FP64 particle state, both on the GPU from the same initial
    state (the FP32 run starts from its rounding): the error of every raw
    observable y_j relative to sum_i |w_i K_ij| after 1, 10, 100 and 200
    steps. Reported per observable group (median and maximum); a particle
    that the rounding moves across a bin edge shows up in the maximum."""
    wl = workload(2)
    T = oracle_targets(oracle, wl)
    n = 100_003
    p64 = wl.initial_particles(n=n, seed=41)
    fd = Fit(wl.potential, wl.layout, wl.params, p64, dtype="f64")
    fs = Fit(wl.potential, wl.layout, wl.params, cast(p64, "f32"), dtype="f32")
    for f in (fd, fs):
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    nr = wl.layout["n_r"]
    done = 0
    rows = []
    for k in (1, 10, 100, 200):
        fd.step(k - done)
        fs.step(k - done)
        done = k
        y64 = fd.observables()["y"]
        y32 = fs.observables()["y"]
        st = fd.particles()
        _, ya, _ = oracle.deposit(st, st["u"], wl.layout, V_p=T["V_p"], sigma_p=T["sigma_p"],
                                  nthreads=8, with_abs=True)
        ok = ya > 0
        e = np.zeros_like(ya)
        e[ok] = np.abs(y32[ok] - y64[ok]) / ya[ok]
        er, ek = e[:nr], e[nr:]
        rows.append((k, np.median(er), er.max(), np.median(ek), ek.max()))
        _say(f"fp32 vs fp64 step {k}: radial median {rows[-1][1]:.2e} max {rows[-1][2]:.2e}; "
             f"GH median {rows[-1][3]:.2e} max {rows[-1][4]:.2e}")
    fd.close()
    fs.close()
    assert rows[0][1] <= 1e-5 and rows[0][3] <= 1e-5
    assert rows[-1][1] <= 1e-3 and rows[-1][3] <= 1e-3



def _clear_of_cell_edges(oracle, pot, par, parts, band):
    """Particles whose (E, x) lie more than ``band`` (relative) from every
    prior-cell edge, so that the GPU and the oracle bin them alike."""
    _, E, xc = oracle.cells(pot, par, parts)
    dE = (par["E_hi"] - par["E_lo"]) / par["n_E"]
    te = (E - par["E_lo"]) / dE
    tx = xc * par["n_x"]
    amb = (np.abs(te - np.round(te)) * dE <= band * abs(par["E_lo"])) | (
        np.abs(tx - np.round(tx)) <= band * par["n_x"])
    return {k: v[~amb] for k, v in parts.items()}


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_prior_smoothing_matches_oracle(oracle, Fit, dtype):
    """Thin-plate GCV smoothing of the prior grid (Sec. 2.3.2): the GPU's
    spectral smoother against the oracle's dense solve, on cell means of the
    same particles (those clear of cell edges, so both bin them alike)."""
    wl = workload(1)
    par = dict(wl.params, smooth=1, n_E=16, n_x=8)
    parts = cast(wl.initial_particles(n=30_011, seed=6), dtype)
    parts = _clear_of_cell_edges(oracle, wl.potential, par, parts, 1e-5)
    n = parts["x"].size
    u = cast({"u": random_weights(n, 13, spread=0.5)}, dtype)["u"]
    _say("prior smoothing", dtype, n)
    f = Fit(wl.potential, wl.layout, par, parts, dtype=dtype, u=u)
    f.update_priors()
    uh = f.particles()["uh"]
    C = par["n_E"] * par["n_x"]
    grid = np.frombuffer(f.get_state()[-8 * C:], dtype=np.float64)
    f.close()
    J = oracle.J_of(wl.layout)
    o = oracle.OracleFit(wl.potential, wl.layout, par, parts, np.ones(J), np.ones(J), u=u)
    o.refresh_priors()
    np.testing.assert_allclose(grid, o.ucell, rtol=1e-10)
    # each particle's prior is its cell's value on that grid: the same bound
    np.testing.assert_allclose(uh, o.arr["uhat"], rtol=1e-6 if dtype == "f32" else 1e-10)


def test_run_with_prior_smoothing_matches_oracle(oracle, Fit):
    """120 FP32 steps with smoothed moving priors (four refreshes) against
    the oracle, to the weight tolerance of the FP32 path."""
    wl = workload(1)
    par = dict(wl.params, smooth=1)
    T = oracle_targets(oracle, wl)
    n = 20_000
    parts = cast(wl.initial_particles(n=n, seed=8), "f32")
    _say("run with smoothing", n)
    f = Fit(wl.potential, wl.layout, par, parts, dtype="f32")
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    o = oracle.OracleFit(wl.potential, wl.layout, par, parts, T["Y"], T["sigma"], T["V_p"],
                         T["sigma_p"], track_flags=True, band=1e-5, nthreads=8)
    f.step(120)
    o.step(120)
    r2, rmax, rall, frac = weight_errors(f.particles()["u"], o.arr["u"], o.flag)
    _say("run with smoothing: rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    f.close()
    assert r2 <= 1e-4 and rmax <= 1e-4


# ------------------------------------------------- spherical-harmonic density
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_alm_observe_matches_oracle(oracle, Fit, dtype):
    """Density observables a_lm,k (Sec. 3.3, eq. alm) on the paper's 60-point
    mesh with l <= 4, plus the Gauss-Hermite annuli, of one state."""
    from workloads import with_alm
    wl = with_alm(workload(2), n_mesh=60, l_max=4)
    n = 50_003
    _say("alm observe", wl.name, dtype, n, "J", wl.J)
    parts = cast(wl.initial_particles(n=n, seed=202), dtype)
    u = cast({"u": random_weights(n, 9)}, dtype)["u"]
    V, S = _gh_centres(wl.layout["n_R"])
    V, S = cast({"V": V, "S": S}, dtype).values()
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype, u=u)
    y = f.observe(V, S)
    band = BAND_F32 if dtype == "f32" else BAND_F64
    yo, ya, yb = oracle.deposit(parts, u, wl.layout, mass=wl.params["mass"], V_p=V, sigma_p=S,
                                band=band, nthreads=8, with_abs=True)
    worst = assert_observables(y, yo, ya, yb, 1e-5 if dtype == "f32" else 1e-12, wl.name)
    _say("alm observe", dtype, "max |dy|/sum|wK| =", worst)
    # the monopole row carries the mass: sum_k a_00,k = Y_00 sum of the mass inside
    nlm = 25
    a00 = np.asarray(y)[:60 * nlm].reshape(60, nlm)[:, 0]
    assert np.all(a00 >= -1e-12)
    f.close()


def test_alm_run_fp64_matches_oracle(oracle, Fit):
    """FP64 state, workload 1 with its radial bins replaced by a_lm (l <= 2)
    on a 30-point mesh: weights and chi^2 history after 100 steps."""
    from workloads import with_alm
    wl = with_alm(workload(1), n_mesh=30, l_max=2)
    n = 20_003
    _say("alm run fp64", wl.name, n)
    T, parts, f, o = _run_pair(oracle, Fit, wl, n, 100, "f64", 1e-12)
    f.step(100)
    hist_o = o.step(100)
    hist_g = f.chi2_history(100)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("alm run fp64: rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    assert r2 <= 1e-10
    assert rmax <= 1e-10
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-9)
    f.close()


def test_alm_run_fp32_matches_oracle(oracle, Fit):
    """FP32 state, workload 2 with a_lm (l <= 4) on 60 mesh radii: weights
    after 50 steps."""
    from workloads import with_alm
    wl = with_alm(workload(2), n_mesh=60, l_max=4)
    n = 30_001
    _say("alm run fp32", wl.name, n)
    T, parts, f, o = _run_pair(oracle, Fit, wl, n, 50, "f32", 1e-5)
    f.step(50)
    hist_o = o.step(50)
    hist_g = f.chi2_history(50)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("alm run fp32: rel2", r2, "max(unflagged)", rmax, "max(all)", rall, "flagged", frac)
    assert r2 <= 1e-4
    assert rmax <= 1e-4
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-4)
    f.close()


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_alm_at_every_block_size_and_batched(oracle, Fit, block):
    """a_lm density observables (l <= 4, 60 mesh radii) with Gauss-Hermite
    annuli at every block size of the step kernel: two states against the
    oracle (the per-observable bar of the FP32 path), then the two fits run
    30 steps with refreshes as a batch against each fit alone."""
    from paper_1202_2355_amd import tuning
    from paper_1202_2355_amd.batch import Batch
    from workloads import with_alm
    wl = with_alm(workload(2), n_mesh=60, l_max=4)
    wl = wl.with_(params=dict(wl.params, prior_every=10))
    T = {"Y": np.ones(wl.J), "sigma": np.full(wl.J, 0.05)}
    V, S = _gh_centres(wl.layout["n_R"])
    V, S = cast({"V": V, "S": S}, "f32").values()
    sizes = (40_009, 9_001)
    parts = [cast(wl.initial_particles(n=n, seed=230 + k), "f32") for k, n in enumerate(sizes)]
    _say("alm block", block, sizes)
    before = tuning.current()
    try:
        tuning.apply(dict(before, block=block, tiles_per_cu=2))
        alone = []
        for k in range(2):
            f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f32")
            y = f.observe(V, S)
            yo, yab, yamb = oracle.deposit(parts[k], np.ones(sizes[k]), wl.layout,
                                           mass=wl.params["mass"], V_p=V, sigma_p=S,
                                           band=BAND_F32, nthreads=8, with_abs=True)
            assert_observables(y, yo, yab, yamb, 1e-5, f"alm block {block} fit {k}")
            f.set_targets(T["Y"], T["sigma"], V, S)
            f.step(30)
            alone.append(f.particles()["u"])
            f.close()
        b = Batch(max_fits=2)
        fits = []
        for k in range(2):
            f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f32")
            f.set_targets(T["Y"], T["sigma"], V, S)
            assert b.admit(f, 30)
            fits.append(f)
        b.run_to_completion(steps_per_launch=10)
        for k, f in enumerate(fits):
            np.testing.assert_allclose(f.particles()["u"], alone[k], rtol=1e-5)
            f.close()
        b.close()
    finally:
        tuning.apply(before)


# ------------------------------------------------ prior-grid options (Sec. 5)
def _oracle_priors(oracle, wl, par, parts, u, band):
    J = oracle.J_of(wl.layout)
    o = oracle.OracleFit(wl.potential, wl.layout, par, parts, np.ones(J), np.ones(J), u=u,
                         track_flags=True, band=band, nthreads=8)
    o.refresh_priors()
    return o


@pytest.mark.parametrize("cells", [1, 2, 3])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_prior_refresh_with_cell_options_matches_oracle(oracle, Fit, dtype, cells):
    """Cells split by the sign of L_z (bit 0) and energy bins linear in
    exp(E) (bit 1): priors of every cell none of whose particles the oracle
    flags as near an edge (or near L_z = 0)."""
    wl = workload(3)
    par = dict(wl.params, cells=cells, n_E=32, n_x=16)
    n = 40_001
    _say("cell options", cells, dtype, n)
    parts = cast(wl.initial_particles(n=n, seed=15), dtype)
    u = cast({"u": random_weights(n, 19, spread=0.5)}, dtype)["u"]
    f = Fit(wl.potential, wl.layout, par, parts, dtype=dtype, u=u)
    f.update_priors()
    uh = f.particles()["uh"]
    f.close()
    band = 1e-5 if dtype == "f32" else 1e-12
    o = _oracle_priors(oracle, wl, par, parts, u, band)
    cell, _, _ = oracle.cells(wl.potential, par, parts)
    lo, hi = prior_bounds(oracle, wl.potential, par, parts, u, o.flag, band)
    unbounded = assert_priors_within(uh, lo, hi, 1e-6 if dtype == "f32" else 1e-13,
                                     f"cell options {cells}")
    _say("cell options", cells, dtype, "flagged", float((o.flag != 0).mean()), "unbounded",
         unbounded)
    assert unbounded < 1e-3
    if cells & 1:
        half = par["n_E"] * par["n_x"]
        assert (cell >= half).any() and (cell < half).any()


def test_prior_smoothing_with_cell_options_matches_oracle(oracle, Fit):
    """Smoothing of both L_z halves, each alone, with energy bins linear in
    exp(E) (FP64 state, particles clear of every cell edge). lambda is the
    first minimum of GCV on a grid whose last stage steps log10(lambda) by
    1/4096; on a flat minimum scores of neighbouring points can agree to
    rounding, and the GPU's spectral scores and the oracle's dense ones may
    then pick neighbours. So every smoothed cell must lie within the oracle's
    values at its lambda and one last-stage step either side, widened by the
    rounding of the oracle's dense Cholesky solve of (I + lambda P), whose
    condition number is 1 + lambda G_max^2 (G_max = 4/hE^2 + 4/hx^2 bounds
    the grid Laplacian; narrow exp(E) cells make it large). The GPU's
    spectral solve has no such loss."""
    wl = workload(1)
    par = dict(wl.params, smooth=1, n_E=16, n_x=8, cells=3)
    parts = wl.initial_particles(n=30_011, seed=16)
    u = random_weights(parts["x"].size, 23, spread=0.5)
    o = _oracle_priors(oracle, wl, par, parts, u, 1e-9)
    keep = o.flag == 0
    parts = {k: v[keep] for k, v in parts.items()}
    u = u[keep]
    _say("smoothing with cell options", parts["x"].size)
    f = Fit(wl.potential, wl.layout, par, parts, dtype="f64", u=u)
    f.update_priors()
    uh = f.particles()["uh"]
    C = oracle.n_cells(par)
    grid = np.frombuffer(f.get_state()[-8 * C:], dtype=np.float64)
    f.close()
    # the data of each half: cell means, 1 (the initial prior) where empty
    cell, _, _ = oracle.cells(wl.potential, par, parts)
    sums = np.bincount(cell, weights=u, minlength=C)
    cnts = np.bincount(cell, minlength=C)
    data = np.where(cnts > 0, sums / np.maximum(cnts, 1), 1.0)
    half = par["n_E"] * par["n_x"]
    step = 10.0 ** (1.0 / 4096)
    hE = (np.exp(par["E_hi"]) - np.exp(par["E_lo"])) / par["n_E"]
    gmax = 4.0 / hE ** 2 + 4.0 * par["n_x"] ** 2
    for h in range(2):
        d = data[h * half:(h + 1) * half]
        w, lam = oracle.smooth_grid(par, d)
        lo = np.minimum.reduce([w, oracle.smooth_grid_at(par, d, lam / step),
                                oracle.smooth_grid_at(par, d, lam * step)])
        hi = np.maximum.reduce([w, oracle.smooth_grid_at(par, d, lam / step),
                                oracle.smooth_grid_at(par, d, lam * step)])
        g = grid[h * half:(h + 1) * half]
        slack = max(1e-12, 8 * np.finfo(float).eps * (1.0 + lam * gmax ** 2)) * np.abs(w)
        _say("half", h, "lambda", lam, "max |gpu - oracle| / |oracle|",
             float(np.max(np.abs(g - w) / np.abs(w))))
        assert np.all(g >= lo - slack) and np.all(g <= hi + slack)
    np.testing.assert_array_equal(uh, grid[cell])


# ---------------------------------------------- logarithmic halo (Sec. 5)
def _halo_workload(oracle, wlid, q=0.7):
    """The workload in its potential plus a flattened logarithmic halo, the
    prior grid's energies spanning [Phi(0), Phi(r = 20)) of the total."""
    from dataclasses import replace
    wl = workload(wlid)
    pot = replace(wl.potential, v0=0.8, r0=2.5, q=q)
    par = dict(wl.params, E_lo=oracle.phi(pot, 0.0), E_hi=oracle.phi(pot, 20.0))
    return wl.with_(name=wl.name + "_halo", potential=pot, params=par)


def test_halo_run_fp64_matches_oracle(oracle, Fit):
    """FP64 state in a flattened logarithmic halo: positions, weights and the
    chi^2 history after 100 steps with two prior refreshes."""
    wl = _halo_workload(oracle, 1)
    n = 20_003
    _say("halo run fp64", wl.name, n)
    T, parts, f, o = _run_pair(oracle, Fit, wl, n, 100, "f64", 1e-12)
    f.step(100)
    hist_o = o.step(100)
    hist_g = f.chi2_history(100)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("halo run fp64: rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(st[k], o.arr[k], rtol=0, atol=1e-9)
    assert r2 <= 1e-10
    assert rmax <= 1e-10
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-9)
    f.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_halo_prior_refresh_matches_oracle(oracle, Fit, dtype):
    """Priors in the halo potential: energies include the halo, circularity
    against equatorial circular orbits (every energy is bound)."""
    wl = _halo_workload(oracle, 3)
    par = dict(wl.params, n_E=32, n_x=16)
    n = 40_001
    _say("halo priors", dtype, n)
    parts = cast(wl.initial_particles(n=n, seed=25), dtype)
    u = cast({"u": random_weights(n, 29, spread=0.5)}, dtype)["u"]
    f = Fit(wl.potential, wl.layout, par, parts, dtype=dtype, u=u)
    f.update_priors()
    uh = f.particles()["uh"]
    f.close()
    band = 1e-5 if dtype == "f32" else 1e-12
    o = _oracle_priors(oracle, wl, par, parts, u, band)
    cell, E, xc = oracle.cells(wl.potential, par, parts)
    assert (E > 0).any()   # bound energies above 0 exist in the halo
    lo, hi = prior_bounds(oracle, wl.potential, par, parts, u, o.flag, band)
    unbounded = assert_priors_within(uh, lo, hi, 1e-6 if dtype == "f32" else 1e-13, "halo priors")
    _say("halo priors", dtype, "flagged", float((o.flag != 0).mean()), "unbounded", unbounded)
    assert unbounded < 1e-3
