"""GPU parity at the edges of the particle count (run on an MI355X): fits of
1, 63, 64 and 65 particles (one tile, shorter than one tile boundary of 64,
exactly one, one more) and a batch that mixes a one-particle fit with larger
ones. FP64 state, so the only difference from the oracle is summation
order: positions within 1e-12, weights within 1e-10, chi^2 within 1e-10.
Each fit's targets are its own initial observables with 5 % errors (a few
particles against a full-model target would drive the weights to overflow,
which the library reports as a non-finite chi^2)."""

import sys

import numpy as np
import pytest

from m2m_testlib import cast
from workloads import workload

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


def _wl():
    wl = workload(1)
    return wl.with_(params=dict(wl.params, prior_every=4))


def _own_targets(oracle, wl, parts):
    Y = oracle.deposit(parts, np.ones(parts["x"].size), wl.layout, mass=wl.params["mass"])
    return {"Y": Y, "sigma": 0.05 * np.abs(Y) + 1e-3 * np.abs(Y).max() + 1e-12, "V_p": None,
            "sigma_p": None}


@pytest.mark.parametrize("n", [1, 63, 64, 65])
def test_tiny_fits_match_oracle(oracle, Fit, n):
    wl = _wl()
    parts = cast(wl.initial_particles(n=n, seed=61 + n), "f64")
    T = _own_targets(oracle, wl, parts)
    _say("tiny fit", n)
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f64")
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, T["Y"], T["sigma"], T["V_p"],
                         T["sigma_p"])
    f.step(10)  # two prior refreshes
    hist_o = o.step(10)
    st = f.particles()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(st[k], o.arr[k], rtol=0, atol=1e-12)
    np.testing.assert_allclose(st["u"], o.arr["u"], rtol=1e-10)
    np.testing.assert_allclose(st["uh"], o.arr["uhat"], rtol=1e-10)
    np.testing.assert_allclose(f.chi2_history(10), hist_o, rtol=1e-10)
    f.close()


def test_batch_with_a_one_particle_fit_equals_alone(oracle, Fit):
    from paper_1202_2355_amd.batch import Batch
    wl = _wl()
    sizes, steps = [1, 65, 5_003], [9, 12, 7]
    _say("tiny batch", sizes)
    parts = [cast(wl.initial_particles(n=n, seed=70 + k), "f64") for k, n in enumerate(sizes)]
    Ts = [_own_targets(oracle, wl, p) for p in parts]
    alone = []
    for k in range(3):
        f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f64")
        T = Ts[k]
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        f.step(steps[k])
        alone.append((f.particles(), f.chi2_history(steps[k])))
        f.close()
    b = Batch(max_fits=4)
    fits = []
    for k in range(3):
        f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f64")
        T = Ts[k]
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        b.admit(f, steps[k])
        fits.append(f)
    assert len(b.run_to_completion(steps_per_launch=4)) == 3
    for k, f in enumerate(fits):
        st = f.particles()
        for key in ("x", "y", "z", "vx", "vy", "vz"):
            np.testing.assert_allclose(st[key], alone[k][0][key], rtol=0, atol=1e-12)
        np.testing.assert_allclose(st["u"], alone[k][0]["u"], rtol=1e-10)
        np.testing.assert_allclose(f.chi2_history(steps[k]), alone[k][1], rtol=1e-10)
        f.close()
    b.close()


def test_overflowing_weights_are_reported_as_a_non_finite_chi2(oracle, Fit):
    """One particle against the targets of a whole model: the force of change
    drives its weight past the largest double within a few steps; the next
    synchronizing call reports M2M_ENONFINITE (the oracle overflows too)."""
    from m2m_testlib import oracle_targets
    from paper_1202_2355_amd._abi import M2M_ENONFINITE, M2MError
    wl = _wl()
    T = oracle_targets(oracle, wl)
    parts = cast(wl.initial_particles(n=1, seed=62), "f64")
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, T["Y"], T["sigma"], T["V_p"],
                         T["sigma_p"])
    o.step(10)
    assert not np.isfinite(o.chi2)
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f64")
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    f.step(10)
    with pytest.raises(M2MError) as e:
        f.weights()
    assert e.value.status == M2M_ENONFINITE
    f.close()


# ----------------------------------------------------------- maximum sizes
def _observe_case(oracle, Fit, wl, lay, dtype, n, seed, gh=False):
    from m2m_testlib import BAND_F32, BAND_F64, assert_observables, random_weights
    parts = cast(wl.initial_particles(n=n, seed=seed), dtype)
    u = cast({"u": random_weights(n, seed + 1)}, dtype)["u"]
    V = S = None
    if gh:
        g = np.random.default_rng(seed)
        V, S = g.uniform(-0.05, 0.05, lay["n_R"]), g.uniform(0.25, 0.6, lay["n_R"])
        V, S = cast({"V": V, "S": S}, dtype).values()
    f = Fit(wl.potential, lay, wl.params, parts, dtype=dtype, u=u)
    y = f.observe(V, S) if gh else f.observe()
    band = BAND_F32 if dtype == "f32" else BAND_F64
    yo, ya, yb = oracle.deposit(parts, u, lay, mass=wl.params["mass"], V_p=V, sigma_p=S,
                                band=band, nthreads=8, with_abs=True)
    worst = assert_observables(y, yo, ya, yb, 1e-5 if dtype == "f32" else 1e-12, str(lay["kin"]))
    _say("observe", lay["kin"], dtype, "J", y.size, "max |dy|/sum|wK| =", worst)
    f.close()


@pytest.mark.parametrize("dtype,n_v", [("f32", 256), ("f64", 128)])
def test_largest_losvd_layouts_observe_like_the_oracle(oracle, Fit, dtype, n_v):
    """256 velocity bins in 40 annuli (J = 10290) is the largest LOSVD layout
    whose in-tile bins and tables fit the LDS of a CU with FP32 state; FP64
    state takes twice the table space (128 bins, J = 5170)."""
    wl = workload(3)
    lay = dict(wl.layout, n_v=n_v)
    _observe_case(oracle, Fit, wl, lay, dtype, 50_003, 80)


def test_gauss_hermite_of_order_eight_observes_like_the_oracle(oracle, Fit):
    wl = workload(2)
    lay = dict(wl.layout, gh_nmax=8)
    _observe_case(oracle, Fit, wl, lay, "f32", 50_003, 82, gh=True)


def test_layout_too_large_for_lds_is_refused(Fit):
    from paper_1202_2355_amd._abi import M2M_EUNSUPPORTED, M2MError
    wl = workload(3)
    lay = dict(wl.layout, n_R=62, n_v=256)  # J = 50 + 62 * 256 = 15922 <= 16384
    parts = cast(wl.initial_particles(n=4_096, seed=84), "f32")
    with pytest.raises(M2MError) as e:
        Fit(wl.potential, lay, wl.params, parts, dtype="f32")
    assert e.value.status == M2M_EUNSUPPORTED


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_largest_prior_grid_refreshes_like_the_oracle(oracle, Fit, dtype):
    """64 x 64 = 4096 cells, the largest prior grid."""
    from m2m_testlib import random_weights
    wl = workload(3)
    P = dict(wl.params, n_E=64, n_x=64)
    n = 50_003
    _say("largest prior grid", dtype, n)
    parts = cast(wl.initial_particles(n=n, seed=86), dtype)
    u = cast({"u": random_weights(n, 87, spread=0.5)}, dtype)["u"]
    f = Fit(wl.potential, wl.layout, P, parts, dtype=dtype, u=u)
    f.update_priors()
    uh = f.particles()["uh"]
    f.close()
    from m2m_testlib import assert_priors_within, prior_bounds
    band = 1e-5 if dtype == "f32" else 1e-12
    J = oracle.J_of(wl.layout)
    o = oracle.OracleFit(wl.potential, wl.layout, P, parts, np.ones(J), np.ones(J), u=u,
                         track_flags=True, band=band, nthreads=8)
    o.refresh_priors()
    lo, hi = prior_bounds(oracle, wl.potential, P, parts, u, o.flag, band)
    cnts = np.bincount(oracle.cells(wl.potential, P, parts)[0], minlength=P["n_E"] * P["n_x"])
    _say("largest prior grid", dtype, "occupied cells", np.count_nonzero(cnts), "flagged",
         float((o.flag != 0).mean()))
    assert np.count_nonzero(cnts) > 1000
    unbounded = assert_priors_within(uh, lo, hi, 1e-6 if dtype == "f32" else 1e-13, "64 x 64 grid")
    _say("largest prior grid", dtype, "unbounded", unbounded)
    assert unbounded < 1e-3
