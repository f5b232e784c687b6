"""The push of the step kernel against what a drift-kick-drift leapfrog in a
fixed spherical potential must do (Sec. 4.1; the potentials of Sec. 3.1 eq.
her and of the dark halo): properties that hold at any size, checked on the
full-size particle sets of the Gauss-Hermite workload (10^6 particles,
Hernquist) and of the LOSVD workload (8 * 10^6, Hernquist + NFW), in the
launch the library picks for them.

Only relaxation steps run here (no weight correction): the particles move,
the weights must stay as they were, bit for bit.

* Angular momentum: the kick is radial and the drift straight, so |r x v| is
  conserved exactly in exact arithmetic; what is left is rounding, which
  grows like a random walk over the steps.
* Energy: bounded, and at a fixed time T the error of each orbit scales as
  dt^2 (halving dt divides it by 4) wherever it is above rounding.
* Reversibility: n steps, flip v, n steps, flip v returns the start state.

Energies and angular momenta are evaluated here in FP64 from the returned
state (relative potential of the particle generators)."""

import sys

import numpy as np
import pytest

from m2m_testlib import cast, oracle_targets
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


def _ang(s):
    x, y, z, vx, vy, vz = (s[k] for k in ("x", "y", "z", "vx", "vy", "vz"))
    return np.sqrt((y * vz - z * vy) ** 2 + (z * vx - x * vz) ** 2 + (x * vy - y * vx) ** 2)


def _energy(pot, s):
    r = np.sqrt(s["x"] ** 2 + s["y"] ** 2 + s["z"] ** 2)
    return 0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2) - pot.psi(r)


def _fit(Fit, T, wl, parts, dtype, **par):
    f = Fit(wl.potential, wl.layout, dict(wl.params, **par), parts, dtype=dtype)
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    return f


def _q(a, p):
    return float(np.percentile(a, p))


@pytest.mark.parametrize("wlid,steps", [(2, 1000), (3, 400)])
def test_push_conserves_angular_momentum(oracle, Fit, wlid, steps):
    """|r x v| per particle after the workload's steps, FP32 and FP64 state:
    the median relative change within 1e-5 (FP32) and 1e-13 (FP64), the
    99th percentile within 1e-4 and 1e-12; the weights are unchanged."""
    wl = workload(wlid)
    p64 = wl.initial_particles()
    L0 = _ang(p64)
    T = oracle_targets(oracle, wl)
    for dtype, med_tol, p99_tol in (("f32", 1e-5, 1e-4), ("f64", 1e-13, 1e-12)):
        parts = cast(p64, dtype)
        _say("angular momentum", wl.name, wl.N, dtype, steps, "steps")
        f = _fit(Fit, T, wl, parts, dtype)
        f.step(steps, correct=False)
        st = f.particles()
        f.close()
        L0d = _ang(parts) if dtype == "f32" else L0
        ok = L0d > 0
        d = np.abs(_ang(st)[ok] - L0d[ok]) / L0d[ok]
        _say(f"  |dL|/L median {np.median(d):.2e} p99 {_q(d, 99):.2e} max {d.max():.2e}")
        assert np.all(st["u"] == 1.0), "relaxation steps changed the weights"
        assert np.all(np.isfinite(d))
        assert np.median(d) <= med_tol and _q(d, 99) <= p99_tol


@pytest.mark.parametrize("wlid", [2, 3])
def test_energy_error_is_second_order_in_dt(oracle, Fit, wlid):
    """FP64 state, the same time T = 10 with dt and dt / 2: for bound orbits
    whose energy error is well above rounding (> 1e-9 relative) the ratio of
    the errors is 4 to within 2 % in the median and 10 % in the 5th and 95th
    percentiles; the median error itself is small (< 1e-5 relative)."""
    wl = workload(wlid)
    n = 200_003
    p64 = wl.initial_particles(n=n, seed=43)
    E0 = _energy(wl.potential, p64)
    dt = wl.params["dt"]
    nsteps = int(round(10.0 / dt))
    T = oracle_targets(oracle, wl)
    err = []
    for k in (1, 2):
        _say("energy", wl.name, n, "dt", dt / k, "steps", k * nsteps)
        f = _fit(Fit, T, wl, p64, "f64", dt=dt / k)
        f.step(k * nsteps, correct=False)
        err.append((_energy(wl.potential, f.particles()) - E0) / np.abs(E0))
        f.close()
    bound = E0 < 0
    big = bound & (np.abs(err[0]) > 1e-9)
    ratio = np.abs(err[0][big]) / np.abs(err[1][big])
    _say(f"  median |dE/E| {np.median(np.abs(err[0][bound])):.2e}; {big.sum()} orbits above rounding: "
         f"ratio median {np.median(ratio):.4f} p5 {_q(ratio, 5):.4f} p95 {_q(ratio, 95):.4f}")
    assert big.sum() >= n // 2
    assert np.median(np.abs(err[0][bound])) <= 1e-5
    assert abs(np.median(ratio) - 4.0) <= 0.08
    assert 3.6 <= _q(ratio, 5) and _q(ratio, 95) <= 4.4


@pytest.mark.parametrize("wlid", [2, 3])
def test_push_is_time_reversible(oracle, Fit, wlid):
    """FP64 state: 500 steps, velocities negated in the caller's arrays, 500
    steps, negated back: positions and velocities return to the start to
    1e-13 (median) and 1e-11 (99th percentile) of |r| and |v|."""
    wl = workload(wlid)
    n = 200_003
    p64 = wl.initial_particles(n=n, seed=44)
    _say("reversibility", wl.name, n)
    f = _fit(Fit, oracle_targets(oracle, wl), wl, p64, "f64")
    f.step(500, correct=False)

    def flip():
        with torch.cuda.stream(f.stream):
            for k in ("vx", "vy", "vz"):
                f.t[k].neg_()

    flip()
    f.step(500, correct=False)
    flip()
    st = f.particles()
    f.close()
    r0 = np.sqrt(p64["x"] ** 2 + p64["y"] ** 2 + p64["z"] ** 2)
    v0 = np.sqrt(p64["vx"] ** 2 + p64["vy"] ** 2 + p64["vz"] ** 2)
    ex = np.sqrt(sum((st[k] - p64[k]) ** 2 for k in ("x", "y", "z"))) / r0
    ev = np.sqrt(sum((st[k] - p64[k]) ** 2 for k in ("vx", "vy", "vz"))) / v0
    _say(f"  position median {np.median(ex):.2e} p99 {_q(ex, 99):.2e} max {ex.max():.2e}; "
         f"velocity median {np.median(ev):.2e} p99 {_q(ev, 99):.2e} max {ev.max():.2e}")
    for e in (ex, ev):
        assert np.median(e) <= 1e-13 and _q(e, 99) <= 1e-11
