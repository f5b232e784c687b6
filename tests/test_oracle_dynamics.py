"""Pins of the oracle's potential, L_c(E) and leapfrog against closed forms
and invariants (no GPU).

* potential and force: eq. her (Sec. 3.1), NFW enclosed mass by quadrature
  of its density, force = -dPhi/dr by finite differences;
* L_c(E): the Hernquist closed form of the circular orbit of energy E;
* drift-kick-drift leapfrog (Sec. 4.1): exact angular-momentum
  conservation, bounded O(dt^2) energy error, time reversibility, circular
  orbits.
"""

import math

import numpy as np
import pytest
from scipy import integrate

HERN = dict(G=1.0, M_star=1.0, a=1.0, upsilon=1.0, M200=0.0, c=0.0, r_s=0.0)
NFW = dict(G=1.0, M_star=1.0, a=1.0, upsilon=1.0, M200=10.0, c=8.0, r_s=12.5)


def test_hernquist_potential_eq_her(oracle):
    for r in (0.0, 0.01, 0.5, 1.0, 3.0, 100.0):
        assert oracle.phi(HERN, r) == pytest.approx(-1.0 / (r + 1.0), rel=1e-15)
    p = dict(HERN, upsilon=2.5, a=0.7)
    assert oracle.phi(p, 2.0) == pytest.approx(-2.5 / 2.7, rel=1e-15)


def test_nfw_central_potential_and_mass_by_quadrature(oracle):
    fc = math.log(9.0) - 8.0 / 9.0
    # Phi(0) of Hernquist(1,1) + NFW(M200 = 10, c = 8, r_s = 12.5)
    assert oracle.phi(NFW, 0.0) == pytest.approx(-1.0 - 10.0 / (fc * 12.5), rel=1e-14)
    assert oracle.phi(NFW, 0.0) == pytest.approx(-1.6114, abs=1e-4)
    # enclosed mass from the force (Gauss) against the integrated densities
    rho0 = 10.0 / (4.0 * math.pi * 12.5 ** 3 * fc)
    for r in (0.3, 5.0, 40.0, 100.0):
        m_nfw = integrate.quad(lambda s: 4 * math.pi * s * s * rho0 / ((s / 12.5) * (1 + s / 12.5) ** 2),
                               0, r, epsabs=0, epsrel=1e-12, limit=200)[0]
        m_her = integrate.quad(lambda s: 4 * math.pi * s * s / (2 * math.pi * s * (s + 1) ** 3),
                               0, r, epsabs=0, epsrel=1e-12, limit=200)[0]
        g = oracle.accel(NFW, r, 0.0, 0.0)
        assert -g[0] * r * r == pytest.approx(m_nfw + m_her, rel=1e-9)
    # NFW total mass at r200 = c r_s is M200
    assert oracle.lib().orc_mass(oracle.C.byref(oracle.potential(dict(NFW, M_star=0.0))),
                                 100.0) == pytest.approx(10.0, rel=1e-13)


@pytest.mark.parametrize("pot", [HERN, NFW])
def test_force_is_minus_potential_gradient(oracle, pot):
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.normal(size=3) * rng.uniform(0.1, 10)
        r = np.linalg.norm(x)
        h = 1e-5 * r
        dphi = (oracle.phi(pot, r + h) - oracle.phi(pot, r - h)) / (2 * h)
        g = oracle.accel(pot, *x)
        np.testing.assert_allclose(g, -dphi * x / r, rtol=1e-7)
    assert np.all(oracle.accel(pot, 0.0, 0.0, 0.0) == 0.0)


def _lc_hernquist(E, GM=1.0, a=1.0):
    s = (GM + math.sqrt(GM * GM - 8.0 * E * GM * a)) / (-4.0 * E)
    rc = s - a
    return math.sqrt(GM * rc) * rc / (rc + a)


def test_lc_matches_hernquist_closed_form(oracle):
    for E in np.concatenate([-np.geomspace(1e-4, 0.999, 40), [-0.5, -0.25]]):
        assert oracle.lc(HERN, E) == pytest.approx(_lc_hernquist(E), rel=1e-11)
    assert oracle.lc(HERN, -1.0) == 0.0
    assert math.isinf(oracle.lc(HERN, 0.0))


def test_lc_composite_is_circular_orbit(oracle):
    """For the composite potential the returned L_c is that of a circular
    orbit (v_c^2 = r dPhi/dr by finite differences) of energy E."""
    for E in (-1.5, -1.0, -0.5, -0.1, -0.01):
        Lc = oracle.lc(NFW, E)
        # find r with r v_c(r) = Lc and check the energy there
        def lc_of_r(r):
            h = 1e-6 * r
            dphi = (oracle.phi(NFW, r + h) - oracle.phi(NFW, r - h)) / (2 * h)
            return r * math.sqrt(r * dphi)
        from scipy.optimize import brentq
        rc = brentq(lambda r: lc_of_r(r) - Lc, 1e-8, 1e6, xtol=1e-14, rtol=1e-14)
        h = 1e-6 * rc
        dphi = (oracle.phi(NFW, rc + h) - oracle.phi(NFW, rc - h)) / (2 * h)
        assert oracle.phi(NFW, rc) + 0.5 * rc * dphi == pytest.approx(E, rel=1e-7)


def _orbits(n=6, seed=3):
    rng = np.random.default_rng(seed)
    parts = {k: np.empty(n) for k in ("x", "y", "z", "vx", "vy", "vz")}
    for i in range(n):
        x = rng.normal(size=3)
        x *= rng.uniform(0.3, 3.0) / np.linalg.norm(x)
        r = np.linalg.norm(x)
        vesc = math.sqrt(2.0 / (r + 1.0))
        v = rng.normal(size=3)
        v *= rng.uniform(0.2, 0.8) * vesc / np.linalg.norm(v)
        for k, val in zip(("x", "y", "z", "vx", "vy", "vz"), (*x, *v)):
            parts[k][i] = val
    return parts


def _L(p):
    return np.stack([p["y"] * p["vz"] - p["z"] * p["vy"],
                     p["z"] * p["vx"] - p["x"] * p["vz"],
                     p["x"] * p["vy"] - p["y"] * p["vx"]], axis=1)


def _E(oracle, pot, p):
    r = np.sqrt(p["x"] ** 2 + p["y"] ** 2 + p["z"] ** 2)
    return 0.5 * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2) + np.array(
        [oracle.phi(pot, ri) for ri in r])


@pytest.mark.parametrize("pot", [HERN, NFW])
def test_leapfrog_conserves_angular_momentum(oracle, pot):
    p0 = _orbits()
    p1 = oracle.push(pot, 0.01, p0, 10000)
    L0, L1 = _L(p0), _L(p1)
    rel = np.linalg.norm(L1 - L0, axis=1) / np.linalg.norm(L0, axis=1)
    assert rel.max() < 1e-13


def test_leapfrog_energy_bounded_second_order(oracle):
    p0 = _orbits(n=4, seed=7)
    E0 = _E(oracle, HERN, p0)

    def max_err(dt, T):
        p = p0
        worst = np.zeros(4)
        nstep = int(round(T / dt))
        chunk = max(1, nstep // 200)
        for _ in range(nstep // chunk):
            p = oracle.push(HERN, dt, p, chunk)
            worst = np.maximum(worst, np.abs(_E(oracle, HERN, p) / E0 - 1.0))
        return worst

    e1 = max_err(0.02, 20.0)
    e2 = max_err(0.01, 20.0)
    ratio = e1 / e2
    assert np.all((ratio > 3.0) & (ratio < 5.5)), ratio
    # no secular drift: ten times longer does not grow the error much
    e_long = max_err(0.02, 200.0)
    assert np.all(e_long < 2.0 * e1 + 1e-14)


def test_leapfrog_time_reversible(oracle):
    p0 = _orbits(n=5, seed=11)
    p1 = oracle.push(NFW, 0.01, p0, 2000)
    back = dict(p1)
    for k in ("vx", "vy", "vz"):
        back[k] = -p1[k]
    p2 = oracle.push(NFW, 0.01, back, 2000)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(p2[k], p0[k], atol=1e-11)
    for k in ("vx", "vy", "vz"):
        np.testing.assert_allclose(-p2[k], p0[k], atol=1e-11)


def test_circular_orbit_radius_and_period(oracle):
    r0 = 1.0
    vc = math.sqrt(r0) / (r0 + 1.0)          # v_c^2 = G M r / (r + a)^2
    period = 2.0 * math.pi * r0 / vc
    dev, perr = {}, {}
    for dt in (0.02, 0.01):
        p = dict(x=np.array([r0]), y=np.zeros(1), z=np.zeros(1), vx=np.zeros(1),
                 vy=np.array([vc]), vz=np.zeros(1))
        n = int(round(period / dt))
        worst, phase = 0.0, 0.0
        prev = 0.0
        for _ in range(n):
            p = oracle.push(HERN, dt, p, 1)
            r = math.hypot(p["x"][0], p["y"][0])
            worst = max(worst, abs(r / r0 - 1.0))
            ang = math.atan2(p["y"][0], p["x"][0])
            d = (ang - prev + math.pi) % (2 * math.pi) - math.pi
            phase += d
            prev = ang
        dev[dt] = worst
        # one period later the orbit has turned by 2 pi (to the step length)
        assert abs(phase - 2 * math.pi) < 2 * vc * dt / r0
        # phase error after the whole number of steps nearest the period,
        # corrected for the rounding of the period to whole steps
        perr[dt] = abs(phase - 2 * math.pi * n * dt / period)
    # the radius of a circular orbit is kept (to far better than dt^2) and
    # the phase error is second order in dt
    assert max(dev.values()) < 1e-8
    assert 3.0 < perr[0.02] / perr[0.01] < 5.0


# ------------------------------------------- the push inside the fit's step loop
def _fit_without_correction(oracle, pot, parts):
    """An oracle fit whose steps only push (correct = 0: relaxation, Sec. 4.1):
    its step loop is the code whose drift-kick-drift the fit runs."""
    from workloads import make_layout, make_params, make_potential
    lay = make_layout(4, 0.05, 20.0)
    par = make_params(make_potential(), prior_every=0)
    J = oracle.J_of(lay)
    return oracle.OracleFit(pot, lay, par, parts, np.ones(J), np.ones(J))


@pytest.mark.parametrize("pot", [HERN, NFW])
def test_step_loop_conserves_angular_momentum(oracle, pot):
    """10^4 relaxation steps of the fit's own step loop: the kick is radial,
    so L = r x v is kept to rounding (P1)."""
    p0 = _orbits()
    f = _fit_without_correction(oracle, pot, p0)
    f.step(10000, correct=False)
    L0, L1 = _L(p0), _L(f.arr)
    rel = np.linalg.norm(L1 - L0, axis=1) / np.linalg.norm(L0, axis=1)
    assert rel.max() < 1e-13


def test_step_loop_is_time_reversible(oracle):
    """n relaxation steps of the fit, velocities flipped, n more steps:
    the start state comes back (P3); a drift and a kick in the wrong order
    would not."""
    p0 = _orbits(n=5, seed=11)
    f = _fit_without_correction(oracle, NFW, p0)
    f.step(2000, correct=False)
    back = {k: f.arr[k].copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    for k in ("vx", "vy", "vz"):
        back[k] = -back[k]
    g = _fit_without_correction(oracle, NFW, back)
    g.step(2000, correct=False)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(g.arr[k], p0[k], atol=1e-11)
    for k in ("vx", "vy", "vz"):
        np.testing.assert_allclose(-g.arr[k], p0[k], atol=1e-11)


def test_step_loop_energy_error_is_second_order(oracle):
    """The fit's step loop conserves energy to O(dt^2) with no drift (P2):
    halving dt cuts the largest energy error about four times."""
    from workloads import make_layout, make_params, make_potential
    p0 = _orbits(n=4, seed=7)
    E0 = _E(oracle, HERN, p0)
    lay = make_layout(4, 0.05, 20.0)
    J = oracle.J_of(lay)
    worst = {}
    for dt in (0.02, 0.01):
        par = make_params(make_potential(), prior_every=0, dt=dt)
        f = oracle.OracleFit(HERN, lay, par, p0, np.ones(J), np.ones(J))
        w = np.zeros(4)
        n = int(round(20.0 / dt))
        for _ in range(100):
            f.step(n // 100, correct=False)
            w = np.maximum(w, np.abs(_E(oracle, HERN, f.arr) / E0 - 1.0))
        worst[dt] = w
    ratio = worst[0.02] / worst[0.01]
    assert np.all((ratio > 3.0) & (ratio < 5.5)), ratio


def test_step_loop_moves_particles_as_the_integrator(oracle):
    """Without correction the fit's particles follow the bare integrator
    bit for bit: the step loop adds nothing to the push."""
    p0 = _orbits(n=7, seed=5)
    f = _fit_without_correction(oracle, NFW, p0)
    f.step(300, correct=False)
    q = oracle.push(NFW, f.m.par.dt, p0, 300)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_array_equal(f.arr[k], q[k])
