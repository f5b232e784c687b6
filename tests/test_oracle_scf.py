"""Pins of the oracle's self-consistent stellar potential (Sec. 2.1; Sec. 5,
spherical-harmonic decomposition at constant M/L): the multipole expansion of
the particles, exact at the nodes and interpolated between them.

At a node the truncated expansion must approach the direct sum over point
masses, -G sum_i m_i / |x - x_i|, as l_max grows: from outside a cloud
(the A_lm terms) and from inside a shell (the B_lm terms). For l_max = 0 it is
the shell theorem. The force must be minus the gradient of the potential,
also in the core and beyond the last node. Potential and force must be
continuous across the nodes. A realization of a Hernquist sphere must
reproduce the analytic Hernquist potential within its sampling noise.
"""

import numpy as np
import pytest

from oracle import oracle as O
from workloads import workload

BASE = dict(G=1.0, M_star=1.0, a=1.0, upsilon=1.0, M200=0.0, c=0.0, r_s=0.0)


def _pot(lmax=4, nr=32, rmin=0.01, rmax=100.0, every=1, **kw):
    return dict(BASE, scf_lmax=lmax, scf_nr=nr, scf_rmin=rmin, scf_rmax=rmax, scf_every=every, **kw)


def _nodes(p):
    k = np.arange(p["scf_nr"])
    return p["scf_rmin"] * (p["scf_rmax"] / p["scf_rmin"]) ** (k / (p["scf_nr"] - 1))


def _cloud(rng, n, r_lo, r_hi, axes=(1.0, 0.7, 0.5)):
    """Anisotropic cloud with radii uniform in [r_lo, r_hi) before squashing."""
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    rad = rng.uniform(r_lo, r_hi, n)
    P = rad[:, None] * v * np.asarray(axes)
    return P, dict(x=P[:, 0], y=P[:, 1], z=P[:, 2])


def _direct(P, u, mass, X, G=1.0, upsilon=1.0):
    m = upsilon * u * mass / len(u)
    return -G * np.sum(m / np.linalg.norm(P - X, axis=1))


def _dirs(rng, k):
    d = rng.normal(size=(k, 3))
    return d / np.linalg.norm(d, axis=1)[:, None]


def test_exterior_expansion_converges_to_the_direct_sum():
    rng = np.random.default_rng(7)
    P, parts = _cloud(rng, 1500, 0.0, 1.0)
    u = rng.uniform(0.5, 1.5, len(P))
    errs = {}
    for lmax in (2, 8):
        p = _pot(lmax=lmax)
        tab = O.scf_table(p, parts, u, mass=2.0)
        rho = _nodes(p)[23]  # ~ 9.2, outside the cloud
        err = 0.0
        for d in _dirs(rng, 6):
            X = rho * d
            ref = _direct(P, u, 2.0, X)
            err = max(err, abs(O.scf_phi(p, tab, *X) - ref) / abs(ref))
        errs[lmax] = err
    # the truncation error falls like (1/rho)^(lmax+1)
    assert errs[8] < 1e-8
    assert errs[2] > 1e-6 and errs[8] < 1e-3 * errs[2]


def test_interior_expansion_converges_to_the_direct_sum():
    rng = np.random.default_rng(8)
    P, parts = _cloud(rng, 1500, 6.0, 9.0, axes=(1.0, 0.8, 0.6))
    u = rng.uniform(0.5, 1.5, len(P))
    p = _pot(lmax=8, upsilon=1.7, G=0.5)
    tab = O.scf_table(p, parts, u, mass=1.0)
    rho = _nodes(p)[12]  # ~ 0.44, inside the shell
    for d in _dirs(rng, 6):
        X = rho * d
        ref = _direct(P, u, 1.0, X, G=0.5, upsilon=1.7)
        assert abs(O.scf_phi(p, tab, *X) - ref) < 1e-9 * abs(ref)


def test_monopole_is_the_shell_theorem():
    rng = np.random.default_rng(9)
    P, parts = _cloud(rng, 800, 0.0, 20.0)
    u = rng.uniform(0.2, 2.0, len(P))
    p = _pot(lmax=0, nr=12, rmin=0.5, rmax=30.0)
    tab = O.scf_table(p, parts, u, mass=3.0)
    r = np.linalg.norm(P, axis=1)
    m = u * 3.0 / len(u)
    y00 = 0.5 / np.sqrt(np.pi)
    for k, rho in enumerate(_nodes(p)):
        inside = r < rho
        phi = -(m[inside].sum() / rho + np.sum(m[~inside] / r[~inside]))
        assert abs(tab[k, 0, 0] * y00 - phi) < 1e-12 * abs(phi)
        # r dPhi/dr = G M(<r) / r
        assert abs(tab[k, 0, 1] * y00 - m[inside].sum() / rho) < 1e-12 * max(abs(phi), 1e-300)


def _grad(p, tab, X, h):
    g = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g[k] = -(O.scf_phi(p, tab, *(X + e)) - O.scf_phi(p, tab, *(X - e))) / (2 * h)
    return g


@pytest.mark.parametrize("r", [0.004, 0.07, 0.9, 3.3, 40.0, 250.0])
def test_force_is_minus_the_gradient_of_the_potential(r):
    """In the core (r < rho_0), between nodes and beyond the last node."""
    rng = np.random.default_rng(10)
    P, parts = _cloud(rng, 600, 0.0, 60.0)
    u = rng.uniform(0.5, 1.5, len(P))
    p = _pot(lmax=4, nr=24)
    tab = O.scf_table(p, parts, u)
    for d in list(_dirs(rng, 4)) + [np.array([1e-4, 0.0, 1.0]) / np.hypot(1e-4, 1.0)]:
        X = r * d
        g = O.scf_accel(p, tab, *X)
        ref = _grad(p, tab, X, 1e-5 * r)
        assert np.linalg.norm(g - ref) < 1e-6 * np.linalg.norm(ref), (r, d)


def test_potential_and_force_are_continuous_across_nodes():
    rng = np.random.default_rng(11)
    P, parts = _cloud(rng, 600, 0.0, 60.0)
    p = _pot(lmax=3, nr=16)
    tab = O.scf_table(p, parts)
    for rho in _nodes(p)[[0, 5, 15]]:
        d = _dirs(rng, 1)[0]
        lo, hi = rho * (1 - 1e-10) * d, rho * (1 + 1e-10) * d
        a, b = O.scf_phi(p, tab, *lo), O.scf_phi(p, tab, *hi)
        assert abs(a - b) < 1e-8 * abs(a)
        ga, gb = O.scf_accel(p, tab, *lo), O.scf_accel(p, tab, *hi)
        assert np.linalg.norm(ga - gb) < 1e-6 * np.linalg.norm(ga)


def test_beyond_the_last_node_the_form_is_exact_for_mass_inside():
    """With all mass inside the last node the decaying form is the exact
    exterior multipole: it approaches the direct sum far out."""
    rng = np.random.default_rng(15)
    P, parts = _cloud(rng, 1000, 0.0, 5.0)
    u = rng.uniform(0.5, 1.5, len(P))
    p = _pot(lmax=8, nr=16, rmin=0.1, rmax=10.0)
    tab = O.scf_table(p, parts, u)
    for r in (25.0, 60.0, 400.0):
        for d in _dirs(rng, 3):
            X = r * d
            ref = _direct(P, u, 1.0, X)
            assert abs(O.scf_phi(p, tab, *X) - ref) < 1e-7 * abs(ref), r


def test_beyond_the_last_node_the_potential_decays():
    """With mass beyond the last node (a wide cloud), Phi_* and the force
    still fall off outside it: r |Phi| and r^2 |g| stay bounded."""
    rng = np.random.default_rng(16)
    P, parts = _cloud(rng, 2000, 0.0, 300.0)
    p = _pot(lmax=4, nr=20, rmin=0.1, rmax=50.0)
    tab = O.scf_table(p, parts)
    d = _dirs(rng, 1)[0]
    rs = np.geomspace(60.0, 1e8, 25)
    rp = np.array([r * abs(O.scf_phi(p, tab, *(r * d))) for r in rs])
    rg = np.array([r * r * np.linalg.norm(O.scf_accel(p, tab, *(r * d))) for r in rs])
    assert rp.max() < 2.0 * rp[0] and rg.max() < 3.0 * rg[0]
    assert np.all(np.isfinite(rp)) and np.all(np.isfinite(rg))


def test_particles_with_a_non_finite_radius_add_nothing():
    rng = np.random.default_rng(17)
    P, parts = _cloud(rng, 300, 0.0, 10.0)
    p = _pot(lmax=2, nr=10)
    tab = O.scf_table(p, parts)
    bad = {k: np.append(v, [np.nan, np.inf]) for k, v in parts.items()}
    u = np.ones(302) * 302 / 300  # the same mass per finite particle
    assert np.allclose(O.scf_table(p, bad, u), tab, rtol=1e-13, atol=0)


@pytest.mark.parametrize("lmax", [0, 4])
def test_hernquist_realization_reproduces_the_analytic_potential(lmax):
    """10^5 particles: about 800 lie inside r = 0.1, so the force there is
    good to a few per cent (shot noise, more of it in the l > 0 terms)."""
    parts = workload(2).initial_particles(n=100_000, seed=12)
    p = _pot(lmax=lmax, nr=40, rmin=0.01, rmax=200.0)
    tab = O.scf_table(p, parts, nthreads=8)
    rng = np.random.default_rng(13)
    for r in (0.1, 0.5, 1.0, 3.0, 10.0):
        for d in _dirs(rng, 3):
            X = r * d
            phi = O.scf_phi(p, tab, *X)
            assert abs(phi + 1.0 / (r + 1.0)) < 0.01 / (r + 1.0), r
            g = O.scf_accel(p, tab, *X)
            ga = O.accel(BASE, *X)
            tol = (0.04 if lmax == 0 else 0.2) if r < 0.3 else 0.03
            assert np.linalg.norm(g - ga) < tol * np.linalg.norm(ga), r


def test_fit_steps_in_the_self_consistent_potential():
    """A Hernquist equilibrium stays in equilibrium in its own potential: the
    relaxation run keeps chi^2 small against targets from its start, close to the
    run in the analytic potential, and the node table follows the particles."""
    wl = workload(1)
    parts = wl.initial_particles(n=4000, seed=14)
    Y = O.deposit(parts, np.ones(4000), wl.layout, mass=wl.params["mass"])
    sig = 0.05 * np.abs(Y) + 1e-3
    runs = {}
    for name, pot in (("analytic", wl.potential.as_dict()),
                      ("scf", dict(wl.potential.as_dict(), scf_lmax=2, scf_nr=20, scf_rmin=0.02,
                                   scf_rmax=50.0, scf_every=5))):
        o = O.OracleFit(pot, wl.layout, wl.params, parts, Y, sig, nthreads=4)
        t0 = o.scf.copy()
        hist = o.step(20, correct=False)
        runs[name] = (hist, o)
        if name == "scf":
            assert o.m.tstep == 20
            again = O.scf_table(pot, o.arr, o.arr["u"], mass=wl.params["mass"]).reshape(-1)
            assert np.array_equal(o.scf, again)  # rebuilt at step 20 from the current state
            assert not np.array_equal(o.scf, t0)
    a, s = runs["analytic"][0], runs["scf"][0]
    assert np.all(s < 5.0 * a + 1.0)
