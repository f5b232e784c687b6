"""Pins of the oracle's prior-grid options for rotating models (Sec. 5):
cells split by the sign of L_z, and energy bins linear in exp(E)."""

import numpy as np

from oracle import oracle as O
from workloads import workload


def _wl():
    return workload(2)


def _parts(n=20_000, seed=41):
    return _wl().initial_particles(n=n, seed=seed)


def test_lz_split_puts_retrograde_particles_in_the_second_grid():
    wl = _wl()
    p = _parts()
    c0, E0, x0 = O.cells(wl.potential, wl.params, p)
    c1, E1, x1 = O.cells(wl.potential, dict(wl.params, cells=1), p)
    half = wl.params["n_E"] * wl.params["n_x"]
    lz = p["x"] * p["vy"] - p["y"] * p["vx"]
    assert np.array_equal(c1, c0 + np.where(lz < 0, half, 0))
    assert np.array_equal(E0, E1) and np.array_equal(x0, x1)
    assert O.n_cells(dict(wl.params, cells=1)) == 2 * half
    # an isotropic model fills both senses about equally
    assert 0.45 < np.mean(lz < 0) < 0.55


def _cell_of_energy(pot, par, E):
    """Cells of particles at r = 1 on a circle in the x-y plane with speeds
    chosen so that their energies are E (velocity along +y: L_z > 0)."""
    phi1 = O.phi(pot, 1.0)
    v = np.sqrt(2.0 * (E - phi1))
    n = E.size
    parts = dict(x=np.ones(n), y=np.zeros(n), z=np.zeros(n), vx=np.zeros(n), vy=v, vz=np.zeros(n))
    c, Eo, _ = O.cells(pot, par, parts)
    assert np.allclose(Eo, E, rtol=0, atol=1e-12)
    return c // par["n_x"]


def test_exp_energy_bins_follow_their_edges_and_narrow_outward():
    wl = _wl()
    par = dict(wl.params, n_E=12, n_x=4, cells=2)
    lo, hi = par["E_lo"], par["E_hi"]
    phi1 = O.phi(wl.potential, 1.0)
    # edges E_k = ln(exp E_lo + k (exp E_hi - exp E_lo) / n_E)
    k = np.arange(1, par["n_E"])
    edges = np.log(np.exp(lo) + k * (np.exp(hi) - np.exp(lo)) / par["n_E"])
    ok = edges > phi1 + 1e-6   # reachable at r = 1
    eps = 1e-9
    above = _cell_of_energy(wl.potential, par, edges[ok] + eps)
    below = _cell_of_energy(wl.potential, par, edges[ok] - eps)
    assert np.array_equal(above, k[ok]) and np.array_equal(below, k[ok] - 1)
    # bins are narrower in E toward E_hi (finer sampling of the outer DF)
    w = np.diff(np.concatenate([[lo], edges, [hi]]))
    assert np.all(np.diff(w) < 0)
    # monotone in E and reaching the last bin
    Es = np.linspace(phi1 + 1e-6, -1e-6, 2000)
    kk = _cell_of_energy(wl.potential, par, Es)
    assert np.all(np.diff(kk) >= 0) and kk[-1] == par["n_E"] - 1


def test_mpr_with_the_split_keeps_the_two_senses_of_rotation_apart():
    """Weights 2 on prograde and 1 on retrograde particles: with the split the
    refreshed priors are exactly the mean weight of each sense; without it
    they mix both."""
    wl = _wl()
    p = _parts(n=40_000, seed=43)
    lz = p["x"] * p["vy"] - p["y"] * p["vx"]
    u = np.where(lz >= 0, 2.0, 1.0)
    J = wl.J
    Y, sig = np.ones(J), np.ones(J)
    for cells, mixed in ((1, False), (0, True)):
        par = dict(wl.params, cells=cells)
        o = O.OracleFit(wl.potential, wl.layout, par, p, Y, sig, V_p=np.zeros(30),
                        sigma_p=np.ones(30), u=u, nthreads=4)
        o.refresh_priors()
        uh = o.arr["uhat"]
        if not mixed:
            assert np.array_equal(uh[lz >= 0], np.full(np.sum(lz >= 0), 2.0))
            assert np.array_equal(uh[lz < 0], np.full(np.sum(lz < 0), 1.0))
        else:
            inner = (uh > 1.0) & (uh < 2.0)
            assert inner.mean() > 0.9
