"""Pins of the oracle's prior-grid smoothing (Sec. 2.3.2, eq. smooth_grid):
thin-plate penalized least squares on the (E, x) grid with lambda chosen by
generalized cross validation. Every check uses an independent route: the
analytic eigenvalues of the reflecting-boundary Laplacian, the explicit
finite-difference thin-plate sum, exact invariants, and the statistical
behaviour that GCV is known for."""

import numpy as np
import pytest

from workloads import make_params, make_potential


def _par(nE, nx):
    return make_params(make_potential(), n_E=nE, n_x=nx)


def _h(par):
    return (par["E_hi"] - par["E_lo"]) / par["n_E"], 1.0 / par["n_x"]


def _thin_plate_energy(w, hE, hx):
    """sum over cells of (d2w/dE2)^2 + (d2w/dx2)^2 with reflected ghost
    cells, plus 2 (d2w/dEdx)^2 at every interior cell corner."""
    g = np.pad(w, 1, mode="edge")
    dEE = (g[2:, 1:-1] - 2 * g[1:-1, 1:-1] + g[:-2, 1:-1]) / hE ** 2
    dxx = (g[1:-1, 2:] - 2 * g[1:-1, 1:-1] + g[1:-1, :-2]) / hx ** 2
    dEx = (w[1:, 1:] - w[1:, :-1] - w[:-1, 1:] + w[:-1, :-1]) / (hE * hx)
    return float((dEE ** 2).sum() + (dxx ** 2).sum() + 2 * (dEx ** 2).sum())


def test_constant_grid_and_mean_are_preserved(oracle):
    par = _par(12, 7)
    w, lam = oracle.smooth_grid(par, np.full(12 * 7, 1.7))
    np.testing.assert_allclose(w, 1.7, rtol=1e-12)
    g = np.random.default_rng(1).uniform(0.5, 1.5, 12 * 7)
    w, lam = oracle.smooth_grid(par, g)
    assert lam > 0
    assert abs(w.sum() / g.sum() - 1) < 1e-12


@pytest.mark.parametrize("axis,j", [(0, 1), (0, 5), (1, 2), (1, 6)])
def test_single_cosine_mode_is_damped_by_its_eigenvalue(oracle, axis, j):
    """A cos(pi j (i + 1/2) / n) pattern along one axis is an eigenvector of
    the reflecting-boundary Laplacian with eigenvalue -4 sin^2(pi j / 2n)/h^2,
    so the smoother scales it by exactly 1 / (1 + lambda Gamma^2)."""
    nE, nx = 10, 8
    par = _par(nE, nx)
    hE, hx = _h(par)
    n, h = (nE, hE) if axis == 0 else (nx, hx)
    mode = np.cos(np.pi * j * (np.arange(n) + 0.5) / n)
    pat = mode[:, None] * np.ones((1, nx)) if axis == 0 else np.ones((nE, 1)) * mode[None, :]
    g = 3.0 + 0.4 * pat
    w, lam = oracle.smooth_grid(par, g.reshape(-1))
    gamma = 4 * np.sin(np.pi * j / (2 * n)) ** 2 / h ** 2
    expect = 3.0 + 0.4 * pat / (1 + lam * gamma ** 2)
    np.testing.assert_allclose(w.reshape(nE, nx), expect, rtol=1e-9, atol=1e-12)


def test_penalty_is_the_finite_difference_thin_plate_energy(oracle):
    """The minimizer satisfies (w - w0) + lambda P w = 0, so w^T P w =
    w^T (w0 - w) / lambda; it must equal the explicit thin-plate sum."""
    nE, nx = 9, 6
    par = _par(nE, nx)
    hE, hx = _h(par)
    rng = np.random.default_rng(7)
    E = np.linspace(0, 1, nE)[:, None]
    x = np.linspace(0, 1, nx)[None, :]
    g = 2 + np.sin(3 * E) * np.cos(2 * x) + 0.2 * rng.standard_normal((nE, nx))
    w, lam = oracle.smooth_grid(par, g.reshape(-1))
    wPw = float(w @ (g.reshape(-1) - w)) / lam
    tp = _thin_plate_energy(w.reshape(nE, nx), hE, hx)
    assert abs(wPw / tp - 1) < 1e-6, (wPw, tp)


def test_gcv_behaviour(oracle):
    nE, nx = 16, 8
    par = _par(nE, nx)
    rng = np.random.default_rng(11)
    E = (np.arange(nE) + 0.5)[:, None] / nE
    x = (np.arange(nx) + 0.5)[None, :] / nx
    truth = 1 + 0.5 * np.exp(-((E - 0.4) ** 2) / 0.05) * (0.5 + x)
    # smooth, noise-free data: almost interpolated
    w, _ = oracle.smooth_grid(par, truth.reshape(-1))
    assert np.abs(w - truth.reshape(-1)).max() < 0.02 * truth.max()
    # pure noise about a constant: pulled towards the mean
    noise = 1 + 0.1 * rng.standard_normal(nE * nx)
    w, _ = oracle.smooth_grid(par, noise)
    assert np.std(w) < 0.3 * np.std(noise)
    # smooth signal plus noise: closer to the truth than the data
    data = truth + 0.05 * rng.standard_normal((nE, nx))
    w, _ = oracle.smooth_grid(par, data.reshape(-1))
    err_w = np.sqrt(np.mean((w - truth.reshape(-1)) ** 2))
    err_d = np.sqrt(np.mean((data - truth) ** 2))
    assert err_w < 0.7 * err_d, (err_w, err_d)


def test_refresh_uses_the_smoothed_cell_means(oracle):
    from workloads import workload
    wl = workload(1)
    n = 3000
    parts = wl.initial_particles(n=n, seed=5)
    par = dict(wl.params, smooth=1, n_E=8, n_x=5)
    J = oracle.J_of(wl.layout)
    f = oracle.OracleFit(wl.potential, wl.layout, par, parts, np.ones(J), np.ones(J))
    u = np.random.default_rng(2).uniform(0.5, 1.5, n)
    f.arr["u"][:] = u
    f.refresh_priors()
    c, _, _ = oracle.cells(wl.potential, par, f.arr)
    C = par["n_E"] * par["n_x"]
    cnt = np.bincount(c, minlength=C)
    mean = np.where(cnt > 0, np.bincount(c, weights=u, minlength=C) / np.maximum(cnt, 1), 1.0)
    smooth, _ = oracle.smooth_grid(par, mean)
    np.testing.assert_allclose(f.arr["uhat"], smooth[c], rtol=1e-13)
    np.testing.assert_allclose(f.ucell, smooth, rtol=1e-13)
