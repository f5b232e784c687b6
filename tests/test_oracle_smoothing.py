"""Pins of the oracle's prior-grid smoothing (Sec. 2.3.2, eq. smooth_grid):
thin-plate penalized least squares on the (E, x) grid with lambda chosen by
generalized cross validation.

The paper fixes two limits of the family: a plane for lambda -> infinity and
the data for lambda -> 0. Each check below uses a route independent of the
oracle's dense stencil assembly and Cholesky solve:
* planes are returned unchanged at every lambda (they cost nothing);
* for large lambda the result tends to numpy's least-squares plane;
* the minimizer's penalty w^T P w equals the thin-plate sum written with
  array slices, and it satisfies the normal equations built from that sum;
* the chosen lambda is the first minimum of GCV computed spectrally from a
  numpy eigendecomposition of the penalty (itself built from the slice sum),
  on the same three-stage search grid;
* invariants of a penalty whose null space holds the planes: the mean and
  the first moments in E and x are preserved;
* the statistical behaviour that GCV is known for.
"""

import numpy as np
import pytest

from workloads import make_params, make_potential


def _par(nE, nx, **kw):
    return make_params(make_potential(), n_E=nE, n_x=nx, **kw)


def _h(par):
    return (par["E_hi"] - par["E_lo"]) / par["n_E"], 1.0 / par["n_x"]


def _centres(par):
    nE, nx = par["n_E"], par["n_x"]
    hE, hx = _h(par)
    E = ((np.arange(nE) + 0.5) * hE)[:, None] * np.ones((1, nx))
    x = ((np.arange(nx) + 0.5) * hx)[None, :] * np.ones((nE, 1))
    return E, x


def _thin_plate_energy(w, hE, hx):
    """sum of (d2w/dE2)^2 over the cells with a neighbour on both sides
    along E, of (d2w/dx2)^2 likewise along x, and of 2 (d2w/dEdx)^2 over the
    interior corners of four cells: finite differences only where their
    stencil lies inside the grid."""
    dEE = (w[2:, :] - 2 * w[1:-1, :] + w[:-2, :]) / hE ** 2
    dxx = (w[:, 2:] - 2 * w[:, 1:-1] + w[:, :-2]) / hx ** 2
    dEx = (w[1:, 1:] - w[1:, :-1] - w[:-1, 1:] + w[:-1, :-1]) / (hE * hx)
    return float((dEE ** 2).sum() + (dxx ** 2).sum() + 2 * (dEx ** 2).sum())


def _penalty_matrix(nE, nx, hE, hx):
    """P with w^T P w = the slice-written thin-plate energy, recovered column
    by column from that energy by polarization:
    P_ij = (E(e_i + e_j) - E(e_i - e_j)) / 4."""
    n = nE * nx
    P = np.zeros((n, n))
    I = np.eye(n)
    for i in range(n):
        for j in range(i, n):
            a = _thin_plate_energy((I[i] + I[j]).reshape(nE, nx), hE, hx)
            b = _thin_plate_energy((I[i] - I[j]).reshape(nE, nx), hE, hx)
            P[i, j] = P[j, i] = (a - b) / 4.0
    return P


def _search_grid_first_min(score, plo, phi):
    """The three-stage search on log10(lambda): steps of 0.25 over
    [plo, phi], then 65 points over the two steps around the best, then 65
    points over the two sub-steps around the best; first minimum wins."""
    K1 = int(np.floor((phi - plo) / 0.25)) + 1
    g = [score(10.0 ** (plo + 0.25 * i)) for i in range(K1)]
    best = int(np.argmin(g))
    a = plo + 0.25 * (best - 1 if best > 0 else 0)
    b = plo + 0.25 * (best + 1 if best < K1 - 1 else K1 - 1)
    for stage in range(2):
        pts = [a + (b - a) * j / 64.0 for j in range(65)]
        g = [score(10.0 ** p) for p in pts]
        bi = int(np.argmin(g))
        if stage == 1:
            return 10.0 ** pts[bi], g
        a, b = (a + (b - a) * (bi - 1 if bi > 0 else 0) / 64.0,
                a + (b - a) * (bi + 1 if bi < 64 else 64) / 64.0)


def _range(par):
    hE, hx = _h(par)
    nE, nx = par["n_E"], par["n_x"]
    ghi = (4 / hE ** 2 if nE > 1 else 0) + (4 / hx ** 2 if nx > 1 else 0)
    glo = min([4 * np.sin(np.pi / (2 * n)) ** 2 / h ** 2 for n, h in ((nE, hE), (nx, hx)) if n > 1])
    return -2 * np.log10(ghi) - 4, -2 * np.log10(glo) + 4


@pytest.mark.parametrize("shape", [(20, 10), (16, 8), (9, 6), (3, 7)])
def test_plane_is_returned_unchanged_at_every_lambda(oracle, shape):
    """Every finite difference of the penalty vanishes on a plane, so the
    smoother returns a plane as it is, at the GCV lambda and at any fixed
    lambda across the search range (to the rounding of a Cholesky solve with
    condition number about 1 + lambda G_hi^2)."""
    par = _par(*shape)
    E, x = _centres(par)
    plane = 2.0 + 0.7 * E - 1.3 * x
    w, lam = oracle.smooth_grid(par, plane.reshape(-1))
    np.testing.assert_allclose(w, plane.reshape(-1), rtol=1e-12)
    plo, phi = _range(par)
    hE, hx = _h(par)
    ghi = 4 / hE ** 2 + 4 / hx ** 2
    for p in np.linspace(plo, phi, 9):
        w = oracle.smooth_grid_at(par, plane.reshape(-1), 10.0 ** p)
        tol = 64 * np.finfo(float).eps * (1 + 10.0 ** p * ghi ** 2)
        err = np.abs(w - plane.reshape(-1)).max() / np.abs(plane).max()
        assert err <= tol, (p, err, tol)


@pytest.mark.parametrize("shape", [(20, 10), (16, 8), (9, 6), (3, 7)])
def test_large_lambda_gives_the_least_squares_plane(oracle, shape):
    """lambda -> infinity projects the data onto the planes (the penalty's
    null space): the distance to numpy's least-squares plane falls as
    1/lambda beyond the search range."""
    par = _par(*shape)
    E, x = _centres(par)
    rng = np.random.default_rng(3)
    d = (1 + 0.3 * np.sin(4 * E) * np.cos(3 * x) + 0.1 * rng.standard_normal(E.shape)).reshape(-1)
    A = np.stack([np.ones(d.size), E.reshape(-1), x.reshape(-1)], 1)
    coef, *_ = np.linalg.lstsq(A, d, rcond=None)
    plane = A @ coef
    scale = np.abs(d - plane).max()
    _, phi = _range(par)
    e1 = np.abs(oracle.smooth_grid_at(par, d, 10.0 ** phi) - plane).max() / scale
    e2 = np.abs(oracle.smooth_grid_at(par, d, 10.0 ** (phi + 1)) - plane).max() / scale
    assert e2 < 1e-5, (e1, e2)
    assert e2 < 0.2 * e1, (e1, e2)
    # and far from the data (the mean would be far from the plane too)
    assert np.abs(d.mean() - plane).max() > 10 * e2 * scale


def test_penalty_is_the_finite_difference_thin_plate_energy(oracle):
    """The minimizer satisfies (w - w0) + lambda P w = 0, so w^T P w =
    w^T (w0 - w) / lambda; it must equal the slice-written thin-plate sum,
    and the residual of the normal equations, with P w from that sum by
    polarization, must vanish."""
    nE, nx = 9, 6
    par = _par(nE, nx)
    hE, hx = _h(par)
    rng = np.random.default_rng(7)
    E, x = _centres(par)
    g = (2 + np.sin(3 * E) * np.cos(2 * x) + 0.2 * rng.standard_normal((nE, nx))).reshape(-1)
    w, lam = oracle.smooth_grid(par, g)
    wPw = float(w @ (g - w)) / lam
    tp = _thin_plate_energy(w.reshape(nE, nx), hE, hx)
    assert abs(wPw / tp - 1) < 1e-8, (wPw, tp)
    P = _penalty_matrix(nE, nx, hE, hx)
    res = (w - g) + lam * (P @ w)
    assert np.abs(res).max() < 1e-10 * np.abs(g).max()


@pytest.mark.parametrize("shape,seed", [((9, 6), 1), ((12, 7), 2), ((16, 8), 3), ((7, 11), 4)])
def test_gcv_lambda_is_the_first_minimum_of_the_spectral_score(oracle, shape, seed):
    """GCV by an independent route: with P = Q diag(g) Q^T from numpy's
    eigendecomposition of the slice-written penalty and w^ = Q^T w0,
      |w0 - A w0|^2 = sum (t/(1+t))^2 w^^2,  tr A = sum 1/(1+t),  t = lambda g.
    The oracle's lambda must be the first minimum of that score on the same
    three-stage grid (or score within rounding of it)."""
    nE, nx = shape
    par = _par(nE, nx)
    hE, hx = _h(par)
    E, x = _centres(par)
    rng = np.random.default_rng(seed)
    w0 = (1 + 0.4 * np.exp(-((E - 0.5) ** 2) / 0.05) * (0.5 + x)
          + 0.05 * rng.standard_normal((nE, nx))).reshape(-1)
    P = _penalty_matrix(nE, nx, hE, hx)
    g, Q = np.linalg.eigh(P)
    g = np.maximum(g, 0.0)
    wh = Q.T @ w0
    n = w0.size

    def score(lam):
        t = lam * g
        r = t / (1 + t)
        return (np.sum((r * wh) ** 2) / n) / (np.sum(r) / n) ** 2

    plo, phi = _range(par)
    lam_np, last = _search_grid_first_min(score, plo, phi)
    _, lam = oracle.smooth_grid(par, w0)
    assert score(lam) <= min(last) * (1 + 1e-9), (lam, lam_np)
    assert lam == pytest.approx(lam_np, rel=2e-3)
    # the smoothed grid is the spectral filter at that lambda
    w, _ = oracle.smooth_grid(par, w0)
    ws = Q @ (wh / (1 + lam * g))
    np.testing.assert_allclose(w, ws, rtol=1e-9, atol=1e-12)


def test_null_space_is_three_planes():
    """The slice-written penalty has exactly the planes as its null space
    (rank n - 3); with values invented beyond the edges (ghost cells equal to
    the edge cells) it would be the constants only (rank n - 1)."""
    par = _par(10, 7)
    hE, hx = _h(par)
    P = _penalty_matrix(10, 7, hE, hx)
    g = np.linalg.eigvalsh(P)
    assert np.sum(g < 1e-9 * g.max()) == 3


def test_mean_and_first_moments_are_preserved(oracle):
    """(I + lambda P) fixes every plane, and P is symmetric, so the smoother
    keeps the projection of the data onto the planes: the sum of the grid
    and its first moments in E and x."""
    par = _par(12, 7)
    w, lam = oracle.smooth_grid(par, np.full(12 * 7, 1.7))
    np.testing.assert_allclose(w, 1.7, rtol=1e-12)
    E, x = _centres(par)
    g = np.random.default_rng(1).uniform(0.5, 1.5, 12 * 7)
    w, lam = oracle.smooth_grid(par, g)
    assert lam > 0
    for m in (np.ones(g.size), E.reshape(-1), x.reshape(-1)):
        assert abs((m @ w) / (m @ g) - 1) < 1e-11


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
    # a noisy plane: the edge rows are recovered as well as the interior
    Eg, xg = _centres(par)
    plane = 1 + 0.8 * Eg + 0.5 * xg
    data = plane + 0.05 * rng.standard_normal((nE, nx))
    w, _ = oracle.smooth_grid(par, data.reshape(-1))
    err = np.abs(w.reshape(nE, nx) - plane)
    edge = np.concatenate([err[0], err[-1], err[:, 0], err[:, -1]])
    assert np.sqrt(np.mean(edge ** 2)) < 0.5 * 0.05


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
