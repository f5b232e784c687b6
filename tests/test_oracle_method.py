"""Pins of the oracle's time smoothing, residuals, force of change and moving
priors (no GPU).

* smoothing (eq. myts): a step function switched on at t = 0 and the
  discrete convolution of the exponential kernel with a piecewise-constant y;
* residuals and chi^2 (eqs. delta, chi) on a hand-worked J = 3 case;
* force of change (eq. modFOC) equals the gradient of the merit function
  F = -chi^2/2 + mu S (eq. SF) for both entropies (eqs. entropy, S+), by
  finite differences of F;
* entropy relaxation alone: ln(u/uhat) shrinks by (1 - eps mu dt) per step
  (S+), and towards uhat/e for the weight entropy (Sec. 2.2);
* zero forcing leaves the weights bit-identical;
* moving priors (Sec. 2.3.1): cell averages conserve the weight sum, are a
  projection, reproduce equal in-cell weights, and the (E, x) cells agree
  with an independent closed-form computation.
"""

import math

import numpy as np
import pytest

from workloads import make_layout, make_params, make_potential, rng, sample_hernquist_isotropic

POT = make_potential()


def _fit(oracle, parts, lay, par, Y, sig, **kw):
    return oracle.OracleFit(POT, lay, par, parts, Y, sig, **kw)


@pytest.fixture(scope="module")
def small():
    return sample_hernquist_isotropic(rng(77), 3000)


def test_smoothing_step_response(oracle, small):
    n = small["x"].size
    lay = make_layout(1, 1e-9, 1e9)
    par = make_params(POT, dt=0.01, alpha=2.1)
    f = _fit(oracle, small, lay, par, [0.5], [1.0])
    y = f.yraw[0]
    f.ytilde[:] = 0.0                          # y switched on at t = 0
    f.step(40, correct=False)
    assert f.ytilde[0] == pytest.approx(y * (1.0 - math.exp(-2.1 * 0.01 * 40)), rel=1e-13)
    assert f.yraw[0] == y


def test_smoothing_is_exponential_kernel_convolution(oracle, small):
    lay = make_layout(12, 0.1, 10.0)
    par = make_params(POT, dt=0.02, alpha=3.0)
    J = 12
    f = _fit(oracle, small, lay, par, np.zeros(J), np.ones(J))
    y0 = f.ytilde.copy()
    ys = []
    for _ in range(60):
        f.step(1, correct=False)
        ys.append(f.yraw.copy())
    ys = np.array(ys)
    n = len(ys)
    a, dt = 3.0, 0.02
    # ytilde(t_n) = alpha int_0^inf y(t_n - tau) e^{-alpha tau} d tau with y = y_m on
    # (t_{m-1}, t_m] and y = y_0 before t = 0
    conv = math.exp(-a * dt * n) * y0
    for m in range(1, n + 1):
        w = math.exp(-a * dt * (n - m)) - math.exp(-a * dt * (n - m + 1))
        conv = conv + w * ys[m - 1]
    np.testing.assert_allclose(f.ytilde, conv, rtol=1e-12, atol=1e-16)


def test_chi2_hand_worked(oracle):
    # three particles, one per log bin [1,2), [2,4), [4,8), mass 3 => w = 1 each
    parts = dict(x=np.array([1.5, 3.0, 6.0]), y=np.zeros(3), z=np.zeros(3),
                 vx=np.zeros(3), vy=np.zeros(3), vz=np.zeros(3))
    lay = make_layout(3, 1.0, 8.0)
    par = make_params(POT, mass=3.0)
    f = _fit(oracle, parts, lay, par, [0.0, 2.0, 4.0], [1.0, 1.0, 2.0])
    np.testing.assert_array_equal(f.yraw, [1.0, 1.0, 1.0])
    np.testing.assert_array_equal(f.delta, [1.0, -1.0, -1.5])
    assert f.chi2 == 4.25


@pytest.mark.parametrize("entropy", ["mpr", "gwr"])
def test_force_of_change_is_merit_gradient(oracle, entropy):
    parts = sample_hernquist_isotropic(rng(5), 40)
    n = 40
    lay = make_layout(5, 0.1, 10.0, 3, 0.1, 10.0, "v2")
    J = 8
    g = np.random.default_rng(1)
    u0 = g.uniform(0.5, 1.5, n)
    uh = g.uniform(0.5, 1.5, n)
    mu, eps, dt = 0.3, 0.7, 0.01
    par = make_params(POT, dt=dt, eps=eps, mu=mu, entropy=entropy, prior_every=0)
    y_of = lambda u: oracle.deposit(parts, u, lay)
    y0 = y_of(u0)
    Y = y0 * g.uniform(0.7, 1.3, J)
    sig = np.abs(y0) * g.uniform(0.05, 0.2, J) + 1e-3

    def F(u):
        d = (y_of(u) - Y) / sig
        if entropy == "mpr":
            S = -np.sum(u * (np.log(u / uh) - 1.0))
        else:
            S = -np.sum(u * np.log(u / uh))
        return -0.5 * np.sum(d * d) + mu * S

    f = _fit(oracle, parts, lay, par, Y, sig, u=u0, uhat=uh)
    f.step(1)
    G = np.log(f.arr["u"] / u0) / (eps * dt)
    grad = np.empty(n)
    for i in range(n):
        h = 1e-6 * u0[i]
        up, um = u0.copy(), u0.copy()
        up[i] += h
        um[i] -= h
        grad[i] = (F(up) - F(um)) / (2 * h)
    np.testing.assert_allclose(G, grad, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("entropy", ["mpr", "gwr"])
def test_entropy_relaxation_closed_form(oracle, small, entropy):
    n = small["x"].size
    g = np.random.default_rng(2)
    u0 = g.uniform(0.2, 3.0, n)
    uh = g.uniform(0.5, 2.0, n)
    eps, mu, dt = 0.5, 0.8, 0.01
    par = make_params(POT, dt=dt, eps=eps, mu=mu, entropy=entropy, prior_every=0)
    lay = make_layout(10, 0.05, 20.0)
    # sigma so large that Delta / sigma underflows to zero: entropy term only
    f = _fit(oracle, small, lay, par, np.zeros(10), np.full(10, 1e300), u=u0, uhat=uh)
    steps = 50
    f.step(steps)
    shift = 0.0 if entropy == "mpr" else 1.0     # S+ -> uhat, weight entropy -> uhat / e
    lhs = np.log(f.arr["u"] / uh) + shift
    rhs = (np.log(u0 / uh) + shift) * (1.0 - eps * mu * dt) ** steps
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-13)


def test_zero_forcing_keeps_weights_bit_identical(oracle, small):
    n = small["x"].size
    g = np.random.default_rng(3)
    u0 = g.uniform(0.2, 3.0, n)
    lay = make_layout(4, 1e6, 1e7, 3, 1e6, 1e7, "v2")   # no particle ever reaches it
    par = make_params(POT, prior_every=0)
    f = _fit(oracle, small, lay, par, np.ones(7), np.ones(7), u=u0, uhat=u0)
    f.step(30)
    np.testing.assert_array_equal(f.arr["u"], u0)


def test_prior_refresh_conserves_sum_and_is_a_projection(oracle, small):
    n = small["x"].size
    g = np.random.default_rng(4)
    u0 = g.uniform(0.2, 3.0, n)
    par = make_params(POT, n_E=20, n_x=10)
    lay = make_layout(10, 0.05, 20.0)
    f = _fit(oracle, small, lay, par, np.zeros(10), np.ones(10), u=u0)
    f.refresh_priors()
    uh = f.arr["uhat"].copy()
    assert uh.sum() == pytest.approx(u0.sum(), rel=1e-13)
    # averaging the averages again changes nothing
    f.arr["u"][:] = uh
    f.refresh_priors()
    np.testing.assert_allclose(f.arr["uhat"], uh, rtol=1e-14)
    # weights that are equal inside each cell are their own priors
    cell, _, _ = oracle.cells(POT, par, small)
    f.arr["u"][:] = 1.0 + (cell % 7) * 0.25
    f.refresh_priors()
    np.testing.assert_allclose(f.arr["uhat"], 1.0 + (cell % 7) * 0.25, rtol=1e-15)


def test_cells_match_independent_closed_form(oracle, small):
    par = make_params(POT, n_E=20, n_x=10)
    cell, E, xc = oracle.cells(POT, par, small)
    x, y, z = small["x"], small["y"], small["z"]
    vx, vy, vz = small["vx"], small["vy"], small["vz"]
    r = np.sqrt(x * x + y * y + z * z)
    E2 = 0.5 * (vx * vx + vy * vy + vz * vz) - 1.0 / (r + 1.0)
    L = np.linalg.norm(np.cross(np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1)), axis=1)
    s = (1.0 + np.sqrt(1.0 - 8.0 * E2)) / (-4.0 * E2)      # Hernquist circular orbit
    rc = s - 1.0
    Lc = np.sqrt(rc) * rc / (rc + 1.0)
    x2 = L / Lc
    k = np.clip(np.floor((E2 + 1.0) / 1.0 * 20), 0, 19).astype(int)
    l_ = np.clip(np.floor(x2 * 10), 0, 9).astype(int)
    np.testing.assert_allclose(E, E2, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(xc, x2, rtol=1e-9)
    tE = (E2 + 1.0) * 20
    tx = x2 * 10
    safe = (np.abs(tE - np.round(tE)) > 1e-6) & (np.abs(tx - np.round(tx)) > 1e-6)
    assert safe.mean() > 0.99
    np.testing.assert_array_equal(cell[safe], (k * 10 + l_)[safe])
