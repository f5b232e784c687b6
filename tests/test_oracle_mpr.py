"""Moving priors against a generating DF the particles can represent exactly
(Sec. 2.3.1 and Sec. 4.1: with moving priors the fit recovers the generating
distribution function; a fixed prior biases it towards the prior).

The target is a tracer population in the fixed Hernquist potential whose DF
is the isotropic Hernquist DF times exp(beta * binding energy): the same
particle set with weights u_true proportional to exp(beta * binding energy)
reproduces it exactly, so the cell masses of u_true on the (E, L/L_c) grid are
the truth. Data: 20 radial mass bins and 12 annuli x 16 LOS velocity bins of
that weighted set, 1 % noise, errors floored at twice the Poisson error of the
model. With a strong entropy term (mu = 1 in the weight units u = N w) the
moving-prior fit must reach the truth on the grid, the fixed-prior S+ fit and
the GWR entropy must not.
"""

import os

import numpy as np
import pytest

from workloads import make_layout, make_params, make_potential, rng, sample_hernquist_isotropic

N = 20_000
STEPS = 1600
BETA = 2.0


def _delta_grid(O, pot, par, parts, u, m_true):
    m = O.cell_mass(pot, par, parts, u)
    k = m_true > 0
    return float(np.sum(np.abs(m[k] - m_true[k])) / m_true[k].sum())


@pytest.fixture(scope="module")
def mpr_runs(oracle):
    O = oracle
    nth = min(8, os.cpu_count() or 1)
    pot = make_potential()
    ic = sample_hernquist_isotropic(rng(21), N)
    x, y, z, vx, vy, vz = (ic[k] for k in ("x", "y", "z", "vx", "vy", "vz"))
    r = np.sqrt(x * x + y * y + z * z)
    eb = pot.psi(r) - 0.5 * (vx * vx + vy * vy + vz * vz)
    ratio = np.exp(BETA * eb)
    u_true = N * ratio / ratio.sum()
    lay = make_layout(20, 0.05, 20.0, 12, 0.05, 10.0, "losvd", n_v=16, v_min=-2.0, v_max=2.0)
    Yt = O.deposit(ic, u_true, lay, nthreads=nth)
    w0 = 1.0 / N
    sig = np.sqrt((0.01 * Yt) ** 2 + 4 * w0 * np.abs(Yt)) + w0
    Y = Yt + 0.01 * np.abs(Yt) * rng(22).standard_normal(Yt.size)
    grid = make_params(pot, n_E=20, n_x=10)
    m_true = O.cell_mass(pot, grid, ic, u_true)
    out = {"initial": _delta_grid(O, pot, grid, ic, np.ones(N), m_true)}
    for name, entropy, every in (("mpr", "mpr", 25), ("fixed", "mpr", 0), ("gwr", "gwr", 25)):
        par = make_params(pot, dt=0.01, eps=0.5, mu=1.0, entropy=entropy, n_E=20, n_x=10,
                          prior_every=every)
        f = O.OracleFit(pot, lay, par, ic, Y, sig, nthreads=nth)
        h = f.step(STEPS)
        out[name] = (_delta_grid(O, pot, grid, f.arr, f.arr["u"], m_true), h[-1] / f.J)
    return out


def test_moving_priors_recover_the_generating_df(mpr_runs):
    d0 = mpr_runs["initial"]
    d_mpr, chi_mpr = mpr_runs["mpr"]
    assert d0 > 0.3
    assert d_mpr < 0.25 * d0, mpr_runs
    assert chi_mpr < 1.0, mpr_runs


def test_fixed_priors_bias_the_fit_towards_the_prior(mpr_runs):
    d_mpr, _ = mpr_runs["mpr"]
    d_fix, chi_fix = mpr_runs["fixed"]
    d_gwr, chi_gwr = mpr_runs["gwr"]
    assert d_mpr < 0.5 * d_fix, mpr_runs
    assert d_mpr < d_gwr, mpr_runs
    assert chi_fix > 2.0 and chi_gwr > 2.0, mpr_runs
