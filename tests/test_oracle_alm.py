"""Pins of the oracle's spherical-harmonic density observables a_lm,k with
cloud-in-cell radial weights (Sec. 3.3, eq. alm).

The spherical harmonics are checked against scipy's independent
implementation; the deposit against a quadrature that integrates products
of harmonics exactly (orthonormality), the cloud-in-cell weights against
their linear form and mass conservation, and the whole against rotation
invariance of the power per degree l.
"""

import numpy as np
import pytest
import scipy.special as sps

from oracle import oracle as O


def _layout(n_r=8, l_max=4, kin="none", n_R=0, gh_nmax=0):
    return dict(n_r=n_r, r_min=0.1, r_max=10.0, n_R=n_R, R_min=0.1, R_max=10.0, kin=kin,
                gh_nmax=gh_nmax, n_v=0, v_min=0.0, v_max=0.0, dens="alm", l_max=l_max)


def _mesh(lay):
    k = np.arange(lay["n_r"])
    r = lay["r_min"] * (lay["r_max"] / lay["r_min"]) ** (k / (lay["n_r"] - 1))
    r[0], r[-1] = lay["r_min"], lay["r_max"]
    return r


def _parts(x, y, z):
    zeros = np.zeros_like(x)
    return dict(x=x, y=y, z=z, vx=zeros, vy=zeros, vz=zeros)


def _lm(l, m):
    return l * l + l + m


def test_ylm_matches_scipy():
    rng = np.random.default_rng(11)
    for l in range(0, 9):
        for m in range(-l, l + 1):
            for _ in range(4):
                th = np.arccos(rng.uniform(-1, 1))
                ph = rng.uniform(-np.pi, np.pi)
                Y = sps.sph_harm_y(l, abs(m), th, ph)
                ref = Y.real if m == 0 else np.sqrt(2) * (Y.real if m > 0 else Y.imag)
                assert abs(O.ylm(l, m, np.cos(th), ph) - ref) < 1e-13, (l, m)


def test_plm_special_values():
    # P_l(1) = 1, P_l^m(1) = 0 for m > 0, P_1^1(x) = -sqrt(1 - x^2) (Condon-Shortley)
    for l in range(0, 9):
        assert abs(O.plm(l, 0, 1.0) - 1.0) < 1e-13
        for m in range(1, l + 1):
            assert abs(O.plm(l, m, 1.0)) < 1e-13
    for x in (-0.7, 0.0, 0.3):
        assert abs(O.plm(1, 1, x) + np.sqrt(1 - x * x)) < 1e-14
        assert abs(O.plm(2, 0, x) - 0.5 * (3 * x * x - 1)) < 1e-14


def _sphere_quadrature(l_max):
    """Nodes and weights integrating polynomials of degree <= 2 l_max + 1 in
    cos(theta) times trigonometric polynomials of order <= 2 l_max + 1 in phi
    exactly over the unit sphere."""
    ct, wt = np.polynomial.legendre.leggauss(l_max + 2)
    nphi = 2 * l_max + 3
    ph = 2 * np.pi * np.arange(nphi) / nphi
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    W = np.outer(wt, np.full(nphi, 2 * np.pi / nphi))
    return CT.ravel(), PH.ravel(), W.ravel()


@pytest.mark.parametrize("l_max", [0, 2, 4])
def test_alm_orthonormality_on_a_mesh_radius(l_max):
    """Particles on the sphere r = r_k at a quadrature, weighted by the
    quadrature weight times Y_l'm', deposit a_lm,k = delta_ll' delta_mm' and
    nothing at the other mesh radii."""
    lay = _layout(l_max=l_max)
    r = _mesh(lay)
    k = 3
    ct, ph, w = _sphere_quadrature(l_max)
    st = np.sqrt(1 - ct * ct)
    x, y, z = r[k] * st * np.cos(ph), r[k] * st * np.sin(ph), r[k] * ct
    nlm = (l_max + 1) ** 2
    for lp in range(l_max + 1):
        for mp in range(-lp, lp + 1):
            u = w * np.array([O.ylm(lp, mp, c, p) for c, p in zip(ct, ph)])
            a = O.deposit(_parts(x, y, z), u, lay, mass=len(u), n_norm=len(u))
            a = a.reshape(lay["n_r"], nlm)
            expect = np.zeros(nlm)
            expect[_lm(lp, mp)] = 1.0
            assert np.max(np.abs(a[k] - expect)) < 1e-12, (lp, mp)
            others = np.delete(a, k, axis=0)
            assert np.max(np.abs(others)) < 1e-12


def test_cic_weights_are_linear_in_r_and_conserve_mass():
    lay = _layout(l_max=2)
    r = _mesh(lay)
    nlm = 9
    y00 = 0.5 / np.sqrt(np.pi)
    k = 4
    for t in (0.0, 0.25, 0.6, 0.999):
        rr = r[k] + t * (r[k + 1] - r[k])
        a = O.deposit(_parts(np.array([0.0]), np.array([0.0]), np.array([rr])), np.ones(1), lay)
        a = a.reshape(lay["n_r"], nlm)
        assert abs(a[k, 0] - (1 - t) * y00) < 1e-12
        assert abs(a[k + 1, 0] - t * y00) < 1e-12
        # on the z axis only m = 0 is non-zero: Y_l0(1) = sqrt((2l+1)/4pi)
        for l in (1, 2):
            assert abs(a[k, _lm(l, 0)] - (1 - t) * np.sqrt((2 * l + 1) / (4 * np.pi))) < 1e-12
    # mass: sum over the mesh of a_00,k equals Y_00 times the mass inside the
    # mesh; particles outside [r_0, r_last) deposit nothing
    rng = np.random.default_rng(3)
    n = 4000
    rad = np.exp(rng.uniform(np.log(0.02), np.log(30.0), n))
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    x, y, z = (rad[:, None] * v).T
    u = rng.uniform(0.5, 1.5, n)
    a = O.deposit(_parts(x, y, z), u, lay, mass=n, n_norm=n).reshape(lay["n_r"], nlm)
    inside = (rad >= r[0]) & (rad < r[-1])
    assert abs(a[:, 0].sum() - y00 * u[inside].sum()) < 1e-10 * u.sum()


def test_alm_power_per_degree_is_rotation_invariant():
    """sum_m a_lm,k^2 does not change when every particle is rotated by the
    same rotation: a wrong sign or normalization of one order m breaks it."""
    lay = _layout(n_r=6, l_max=4)
    rng = np.random.default_rng(5)
    n = 300
    rad = np.exp(rng.uniform(np.log(0.2), np.log(8.0), n))
    v = rng.normal(size=(n, 3)) * np.array([1.0, 0.6, 0.3])
    v /= np.linalg.norm(v, axis=1)[:, None]
    P = rad[:, None] * v
    u = rng.uniform(0.2, 2.0, n)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    Q = P @ q.T
    a = O.deposit(_parts(*P.T), u, lay).reshape(lay["n_r"], 25)
    b = O.deposit(_parts(*Q.T), u, lay).reshape(lay["n_r"], 25)
    for l in range(5):
        sl = slice(l * l, (l + 1) * (l + 1))
        pa = (a[:, sl] ** 2).sum(axis=1)
        pb = (b[:, sl] ** 2).sum(axis=1)
        assert np.allclose(pa, pb, rtol=1e-10, atol=1e-14), l
        if l > 0:  # the anisotropic set has power beyond l = 0
            assert pa.max() > 1e-6


def test_alm_layout_and_kinematic_offset():
    lay = _layout(n_r=5, l_max=3, kin="gh", n_R=4, gh_nmax=4)
    assert O.J_of(lay) == 5 * 16 + 4 * 4
    K = O.kernels(lay, 0.7, 0.2, 0.4, 0.1, V_p=np.zeros(4), sigma_p=np.ones(4))
    dens = [j for j in K if j < 80]
    kin = [j for j in K if j >= 80]
    assert len(dens) == 2 * 16 and len(kin) == 4
    # the GH entries of the annulus of R = sqrt(0.53) start at 80 + 4 p
    R = np.hypot(0.7, 0.2)
    e = 0.1 * 100.0 ** (np.arange(5) / 4)
    p = int(np.searchsorted(e, R, side="right") - 1)
    assert sorted(kin) == [80 + 4 * p + n for n in range(4)]
