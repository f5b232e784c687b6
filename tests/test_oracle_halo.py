"""Pins of the oracle's logarithmic halo, Phi_D = v0^2/2 ln(r0^2 + R^2 +
z^2/q^2) (Sec. 5, eq. log_halo): the force is minus the gradient of the
potential, the flattening acts along z, circular orbits of the pure halo
follow their closed form, and orbits in the flattened halo keep L_z and
their energy."""

import numpy as np

from oracle import oracle as O

HALO = dict(G=1.0, M_star=1.0, a=1.0, upsilon=1.0, M200=0.0, c=0.0, r_s=0.0, v0=0.8, r0=2.5,
            q=0.7)
PURE = dict(HALO, M_star=0.0, q=1.0)


def test_force_is_minus_the_gradient_of_the_potential():
    rng = np.random.default_rng(2)
    h = 1e-5
    for _ in range(20):
        p = rng.normal(size=3) * 3.0
        g = O.accel(HALO, *p)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            d = (O.phi3(HALO, *(p + e)) - O.phi3(HALO, *(p - e))) / (2 * h)
            assert abs(g[k] + d) < 1e-8 * max(1.0, abs(d)), (p, k)


def test_flattening_acts_along_z_only():
    # Phi_D(R, 0) = Phi_D(0, q R); the Hernquist part is off
    pot = dict(HALO, M_star=0.0)
    for R in (0.3, 1.0, 4.0, 20.0):
        assert abs(O.phi3(pot, R, 0.0, 0.0) - O.phi3(pot, 0.0, 0.0, pot["q"] * R)) < 1e-14
        assert abs(O.phi3(pot, R, 0.0, 0.0) - O.phi3(pot, 0.0, R, 0.0)) < 1e-14
        assert abs(O.phi(pot, R) - O.phi3(pot, R, 0.0, 0.0)) < 1e-14
    # the value at the centre: v0^2 ln r0
    assert abs(O.phi3(pot, 0.0, 0.0, 0.0) - pot["v0"] ** 2 * np.log(pot["r0"])) < 1e-14


def test_circular_orbits_of_the_pure_halo():
    """v_c^2 = v0^2 R^2 / (r0^2 + R^2), E_c = Phi + v_c^2/2, L_c = R v_c; the
    rotation curve is flat far out."""
    v0, r0 = PURE["v0"], PURE["r0"]
    for R in (0.1, 1.0, 3.0, 30.0, 300.0):
        vc2 = v0 * v0 * R * R / (r0 * r0 + R * R)
        Ec = 0.5 * v0 * v0 * np.log(r0 * r0 + R * R) + 0.5 * vc2
        assert abs(O.lc(PURE, Ec) - R * np.sqrt(vc2)) < 1e-9 * R * np.sqrt(vc2)
    # every energy above the centre has a circular orbit (no escape)
    assert np.isfinite(O.lc(PURE, 50.0))


def test_orbits_in_the_flattened_halo_keep_lz_and_energy():
    rng = np.random.default_rng(3)
    n = 8
    p = {k: rng.normal(size=n) * s for k, s in (("x", 2.0), ("y", 2.0), ("z", 1.0),
                                                 ("vx", 0.4), ("vy", 0.4), ("vz", 0.4))}

    def energy(q):
        return np.array([0.5 * (q["vx"][i] ** 2 + q["vy"][i] ** 2 + q["vz"][i] ** 2) +
                         O.phi3(HALO, q["x"][i], q["y"][i], q["z"][i]) for i in range(n)])

    def lz(q):
        return q["x"] * q["vy"] - q["y"] * q["vx"]

    E0, L0 = energy(p), lz(p)
    q = O.push(HALO, 0.01, p, 2000)
    assert np.max(np.abs(lz(q) - L0)) < 1e-12 * np.max(np.abs(L0))
    assert np.max(np.abs(energy(q) - E0) / np.abs(E0)) < 1e-4
    # without the halo's z/q^2 the orbit would not keep its energy
    bad = dict(HALO, q=1.0)
    qb = O.push(bad, 0.01, p, 2000)
    assert np.max(np.abs(energy(qb) - E0) / np.abs(E0)) > 1e-3
