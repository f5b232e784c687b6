"""Pins of the oracle's observables (deposit, selection, Gauss-Hermite kernels)
against closed forms, invariants, brute force and a paper-printed value.

* radial mass bins of an equal-weight isotropic Hernquist sample against
  M(r) = M r^2 / (r + a)^2 (multinomial error);
* projected annulus masses against a numerical Abel projection and the
  closed-form M_p(R), and the paper's R_eff = 1.82 a (Sec. 3.1);
* v_z^2 moments in annuli against the isotropic Jeans dispersion;
* virial sums: sum w v_z^2 -> G M^2 / (18 a);
* brute-force re-binning on tiny N and exact weight-sum conservation;
* Gauss-Hermite kernels (eq. lumghn): Hermite polynomials against numpy,
  orthonormality, zero moments of a matched Gaussian, and the first-order
  relations of eq. h1h2.
"""

import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite as npherm
from scipy import integrate

from workloads import hernquist_projected_mass, make_layout, rng, sample_hernquist_isotropic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sample():
    return sample_hernquist_isotropic(rng(1234), 200_000)


def _edges(lo, hi, n):
    return np.array([lo if k == 0 else hi if k == n else lo * (hi / lo) ** (k / n)
                     for k in range(n + 1)])


def _Mr(r):
    return r * r / (r + 1.0) ** 2


def test_radial_bins_match_hernquist_mass_profile(oracle, sample):
    N = sample["x"].size
    lay = make_layout(30, 0.05, 20.0)
    y = oracle.deposit(sample, np.ones(N), lay)
    e = _edges(0.05, 20.0, 30)
    p = np.diff(_Mr(e))
    sd = np.sqrt(p * (1 - p) / N)
    assert np.all(np.abs(y - p) < 5 * sd)
    # fractions inside and beyond the grid (0.23 % inside 0.05, 9.30 % outside 20)
    assert _Mr(0.05) == pytest.approx(0.00227, abs=1e-5)
    assert 1 - _Mr(20.0) == pytest.approx(0.0930, abs=1e-4)
    assert y.sum() == pytest.approx(_Mr(20.0) - _Mr(0.05), abs=5 * math.sqrt(0.1 / N))


def _abel_projected_mass(R):
    """Mass inside projected radius R by integrating the projection of rho."""
    rho = lambda r: 1.0 / (2 * math.pi * r * (r + 1) ** 3)
    # M_p(R) = M_total - mass with projected radius > R
    #        = 1 - int_R^inf 4 pi r^2 rho(r) sqrt(1 - R^2/r^2) dr
    out = integrate.quad(lambda r: 4 * math.pi * r * r * rho(r) * math.sqrt(1 - (R / r) ** 2),
                         R, np.inf, epsabs=1e-14, epsrel=1e-12, limit=400)[0]
    return 1.0 - out


def test_projected_mass_closed_form_against_abel(oracle):
    for R in (0.05, 0.3, 1.0, 1.8153, 5.0, 20.0):
        assert hernquist_projected_mass(R) == pytest.approx(_abel_projected_mass(R), rel=1e-9)


def test_annulus_selection_matches_projected_mass(oracle, sample):
    N = sample["x"].size
    # one LOSVD bin wide enough for every particle: the annulus entry is its mass
    lay = make_layout(1, 1e-9, 1e9, 20, 0.05, 20.0, "losvd", n_v=1, v_min=-10.0, v_max=10.0)
    y = oracle.deposit(sample, np.ones(N), lay)[1:]
    e = _edges(0.05, 20.0, 20)
    p = np.diff([_abel_projected_mass(R) for R in e])
    sd = np.sqrt(p * (1 - p) / N)
    assert np.all(np.abs(y - p) < 5 * sd)


def test_paper_effective_radius(oracle, sample):
    g = {}
    with open(os.path.join(GOLDEN, "hernquist_reff.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                g[k] = float(v)
    Reff, tol = g["R_eff_over_a"], g["R_eff_over_a_abs_tol"]
    # the closed-form half-light radius agrees with the printed one
    from scipy.optimize import brentq
    r_half = brentq(lambda R: _abel_projected_mass(R) - g["half_light_fraction"], 0.5, 5.0)
    assert abs(r_half - Reff) < tol
    # and the oracle's annulus selection puts half the sample inside it
    N = sample["x"].size
    lay = make_layout(1, 1e-9, 1e9, 1, 1e-9, Reff, "losvd", n_v=1, v_min=-10.0, v_max=10.0)
    inside = oracle.deposit(sample, np.ones(N), lay)[1]
    assert inside == pytest.approx(g["half_light_fraction"], abs=0.01)


def _sigma_r2_iso(r):
    """Isotropic Hernquist radial dispersion (G = M = a = 1), closed form."""
    x = r
    return (1.0 / 12.0) * (12 * x * (1 + x) ** 3 * math.log((1 + x) / x)
                           - x / (1 + x) * (25 + 52 * x + 42 * x * x + 12 * x ** 3))


def test_sigma_r2_closed_form_matches_jeans():
    rho = lambda r: 1.0 / (2 * math.pi * r * (r + 1) ** 3)
    for r in (0.05, 0.5, 1.0, 4.0):
        jeans = integrate.quad(lambda s: rho(s) * s * s / (s + 1) ** 2 / s ** 2, r, np.inf,
                               epsabs=0, epsrel=1e-12, limit=400)[0] / rho(r)
        assert _sigma_r2_iso(r) == pytest.approx(jeans, rel=1e-9)


def test_v2_moments_in_annuli_match_jeans(oracle, sample):
    N = sample["x"].size
    lay = make_layout(1, 1e-9, 1e9, 8, 0.1, 10.0, "v2")
    y = oracle.deposit(sample, np.ones(N), lay)[1:]
    e = _edges(0.1, 10.0, 8)
    rho = lambda r: 1.0 / (2 * math.pi * r * (r + 1) ** 3)

    def p_in(R0, r):  # probability that an isotropic direction puts R below R0
        return 1.0 if r <= R0 else 1.0 - math.sqrt(1.0 - (R0 / r) ** 2)

    expect = []
    for k in range(8):
        f = lambda r: 4 * math.pi * r * r * rho(r) * _sigma_r2_iso(r) * (p_in(e[k + 1], r) - p_in(e[k], r))
        # sigma_r2 closed form loses digits at large r: cap the range
        expect.append(integrate.quad(f, 1e-9, 2000.0, points=[e[k], e[k + 1]], limit=500)[0])
    expect = np.array(expect)
    R = np.hypot(sample["x"], sample["y"])
    K = sample["vz"] ** 2 / N
    sd = np.array([math.sqrt(np.sum(K[(R >= e[k]) & (R < e[k + 1])] ** 2)) for k in range(8)])
    assert np.all(np.abs(y - expect) < 5 * sd), (y, expect, sd)


def test_virial_sum_vz2(oracle, sample):
    N = sample["x"].size
    lay = make_layout(1, 1e-9, 1e9, 1, 1e-9, 1e9, "v2")
    y = oracle.deposit(sample, np.ones(N), lay)
    assert y[0] == pytest.approx(1.0, abs=1e-10)       # every particle is inside
    sd = math.sqrt(np.sum((sample["vz"] ** 2 / N) ** 2))
    assert abs(y[1] - 1.0 / 18.0) < 5 * sd


def test_brute_force_rebinning_tiny_n(oracle):
    g = np.random.default_rng(5)
    n = 64
    lay = make_layout(6, 0.1, 10.0, 5, 0.2, 8.0, "losvd", n_v=8, v_min=-2.0, v_max=2.0)
    re, Re = _edges(0.1, 10.0, 6), _edges(0.2, 8.0, 5)
    ve = np.array([-2.0 + 4.0 * k / 8 if 0 < k < 8 else (-2.0 if k == 0 else 2.0) for k in range(9)])
    r = g.uniform(0.05, 12.0, n)
    r[:7] = re                                # exactly on every radial edge
    ct = g.uniform(-1, 1, n)
    ph = g.uniform(0, 2 * np.pi, n)
    st = np.sqrt(1 - ct * ct)
    parts = dict(x=r * st * np.cos(ph), y=r * st * np.sin(ph), z=r * ct,
                 vx=g.normal(size=n), vy=g.normal(size=n), vz=g.uniform(-2.5, 2.5, n))
    parts["vz"][10:19] = ve                   # exactly on every velocity edge
    u = g.integers(1, 2048, n) / 1024.0
    y = oracle.deposit(parts, u, lay, mass=float(n))
    expect = np.zeros(6 + 5 * 8)
    rr = np.sqrt(parts["x"] ** 2 + parts["y"] ** 2 + parts["z"] ** 2)
    RR = np.sqrt(parts["x"] ** 2 + parts["y"] ** 2)
    for i in range(n):
        for k in range(6):
            if re[k] <= rr[i] < re[k + 1]:
                expect[k] += u[i]
        for p in range(5):
            if Re[p] <= RR[i] < Re[p + 1]:
                for b in range(8):
                    if ve[b] <= parts["vz"][i] < ve[b + 1]:
                        expect[6 + p * 8 + b] += u[i]
    np.testing.assert_array_equal(y, expect)
    # threads only regroup the sum
    np.testing.assert_allclose(oracle.deposit(parts, u, lay, mass=float(n), nthreads=4), expect,
                               rtol=1e-15, atol=0)


def test_weight_sum_conservation_exact(oracle):
    g = np.random.default_rng(9)
    n = 500
    parts = {k: g.normal(size=n) for k in ("x", "y", "z", "vx", "vy", "vz")}
    u = g.integers(1, 4096, n) / 512.0
    lay = make_layout(17, 1e-9, 1e9)
    y = oracle.deposit(parts, u, lay, mass=float(n))
    assert y.sum() == u.sum()                 # dyadic weights: exact in FP64


def test_hermite_polynomials_match_numpy(oracle):
    for n in range(9):
        c = np.zeros(n + 1)
        c[n] = 1
        for x in (-3.1, -0.7, 0.0, 0.4, 1.3, 2.9):
            assert oracle.hermite(n, x) == pytest.approx(npherm.hermval(x, c), rel=1e-12, abs=1e-12)


def test_gauss_hermite_functions_orthonormal(oracle):
    for n in range(5):
        for m in range(5):
            v = integrate.quad(lambda t: oracle.gh_u(n, t) * oracle.gh_u(m, t), -np.inf, np.inf,
                               epsabs=1e-13)[0]
            assert 2 * math.sqrt(math.pi) * v == pytest.approx(1.0 if n == m else 0.0, abs=1e-10)


def _gh_moment(oracle, lay, n, V, S, mean, sd):
    """b_n / l of a Gaussian LOSVD N(mean, sd^2) with GH centre (V, S),
    integrating the oracle's own kernel of one point in annulus 0."""
    def k_of(v):
        ks = oracle.kernels(lay, 0.5, 0.0, 0.0, v, V_p=[V], sigma_p=[S])
        return ks.get(lay["n_r"] + n - 1, 0.0)
    pdf = lambda v: math.exp(-0.5 * ((v - mean) / sd) ** 2) / (math.sqrt(2 * math.pi) * sd)
    return integrate.quad(lambda v: k_of(v) * pdf(v), mean - 12 * sd, mean + 12 * sd,
                          epsabs=1e-13, epsrel=1e-11, limit=400)[0]


def test_matched_gaussian_has_zero_gh_moments(oracle):
    lay = make_layout(1, 10.0, 20.0, 1, 0.1, 1.0, "gh", gh_nmax=4)
    for n in (1, 2, 3, 4):
        assert abs(_gh_moment(oracle, lay, n, 0.3, 0.7, 0.3, 0.7)) < 1e-10


def test_gh_first_order_relations_h1h2(oracle):
    """Eq. h1h2: moving the GH centre by dV changes h_1 by -dV / (sqrt2 sigma);
    scaling its width by d sigma changes h_2 by -d sigma / (sqrt2 sigma)."""
    lay = make_layout(1, 10.0, 20.0, 1, 0.1, 1.0, "gh", gh_nmax=4)
    S, d = 0.7, 1e-4
    h1 = _gh_moment(oracle, lay, 1, 0.3 + d, S, 0.3, S)
    assert h1 == pytest.approx(-d / (math.sqrt(2) * S), rel=1e-3)
    h2 = _gh_moment(oracle, lay, 2, 0.3, S + d, 0.3, S)
    assert h2 == pytest.approx(-d / (math.sqrt(2) * S), rel=1e-3)


def test_ambiguity_covers_both_sides_of_an_edge(oracle):
    """A point just outside the outer edge has no kernel, but it is within the
    band of that edge: its weight counts as ambiguous for the last bin. A point
    on an inner edge is ambiguous for the bins on both sides."""
    lay = make_layout(4, 1.0, 16.0)          # edges 1, 2, 4, 8, 16
    for r, inside in ((16.0 * (1 + 1e-9), False), (16.0 * (1 - 1e-9), True), (8.0, True)):
        p = dict(x=np.array([r]), y=np.zeros(1), z=np.zeros(1), vx=np.zeros(1), vy=np.zeros(1),
                 vz=np.zeros(1))
        y, ya, yb = oracle.deposit(p, np.ones(1), lay, band=1e-7, with_abs=True)
        assert y[3] == (1.0 if inside else 0.0)
        assert yb[3] == 1.0
        assert yb[2] == (1.0 if r == 8.0 else 0.0)
        assert yb[0] == yb[1] == 0.0
