"""Spherical equilibrium models used to draw initial conditions and targets.

Units: G, masses and lengths are explicit parameters (the workloads use
G = M = a = 1). Everything here is float64 numpy and seeded by the caller's
``numpy.random.Generator``.

What is drawn
-------------
* Potentials: Hernquist sphere (paper Sec. 3.1, eq. her) of mass
  ``M_star * upsilon`` and scale ``a``, optionally plus an NFW halo of virial
  mass ``M200``, concentration ``c`` and scale radius ``r_s``.
* Tracers: Hernquist (the paper's targets and initial models, Sec. 3.1 and
  Sec. 4.1) and Plummer (a "Plummer-like" initial model).
* Distribution functions: the isotropic Hernquist DF in closed form
  (Hernquist 1990) and Osipkov-Merritt DFs f(Q), Q = E_rel - L^2/(2 r_a^2),
  of any tracer in any of the potentials above by Eddington inversion of
  rho_Q = (1 + r^2/r_a^2) rho (Sec. 3.1 uses OM anisotropy with r_a = 2a).
* Gaussian velocities from the isotropic Jeans dispersion of a tracer in a
  potential (for the Plummer-like initial model).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


# --------------------------------------------------------------------------
# Potentials
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Potential:
    """Hernquist(G*M_star*upsilon, a) [+ NFW(G*M200, c, r_s)] potential, and
    optionally the logarithmic halo v0^2/2 ln(r0^2 + R^2 + z^2/q^2) (v0 > 0).
    The samplers here use the spherical parts only; the halo is carried for
    the fits (it makes every orbit bound, so psi/psi0 ignore it)."""

    G: float = 1.0
    M_star: float = 1.0
    a: float = 1.0
    upsilon: float = 1.0
    M200: float = 0.0
    c: float = 0.0
    r_s: float = 0.0
    v0: float = 0.0
    r0: float = 1.0
    q: float = 1.0

    @property
    def has_nfw(self) -> bool:
        return self.M200 > 0.0

    def _fc(self) -> float:
        return float(np.log1p(self.c) - self.c / (1.0 + self.c))

    def psi(self, r):
        """Relative potential -Phi(r) > 0 (Phi -> 0 at infinity)."""
        r = np.asarray(r, dtype=np.float64)
        out = self.G * self.M_star * self.upsilon / (r + self.a)
        if self.has_nfw:
            x = r / self.r_s
            small = x < 1e-6
            xs = np.where(small, 1.0, x)
            t = np.where(small, (1.0 - 0.5 * x + x * x / 3.0) / self.r_s,
                         np.log1p(xs) / np.where(small, 1.0, r))
            out = out + self.G * self.M200 / self._fc() * t
        return out

    def psi0(self) -> float:
        """Central relative potential -Phi(0)."""
        out = self.G * self.M_star * self.upsilon / self.a
        if self.has_nfw:
            out += self.G * self.M200 / (self._fc() * self.r_s)
        return float(out)

    def mass(self, r):
        """Total enclosed mass M(<r)."""
        r = np.asarray(r, dtype=np.float64)
        m = self.M_star * self.upsilon * r * r / (r + self.a) ** 2
        if self.has_nfw:
            x = r / self.r_s
            small = x < 1e-4
            series = x * x * (0.5 - 2.0 * x / 3.0 + 0.75 * x * x)
            m = m + self.M200 / self._fc() * np.where(
                small, series, np.log1p(x) - x / (1.0 + x))
        return m

    def as_dict(self) -> dict:
        return dict(G=self.G, M_star=self.M_star, a=self.a, upsilon=self.upsilon,
                    M200=self.M200, c=self.c, r_s=self.r_s, v0=self.v0, r0=self.r0, q=self.q)


# --------------------------------------------------------------------------
# Tracers
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class HernquistTracer:
    M: float = 1.0
    a: float = 1.0

    def rho(self, r):
        r = np.asarray(r, dtype=np.float64)
        return self.M * self.a / (2.0 * np.pi * r * (r + self.a) ** 3)

    def drho_dr(self, r):
        r = np.asarray(r, dtype=np.float64)
        a = self.a
        return -self.M * a / (2.0 * np.pi) * (4.0 * r + a) / (r * r * (r + a) ** 4)

    def mass(self, r):
        r = np.asarray(r, dtype=np.float64)
        return self.M * r * r / (r + self.a) ** 2

    def sample_radius(self, u):
        q = np.sqrt(u)
        return self.a * q / (1.0 - q)


@dataclass(frozen=True)
class PlummerTracer:
    M: float = 1.0
    b: float = 1.0

    def rho(self, r):
        r = np.asarray(r, dtype=np.float64)
        return 3.0 * self.M / (4.0 * np.pi * self.b ** 3) * (1.0 + (r / self.b) ** 2) ** -2.5

    def drho_dr(self, r):
        r = np.asarray(r, dtype=np.float64)
        b = self.b
        return (3.0 * self.M / (4.0 * np.pi * b ** 3) * -5.0 * r / b ** 2
                * (1.0 + (r / b) ** 2) ** -3.5)

    def mass(self, r):
        r = np.asarray(r, dtype=np.float64)
        return self.M * r ** 3 / (r * r + self.b ** 2) ** 1.5

    def sample_radius(self, u):
        return self.b / np.sqrt(u ** (-2.0 / 3.0) - 1.0)


def hernquist_projected_mass(R, M=1.0, a=1.0):
    """Mass of a Hernquist sphere inside projected radius R (Hernquist 1990)."""
    s = np.atleast_1d(np.asarray(R, dtype=np.float64)) / a
    out = np.empty_like(s)
    lo = s < 1.0 - 1e-6
    hi = s > 1.0 + 1e-6
    mid = ~(lo | hi)
    sl = s[lo]
    X = np.log((1.0 + np.sqrt(1.0 - sl * sl)) / sl) / np.sqrt(1.0 - sl * sl)
    out[lo] = M * sl * sl * (X - 1.0) / (1.0 - sl * sl)
    sh = s[hi]
    X = np.arccos(1.0 / sh) / np.sqrt(sh * sh - 1.0)
    out[hi] = M * sh * sh * (X - 1.0) / (1.0 - sh * sh)
    out[mid] = M / 3.0 * (1.0 + 0.0 * s[mid])  # limit at s = 1 (slope is smooth)
    out[s == 0.0] = 0.0
    return out if np.ndim(R) else float(out[0])


# --------------------------------------------------------------------------
# Distribution functions
# --------------------------------------------------------------------------
class hernquist_isotropic_df:
    """Closed-form isotropic DF of a self-consistent Hernquist sphere.

    f(E) = M / (8 sqrt2 pi^3 a^3 vg^3) (1-q^2)^(-5/2)
           [3 asin q + q sqrt(1-q^2) (1-2q^2)(8q^4-8q^2-3)],
    q = sqrt(a E / (G M)), vg = sqrt(G M / a)   (Hernquist 1990, eq. 17).
    """

    def __init__(self, G=1.0, M=1.0, a=1.0):
        self.G, self.M, self.a = G, M, a
        self.psi0 = G * M / a

    def f(self, Q):
        Q = np.asarray(Q, dtype=np.float64)
        q2 = np.clip(Q / self.psi0, 0.0, 1.0 - 1e-15)
        q = np.sqrt(q2)
        vg = np.sqrt(self.G * self.M / self.a)
        pre = self.M / (8.0 * np.sqrt(2.0) * np.pi ** 3 * self.a ** 3 * vg ** 3)
        br = (3.0 * np.arcsin(q)
              + q * np.sqrt(1.0 - q2) * (1.0 - 2.0 * q2) * (8.0 * q2 * q2 - 8.0 * q2 - 3.0))
        out = pre * br / (1.0 - q2) ** 2.5
        return np.where(Q > 0.0, np.maximum(out, 0.0), 0.0)


class EddingtonDF:
    """Osipkov-Merritt DF f(Q) of ``tracer`` in ``pot`` by Eddington inversion.

    rho_Q(r) = (1 + r^2/r_a^2) rho(r) (r_a = inf: isotropic) and
    f(Q) = 1/(sqrt8 pi^2) d/dQ int_0^Q (d rho_Q / d psi) d psi / sqrt(Q - psi).
    The inner integral is evaluated along r with r = r_k exp(s^2), which
    removes the inverse-square-root endpoint singularity, by panelled
    Gauss-Legendre quadrature; the outer derivative by finite differences on
    the log-spaced radius grid.
    """

    def __init__(self, pot: Potential, tracer, r_a=np.inf, n=1400,
                 r_lo=1e-6, r_hi=1e8, panels=12, nodes=48):
        self.pot, self.tracer, self.r_a = pot, tracer, float(r_a)
        rk = np.logspace(np.log10(r_lo), np.log10(r_hi), n)
        Qk = pot.psi(rk)
        x, w = np.polynomial.legendre.leggauss(nodes)
        R_int = 1e18
        S = np.sqrt(np.log(R_int / rk))
        G = np.zeros(n)
        edges = np.linspace(0.0, 1.0, panels + 1)
        for p in range(panels):
            lo, hi = edges[p], edges[p + 1]
            t = lo + (hi - lo) * 0.5 * (x + 1.0)
            wt = (hi - lo) * 0.5 * w
            s = t[None, :] * S[:, None]
            r = rk[:, None] * np.exp(s * s)
            dQ = Qk[:, None] - pot.psi(r)
            dQ = np.maximum(dQ, 1e-300)
            integ = -self._drhoQ_dr(r) * 2.0 * s * r / np.sqrt(dQ)
            G += (integ * (wt[None, :] * S[:, None])).sum(axis=1)
        dG = np.gradient(G, Qk)
        f = dG / (np.sqrt(8.0) * np.pi ** 2)
        order = np.argsort(Qk)
        self.Q = Qk[order]
        self.fk = np.maximum(f[order], 0.0)
        with np.errstate(divide="ignore"):
            self.lnf = np.log(np.maximum(self.fk, 1e-300))
        self.Qmin, self.Qmax = self.Q[0], self.Q[-1]

    def _drhoQ_dr(self, r):
        rho = self.tracer.rho(r)
        drho = self.tracer.drho_dr(r)
        if np.isinf(self.r_a):
            return drho
        ra2 = self.r_a ** 2
        return (1.0 + r * r / ra2) * drho + 2.0 * r / ra2 * rho

    def f(self, Q):
        Q = np.asarray(Q, dtype=np.float64)
        val = np.exp(np.interp(Q, self.Q, self.lnf))
        return np.where(Q > self.Qmin, val, 0.0)


# --------------------------------------------------------------------------
# Sampling
# --------------------------------------------------------------------------
R_CLIP = 1e7

def _unit_vectors(rng, n):
    ct = rng.uniform(-1.0, 1.0, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    return ct, st, ph


def sample_positions(rng, tracer, n):
    """Radii from the tracer's cumulative mass, isotropic directions."""
    u = rng.random(n)
    u = np.clip(u, 1e-300, 1.0 - 1e-16)
    # radii beyond 1e7 scale lengths (probability ~2e-7 for a Hernquist
    # tracer) are placed at 1e7, where the tabulated DFs are still resolved
    r = np.minimum(tracer.sample_radius(u), R_CLIP)
    ct, st, ph = _unit_vectors(rng, n)
    x = r * st * np.cos(ph)
    y = r * st * np.sin(ph)
    z = r * ct
    return r, ct, st, ph, x, y, z


def _envelope(pot, df, r_grid):
    s = np.concatenate([np.geomspace(1e-6, 0.05, 400), np.linspace(0.05, 1.0, 600)[1:]])
    env = np.empty(r_grid.size)
    for k0 in range(0, r_grid.size, 64):
        rr = r_grid[k0:k0 + 64]
        psi = pot.psi(rr)
        p = s[None, :] ** 2 * df.f(psi[:, None] * (1.0 - s[None, :] ** 2))
        env[k0:k0 + 64] = p.max(axis=1)
    return env


def sample_om_velocities(rng, pot, df, r, ct, st, ph, r_a=np.inf):
    """Velocities of an OM (or isotropic, r_a = inf) model at given positions.

    In OM models f depends on Q = psi - (v_r^2 + (1 + r^2/r_a^2) v_t^2)/2, so
    the pseudo-velocity (v_r, v_t sqrt(1 + r^2/r_a^2)) is isotropic with speed
    density ~ s^2 f(psi (1 - s^2)), s = |v'| / sqrt(2 psi), sampled here by
    rejection under a tabulated envelope.
    """
    n = r.size
    psi = pot.psi(r)
    r_grid = np.logspace(-7, 9, 400)
    env_g = _envelope(pot, df, r_grid) * 1.6
    lr = np.clip(np.log10(r), -7.0, 9.0)
    pos = (lr + 7.0) / 16.0 * (r_grid.size - 1)
    i0 = np.clip(np.floor(pos).astype(np.int64), 0, r_grid.size - 2)
    env = np.maximum(env_g[i0], env_g[i0 + 1]) * 1.25
    s_out = np.empty(n)
    todo = np.arange(n)
    violations = 0
    while todo.size:
        s = rng.random(todo.size)
        u = rng.random(todo.size)
        p = s * s * df.f(psi[todo] * (1.0 - s * s))
        violations += int(np.count_nonzero(p > env[todo]))
        acc = u * env[todo] < p
        s_out[todo[acc]] = s[acc]
        todo = todo[~acc]
    if violations:
        raise RuntimeError(f"rejection envelope violated {violations} times")
    vp = s_out * np.sqrt(2.0 * psi)
    cv, sv, pv = _unit_vectors(rng, n)
    vr = vp * cv
    scale = 1.0 if np.isinf(r_a) else 1.0 / np.sqrt(1.0 + (r / r_a) ** 2)
    vth = vp * sv * np.cos(pv) * scale
    vph = vp * sv * np.sin(pv) * scale
    cp, sp = np.cos(ph), np.sin(ph)
    vx = vr * st * cp + vth * ct * cp - vph * sp
    vy = vr * st * sp + vth * ct * sp + vph * cp
    vz = vr * ct - vth * st
    return vx, vy, vz


def _jeans_sigma2_table(pot, tracer, n=6000, r_lo=1e-7, r_hi=1e9):
    r = np.logspace(np.log10(r_lo), np.log10(r_hi), n)
    integ = tracer.rho(r) * pot.G * pot.mass(r) / r  # d/dlnr form: rho G M / r^2 * r
    lnr = np.log(r)
    # cumulative integral from r to r_hi (trapezoid in ln r)
    seg = 0.5 * (integ[1:] + integ[:-1]) * np.diff(lnr)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    sig2 = tail / tracer.rho(r)
    return r, sig2


def sample_gaussian_jeans_velocities(rng, pot, tracer, r):
    """Isotropic Gaussian velocities with the Jeans dispersion of ``tracer``
    in ``pot``; draws with E >= 0 are redrawn (bound particles only)."""
    rt, s2 = _jeans_sigma2_table(pot, tracer)
    sig = np.sqrt(np.interp(np.log(r), np.log(rt), s2))
    psi = pot.psi(r)
    n = r.size
    v = np.empty((3, n))
    todo = np.arange(n)
    while todo.size:
        g = rng.standard_normal((3, todo.size)) * sig[todo]
        ok = 0.5 * (g * g).sum(axis=0) < psi[todo]
        v[:, todo[ok]] = g[:, ok]
        todo = todo[~ok]
    return v[0], v[1], v[2]


def _pack(x, y, z, vx, vy, vz):
    return dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz)


def sample_om_model(rng, n, pot: Potential, tracer, r_a=np.inf, df=None):
    """n particles of an OM (isotropic if r_a = inf) model of ``tracer``."""
    if df is None:
        df = EddingtonDF(pot, tracer, r_a)
    r, ct, st, ph, x, y, z = sample_positions(rng, tracer, n)
    vx, vy, vz = sample_om_velocities(rng, pot, df, r, ct, st, ph, r_a)
    return _pack(x, y, z, vx, vy, vz)


def sample_hernquist_isotropic(rng, n, G=1.0, M=1.0, a=1.0):
    """Equal-mass isotropic self-consistent Hernquist sphere (closed-form DF)."""
    pot = Potential(G=G, M_star=M, a=a)
    df = hernquist_isotropic_df(G, M, a)
    return sample_om_model(rng, n, pot, HernquistTracer(M, a), np.inf, df)


def sample_plummer_jeans(rng, n, pot: Potential, b=1.0):
    """Plummer-like initial model: Plummer radii, Gaussian Jeans velocities."""
    tr = PlummerTracer(1.0, b)
    r, ct, st, ph, x, y, z = sample_positions(rng, tr, n)
    vx, vy, vz = sample_gaussian_jeans_velocities(rng, pot, tr, r)
    return _pack(x, y, z, vx, vy, vz)
