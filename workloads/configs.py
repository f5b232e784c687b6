"""The benchmark workloads: sizes, layouts, parameters and seeded draws.

Every workload is a plain description (dicts of numbers and strings). The
oracle binding and the HIP binding each translate it into their own argument
structures; the string codes ``"mpr"/"gwr"`` (entropy) and
``"none"/"v2"/"gh"/"losvd"`` (kinematic observable kind) are the only
vocabulary shared with them.

Workloads (G = M = a = 1 units; the paper sets the physical scale in Sec. 3.1):

1. ``hernquist_v2_n20k``: N = 2e4 isotropic Hernquist particles in the
   Hernquist potential, 200 steps, 30 log radial mass bins on [0.05, 20] plus
   v_z^2 moments in 20 log annuli on [0.05, 20]; targets from an OM r_a = 1
   Hernquist realization, 2 % noise; 20 x 10 (E, L/Lc) prior grid every 25
   steps. FP64 particle state.
2. ``hernquist_gh_n1m``: N = 1e6, 1000 steps, 40 radial bins plus
   Gauss-Hermite b_1..b_4 in 30 annuli; OM r_a = 1 targets, 2 % noise; 50 x 20
   grid. FP32 particle state.
3. ``nfw_losvd_n8m``: N = 8e6 Plummer-like (b = 1) particles in a Hernquist
   (1, 1) + NFW (M200 = 10, c = 8, r200 = 100) potential, 2000 steps, 50
   radial bins plus 64-bin LOS velocity histograms on [-4, 4) in 40 annuli;
   OM r_a = 2 Hernquist-tracer targets, 5 % noise; 64 x 32 grid.
4. ``batch64_gh``: 64 fits, N_f = round(2^(16 + 5U)), each in its own
   Hernquist(upsilon_f) + NFW(10, c_f) potential, the layout of workload 2.
5. ``serve_losvd``: a Poisson request trace (20 fits/s), N log-uniform in
   [1e5, 4e6], 500-2000 steps, the layout of workload 3, noise in
   {1, 2, 5} %.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .targets import density_length
from .dynamics import (
    EddingtonDF,
    HernquistTracer,
    Potential,
    hernquist_isotropic_df,
    sample_om_model,
    sample_plummer_jeans,
)


def rng(seed: int) -> np.random.Generator:
    """Philox counter-based generator keyed by ``seed``."""
    return np.random.Generator(np.random.Philox(key=int(seed)))


def make_potential(upsilon=1.0, M200=0.0, c=0.0, r200=100.0, G=1.0, M_star=1.0, a=1.0):
    r_s = r200 / c if M200 > 0 else 0.0
    return Potential(G=G, M_star=M_star, a=a, upsilon=upsilon, M200=M200,
                     c=c if M200 > 0 else 0.0, r_s=r_s)


def make_layout(n_r, r_min, r_max, n_R=0, R_min=0.05, R_max=20.0, kin="none",
                gh_nmax=0, n_v=0, v_min=0.0, v_max=0.0, dens="bins", l_max=0):
    """Observable layout. dens = "bins": n_r radial mass bins on [r_min, r_max);
    dens = "alm": spherical-harmonic coefficients a_lm,k, l <= l_max, on n_r
    log-spaced mesh radii from r_min to r_max (cloud-in-cell weights)."""
    return dict(n_r=int(n_r), r_min=float(r_min), r_max=float(r_max), n_R=int(n_R),
                R_min=float(R_min), R_max=float(R_max), kin=kin, gh_nmax=int(gh_nmax),
                n_v=int(n_v), v_min=float(v_min), v_max=float(v_max), dens=dens,
                l_max=int(l_max))


def J_of(layout: dict) -> int:
    per = {"none": 0, "v2": 1, "gh": layout["gh_nmax"], "losvd": layout["n_v"]}[layout["kin"]]
    return density_length(layout) + layout["n_R"] * per


def with_alm(wl: "Workload", n_mesh: int = 60, l_max: int = 4) -> "Workload":
    """The workload with its radial mass bins replaced by the spherical-harmonic
    density coefficients a_lm,k (Sec. 3.3, eq. alm) on an n_mesh-point
    log-spaced mesh over the same radial range (the paper uses 60 points)."""
    lay = dict(wl.layout, n_r=int(n_mesh), dens="alm", l_max=int(l_max))
    return wl.with_(name=f"{wl.name}_alm{l_max}", layout=lay)


def with_scf(wl: "Workload", l_max: int = 4, n_nodes: int = 32, r_min: float = 0.02,
             r_max: float = 100.0, every: int = 10) -> "Workload":
    """The workload with its stellar potential computed from the particles (a
    multipole expansion to degree l_max with n_nodes log-spaced nodes over
    [r_min, r_max], rebuilt every `every` steps; Sec. 2.1, Sec. 5) instead of
    the analytic Hernquist part."""
    par = dict(wl.params, scf_lmax=int(l_max), scf_nr=int(n_nodes), scf_rmin=float(r_min),
               scf_rmax=float(r_max), scf_every=int(every))
    return wl.with_(name=f"{wl.name}_scf{l_max}", params=par)


def make_params(pot: Potential, dt=0.01, eps=0.1, mu=1e-2, alpha=2.1, mass=1.0,
                entropy="mpr", n_E=20, n_x=10, prior_every=25, smooth=0):
    """Step parameters. alpha is the smoothing rate per unit time (the
    workloads' "alpha = 2.1 dt" is read as alpha dt = 0.021 at dt = 0.01).
    The (E, x) grid spans E in [Phi(0), 0). smooth = 1 smooths the prior grid
    (thin-plate spline, lambda by GCV) at every refresh."""
    return dict(dt=float(dt), eps=float(eps), mu=float(mu), alpha=float(alpha),
                mass=float(mass), entropy=entropy, n_E=int(n_E), n_x=int(n_x),
                prior_every=int(prior_every), E_lo=-pot.psi0(), E_hi=0.0, smooth=int(smooth))


@dataclass
class Workload:
    name: str
    N: int
    state: str                      # "f64" or "f32" particle state
    potential: Potential
    layout: dict
    params: dict
    steps: int
    ic: str                         # "hernquist_iso" | "iso_in_pot" | "plummer_jeans"
    target_ra: float
    noise: float
    n_target: int
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def J(self) -> int:
        return J_of(self.layout)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    # ---------------------------------------------------------------- draws
    def initial_particles(self, n=None, seed=None) -> dict:
        """Initial particle model (float64 SoA dict x, y, z, vx, vy, vz)."""
        n = self.N if n is None else int(n)
        g = rng(self.seed * 1000 + 1 if seed is None else seed)
        if self.ic == "hernquist_iso":
            pot = self.potential
            df = hernquist_isotropic_df(pot.G, pot.M_star * pot.upsilon, pot.a)
            return sample_om_model(g, n, pot, HernquistTracer(1.0, pot.a), np.inf, df)
        if self.ic == "iso_in_pot":
            return sample_om_model(g, n, self.potential, HernquistTracer(1.0, 1.0), np.inf)
        if self.ic == "plummer_jeans":
            return sample_plummer_jeans(g, n, self.potential, b=1.0)
        raise ValueError(self.ic)

    def target_particles(self, n=None, seed=None) -> dict:
        """Realization of the target DF: Hernquist tracer with OM anisotropy
        radius ``target_ra`` in the workload's potential."""
        n = self.n_target if n is None else int(n)
        g = rng(self.seed * 1000 + 2 if seed is None else seed)
        df = EddingtonDF(self.potential, HernquistTracer(1.0, 1.0), self.target_ra)
        return sample_om_model(g, n, self.potential, HernquistTracer(1.0, 1.0),
                               self.target_ra, df)

    def noise_rng(self) -> np.random.Generator:
        return rng(self.seed * 1000 + 3)


def _wl1() -> Workload:
    pot = make_potential()
    lay = make_layout(30, 0.05, 20.0, 20, 0.05, 20.0, "v2")
    par = make_params(pot, n_E=20, n_x=10)
    return Workload("hernquist_v2_n20k", 20_000, "f64", pot, lay, par, 200,
                    "hernquist_iso", 1.0, 0.02, 1 << 20, seed=1)


def _wl2() -> Workload:
    pot = make_potential()
    lay = make_layout(40, 0.05, 20.0, 30, 0.05, 20.0, "gh", gh_nmax=4)
    par = make_params(pot, n_E=50, n_x=20)
    return Workload("hernquist_gh_n1m", 1_000_000, "f32", pot, lay, par, 1000,
                    "hernquist_iso", 1.0, 0.02, 1 << 22, seed=2)


def _wl3() -> Workload:
    pot = make_potential(upsilon=1.0, M200=10.0, c=8.0, r200=100.0)
    lay = make_layout(50, 0.05, 20.0, 40, 0.05, 20.0, "losvd", n_v=64, v_min=-4.0, v_max=4.0)
    par = make_params(pot, n_E=64, n_x=32)
    return Workload("nfw_losvd_n8m", 8_000_000, "f32", pot, lay, par, 2000,
                    "plummer_jeans", 2.0, 0.05, 1 << 22, seed=3)


WORKLOADS = {
    1: _wl1,
    2: _wl2,
    3: _wl3,
}


def workload(k: int) -> Workload:
    return WORKLOADS[k]()


UPSILONS = np.round(np.arange(0.5, 2.0 + 1e-9, 0.025), 3)


def batch_fits(n_fits=64, seed=4, base=None):
    """Workload 4: per-fit sizes N_f = round(2^(16 + 5U)) and potentials
    Hernquist(upsilon_f) + NFW(M200 = 10, c_f, r200 = 100), upsilon_f from
    {0.5, 0.525, ..., 2.0}, c_f ~ U[5, 15]; layout and steps of workload 2."""
    base = _wl2() if base is None else base
    g = rng(seed)
    Ns = np.rint(2.0 ** (16.0 + 5.0 * g.random(n_fits))).astype(np.int64)
    ups = g.choice(UPSILONS, n_fits)
    cs = g.uniform(5.0, 15.0, n_fits)
    fits = []
    for f in range(n_fits):
        pot = make_potential(upsilon=float(ups[f]), M200=10.0, c=float(cs[f]))
        par = make_params(pot, n_E=base.params["n_E"], n_x=base.params["n_x"])
        fits.append(Workload(f"batch{f}", int(Ns[f]), "f32", pot, dict(base.layout), par,
                             base.steps, "iso_in_pot", 1.0, 0.02, 1 << 18,
                             seed=seed * 100000 + f))
    return fits


def serve_trace(n_requests=500, rate=20.0, seed=5, state="f32"):
    """Workload 5: Poisson arrivals (rate per second), N log-uniform in
    [1e5, 4e6], 500-2000 steps, noise in {1, 2, 5} %, potentials as in the
    batched workload, the layout of workload 3. Returns (arrival_s, fits)."""
    base = _wl3()
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    Ns = np.rint(np.exp(g.uniform(np.log(1e5), np.log(4e6), n_requests))).astype(np.int64)
    steps = g.integers(500, 2001, n_requests)
    noise = g.choice(np.array([0.01, 0.02, 0.05]), n_requests)
    ups = g.choice(UPSILONS, n_requests)
    cs = g.uniform(5.0, 15.0, n_requests)
    fits = []
    for k in range(n_requests):
        pot = make_potential(upsilon=float(ups[k]), M200=10.0, c=float(cs[k]))
        par = make_params(pot, n_E=base.params["n_E"], n_x=base.params["n_x"])
        fits.append(Workload(f"req{k}", int(Ns[k]), state, pot, dict(base.layout), par,
                             int(steps[k]), "plummer_jeans", 2.0, float(noise[k]), 1 << 18,
                             seed=seed * 100000 + k))
    return t, fits
