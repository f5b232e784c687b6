"""Target data sets built from a realization of the target DF.

As in the paper (Sec. 3.1), target observables are the model observables of a
particle realization of the target, measured "in the exact same way" as the
model's own (Sec. 3.2). This module therefore takes the measurement as a
callable ``observe(V_p, sigma_p) -> y`` supplied by whichever engine is in
use (the oracle in tests, the library in the benchmark) and adds only:

* the Gauss-Hermite centres (V_p, sigma_p) per annulus, found by the
  first-order relations of Sec. 3.3 (eq. h1h2) until h_1 = h_2 = 0;
* seeded Gaussian observation errors with a stated error model.
"""

from __future__ import annotations

import numpy as np

from .dynamics import hernquist_projected_mass

SQRT2 = float(np.sqrt(2.0))


def density_length(layout: dict) -> int:
    """Observables of the density part: n_r radial bins, or (l_max + 1)^2
    spherical-harmonic coefficients at each of the n_r mesh radii."""
    if layout.get("dens", "bins") == "alm":
        return layout["n_r"] * (layout.get("l_max", 0) + 1) ** 2
    return layout["n_r"]


def annulus_luminosity(layout: dict, M=1.0, a=1.0) -> np.ndarray:
    """l_p of a Hernquist(M, a) tracer in the layout's log annuli (closed form)."""
    n = layout["n_R"]
    k = np.arange(n + 1)
    edges = layout["R_min"] * (layout["R_max"] / layout["R_min"]) ** (k / n)
    mp = hernquist_projected_mass(edges, M, a)
    return np.diff(mp)


def fit_gauss_hermite_centres(observe, layout: dict, lum: np.ndarray,
                              iters: int = 60, tol: float = 1e-9):
    """(V_p, sigma_p) per annulus such that h_1 = h_2 = 0.

    h_n = b_n / l_p. Eq. h1h2 gives dh_1 = -dV/(sqrt2 sigma) and
    dh_2 = -d sigma/(sqrt2 sigma), so V += sqrt2 sigma h_1 and
    sigma *= 1 + sqrt2 h_2 cancel the current h_1, h_2 to first order.
    """
    n_r, n_R, nmax = density_length(layout), layout["n_R"], layout["gh_nmax"]
    if nmax < 2:
        raise ValueError("Gauss-Hermite centres need b_1 and b_2")
    V = np.zeros(n_R)
    s = np.full(n_R, 0.3)
    safe = np.where(lum > 0, lum, 1.0)
    for _ in range(iters):
        y = np.asarray(observe(V, s), dtype=np.float64)
        b = y[n_r:n_r + n_R * nmax].reshape(n_R, nmax)
        h1 = np.where(lum > 0, b[:, 0] / safe, 0.0)
        h2 = np.where(lum > 0, b[:, 1] / safe, 0.0)
        V = V + SQRT2 * s * h1
        s = s * np.clip(1.0 + SQRT2 * h2, 0.5, 2.0)
        if max(np.abs(h1).max(), np.abs(h2).max()) < tol:
            break
    return V, s


def add_noise(Y_true: np.ndarray, layout: dict, s: float, g: np.random.Generator,
              lum: np.ndarray | None = None):
    """Noisy targets Y = Y_true + sigma * N(0, 1) with errors sigma:

    * radial mass and v^2 moments: sigma = s |Y_true| (floored at 1e-3 of the
      group's largest value, so empty bins still carry a finite error);
    * spherical-harmonic coefficients a_lm,k: sigma = s |a_00,k| for every
      (l, m) at mesh radius k, with the same floor (the errors of the
      higher moments scale with the density there; the values of l > 0
      are about zero for a spherical target);
    * Gauss-Hermite b_n: sigma = s l_p (b_n can vanish, l_p cannot);
    * LOSVD bins: sigma = s max(Y, 0.01 max_k Y_{p,k}) per annulus.
    """
    Y_true = np.asarray(Y_true, dtype=np.float64)
    n_r, n_R, kin = density_length(layout), layout["n_R"], layout["kin"]
    sig = np.empty_like(Y_true)
    if layout.get("dens", "bins") == "alm":
        nlm = (layout.get("l_max", 0) + 1) ** 2
        a00 = np.abs(Y_true[:n_r].reshape(-1, nlm)[:, 0])
        sig[:n_r] = np.repeat(s * np.maximum(a00, 1e-3 * a00.max()), nlm)
    else:
        rad = np.abs(Y_true[:n_r])
        sig[:n_r] = s * np.maximum(rad, 1e-3 * rad.max())
    rest = Y_true[n_r:]
    if kin == "v2":
        a = np.abs(rest)
        sig[n_r:] = s * np.maximum(a, 1e-3 * a.max())
    elif kin == "gh":
        nmax = layout["gh_nmax"]
        if lum is None:
            raise ValueError("Gauss-Hermite errors need the annulus luminosities")
        sig[n_r:] = s * np.repeat(lum, nmax)
    elif kin == "losvd":
        nv = layout["n_v"]
        h = rest.reshape(n_R, nv)
        peak = np.maximum(h.max(axis=1, keepdims=True), 1e-4 * max(h.max(), 1e-300))
        sig[n_r:] = (s * np.maximum(h, 0.01 * peak)).ravel()
    Y = Y_true + sig * g.standard_normal(Y_true.size)
    return Y, sig


def floor_model_noise(Y_true: np.ndarray, sigma: np.ndarray, n_model: int, mass=1.0):
    """Errors no smaller than the particle noise of an n_model-particle model:
    sigma^2 + 4 (|Y_true| + m1) m1 with m1 = mass / n_model (twice the Poisson
    error of a model observable carrying |Y_true| in particles of mass m1, and
    at least two particle masses where the target is empty). Data sets served
    to fits of at least n_model particles use it, so that no bin asks for
    more accuracy than the model's own sampling can give."""
    m1 = mass / float(n_model)
    return np.sqrt(sigma * sigma + 4.0 * (np.abs(Y_true) + m1) * m1)


def make_targets(observe, wl, lum=None):
    """Targets of workload ``wl`` measured by ``observe(V_p, sigma_p)`` on its
    target realization. Returns dict(Y, sigma, V_p, sigma_p, Y_true)."""
    lay = wl.layout
    n_R = lay["n_R"]
    V = np.zeros(n_R)
    sp = np.ones(n_R)
    if lay["kin"] == "gh":
        lum = annulus_luminosity(lay) if lum is None else lum
        V, sp = fit_gauss_hermite_centres(observe, lay, lum)
    Y_true = np.asarray(observe(V, sp), dtype=np.float64)
    Y, sig = add_noise(Y_true, lay, wl.noise, wl.noise_rng(), lum)
    return dict(Y=Y, sigma=sig, V_p=V, sigma_p=sp, Y_true=Y_true)
