"""Potential scans: fits of one data set in a family of potentials, stepped
together as one batch.

The paper determines the mass-to-light ratio of its galaxy models together
with their orbital structure (Sec. 5); the way it adjusts it is not part of
the paper. Here the potential is scanned instead: one fit per candidate
(mass-to-light ratio, halo), the same targets for all, every fit stepped in
one batched launch per step, and the chi^2 at the end of each fit ranks the
candidates. The parabola through the lowest chi^2 and its two neighbours
gives a value between grid points.
"""

from __future__ import annotations

import numpy as np

from .batch import Batch
from .fit import Fit


def scan(potentials, layout: dict, params, targets: dict, make_particles, n_steps: int,
         dtype: str = "f32", steps_per_launch: int = 64, max_fits: int = 64,
         hbm_budget: int = 0):
    """Final chi^2 of one fit per potential.

    potentials: potentials in the form ``Fit`` takes; params: step parameters,
    one dict for all or a callable potential -> dict (the prior grid's energy
    range depends on the potential); targets: dict with Y, sigma and for
    Gauss-Hermite layouts V_p, sigma_p; make_particles(potential) -> the
    initial particle arrays of that potential's fit (device or host). Fits
    are admitted as the batch's slots and HBM budget allow and run n_steps
    correction steps each.
    """
    fits = []
    try:
        for pot in potentials:
            par = params(pot) if callable(params) else params
            f = Fit(pot, layout, par, make_particles(pot), dtype=dtype)
            fits.append(f)
            f.set_targets(targets["Y"], targets["sigma"], targets.get("V_p"),
                          targets.get("sigma_p"))
        b = Batch(max_fits=max_fits, hbm_budget=hbm_budget)
        try:
            waiting = list(fits)
            while waiting or b.active:
                while waiting and b.admit(waiting[0], n_steps):
                    waiting.pop(0)
                if not b.active:
                    raise RuntimeError("a fit does not fit the batch's HBM budget")
                b.run(steps_per_launch)
                b.poll()
        finally:
            b.close()
        return np.array([f.observables()["chi2"] for f in fits])
    finally:
        for f in fits:
            f.close()


def best_of(values, chi2):
    """Value at the vertex of the parabola through the lowest chi^2 and its
    neighbours on the scan grid (the grid value itself at either end)."""
    v = np.asarray(values, dtype=np.float64)
    c = np.asarray(chi2, dtype=np.float64)
    i = int(np.argmin(c))
    if i == 0 or i == v.size - 1:
        return float(v[i])
    x0, x1, x2 = v[i - 1], v[i], v[i + 1]
    y0, y1, y2 = c[i - 1], c[i], c[i + 1]
    den = (x0 - x1) * (x0 - x2) * (x1 - x2)
    a = (x2 * (y1 - y0) + x1 * (y0 - y2) + x0 * (y2 - y1)) / den
    bb = (x2 * x2 * (y0 - y1) + x1 * x1 * (y2 - y0) + x0 * x0 * (y1 - y2)) / den
    if not a > 0:
        return float(x1)
    return float(np.clip(-bb / (2.0 * a), x0, x2))
