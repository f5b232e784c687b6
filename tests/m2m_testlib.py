"""Shared helpers of the parity tests: seeded inputs, oracle-made targets and
the comparison criteria. Inputs come from ``workloads``; expected values from
the FP64 oracle only."""

from __future__ import annotations

import numpy as np

from workloads import make_targets, rng

FIELDS = ("x", "y", "z", "vx", "vy", "vz")

# relative distance to an edge within which FP32 and FP64 may bin a point
# differently: 4 ulps of float32 (2^-21)
BAND_F32 = 4.0 * 2.0 ** -23
BAND_F64 = 4.0 * 2.0 ** -52


def cast(parts: dict, dtype: str) -> dict:
    """Round a float64 particle dict to the GPU dtype and back to float64, so
    the oracle and the GPU start from the identical state."""
    t = np.float32 if dtype == "f32" else np.float64
    return {k: np.asarray(v, dtype=t).astype(np.float64) for k, v in parts.items()}


def oracle_targets(O, wl, n_target=1 << 18, nthreads=8):
    """Targets of workload ``wl`` measured by the oracle on a seeded target
    realization (Sec. 3.1: targets are observables of a target model)."""
    tp = wl.target_particles(n=n_target)
    ones = np.ones(tp["x"].size)

    def observe(V, S):
        return O.deposit(tp, ones, wl.layout, mass=wl.params["mass"], V_p=V, sigma_p=S,
                         nthreads=nthreads)

    return make_targets(observe, wl)


def random_weights(n, seed, spread=0.3):
    g = rng(seed)
    return np.exp(spread * g.standard_normal(n))


def observable_tolerance(yabs, yamb, rel):
    """|y_gpu - y_oracle| <= rel * sum|w K| + sum over edge-ambiguous |w K|."""
    return rel * yabs + yamb


def assert_observables(y_gpu, y_ora, yabs, yamb, rel, what=""):
    tol = observable_tolerance(yabs, yamb, rel)
    err = np.abs(np.asarray(y_gpu) - y_ora)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{what}: {bad.size} observables out of tolerance; worst j="
                           f"{bad[np.argmax(err[bad] / np.maximum(tol[bad], 1e-300))]}, "
                           f"err={err[bad].max():.3e}")
    scale = np.maximum(yabs, 1e-300)
    return float(np.max(err / scale))


def weight_errors(u_gpu, u_ora, flagged=None):
    u_gpu = np.asarray(u_gpu, dtype=np.float64)
    rel2 = float(np.linalg.norm(u_gpu - u_ora) / np.linalg.norm(u_ora))
    relmax = np.abs(u_gpu / u_ora - 1.0)
    if flagged is not None:
        ok = flagged == 0
        return rel2, float(relmax[ok].max()) if ok.any() else 0.0, float(relmax.max()), float(
            (~ok).mean())
    return rel2, float(relmax.max()), float(relmax.max()), 0.0


def _cell_of_coords(par, E, xc, lzneg):
    """Prior cell of energy E, circularity xc and L_z sign (Sec. 2.3.1 with
    the clamping into the end cells and the options of Sec. 5)."""
    nE, nx, cells = int(par["n_E"]), int(par["n_x"]), int(par.get("cells", 0))
    if cells & 2:
        t = (np.exp(E) - np.exp(par["E_lo"])) / (np.exp(par["E_hi"]) - np.exp(par["E_lo"])) * nE
    else:
        t = (E - par["E_lo"]) / (par["E_hi"] - par["E_lo"]) * nE
    k = np.where(E - par["E_lo"] >= 0.0, np.floor(t), 0.0)
    k = np.clip(k, 0, nE - 1).astype(np.int64)
    l = np.clip(np.floor(xc * nx), 0, nx - 1).astype(np.int64)
    c = k * nx + l
    if cells & 1:
        c = c + np.where(lzneg, nE * nx, 0)
    return c


def candidate_cells(O, pot, par, parts, band):
    """Cells a particle may be binned into when its coordinates are rounded
    differently: its (E, x = L/L_c) moved by twice the oracle's flag band
    (band |E_lo| in E, band in x) either way, and the other L_z half where
    |L_z|/(r v) is within the band. Array (n, 18), column 0 the particle's
    own cell."""
    q = {k: np.asarray(parts[k], dtype=np.float64) for k in FIELDS}
    c0, E, xc = O.cells(pot, par, q)
    lz = q["x"] * q["vy"] - q["y"] * q["vx"]
    rv = np.sqrt(q["x"] ** 2 + q["y"] ** 2 + q["z"] ** 2) * np.sqrt(
        q["vx"] ** 2 + q["vy"] ** 2 + q["vz"] ** 2)
    lzr = np.where(rv > 0, lz / np.maximum(rv, 1e-300), 0.0)
    dE = 2.0 * band * abs(par["E_lo"])
    dx = 2.0 * band
    neg = lz < 0.0
    flip = np.abs(lzr) <= band
    out = [c0]
    for sE in (-1, 0, 1):
        for sx in (-1, 0, 1):
            for fl in (False, True):
                if not fl and sE == 0 and sx == 0:
                    continue
                ln = np.where(fl & flip, ~neg, neg)
                out.append(_cell_of_coords(par, E + sE * dE, xc + sx * dx, ln))
    return np.stack(out, axis=1)


def prior_bounds(O, pot, par, parts, u, flagged, band, empty=1.0):
    """Bounds on each particle's new prior (the mean u of its cell, Sec.
    2.3.1) that hold whichever side of an edge the flagged particles (those
    the oracle saw within ``band`` of a cell edge) are binned on.

    For a cell c with the oracle's sum S and count n, moving particles in or
    out changes the mean by at most sum |u_k - mean_c| over the particles that
    may enter or leave it, divided by n minus the number that may leave. A
    flagged particle's own prior may be the mean of any of its candidate
    cells. Cells that might be emptied, and cells without particles, are not
    bounded (their prior is the previous one, ``empty``)."""
    cell, _, _ = O.cells(pot, par, parts)
    C = O.n_cells(par)
    u = np.asarray(u, dtype=np.float64)
    S = np.bincount(cell, weights=u, minlength=C)
    n = np.bincount(cell, minlength=C).astype(np.float64)
    mean = np.where(n > 0, S / np.maximum(n, 1), empty)
    idx = np.nonzero(np.asarray(flagged) != 0)[0]
    cand = candidate_cells(O, pot, par, {k: np.asarray(parts[k])[idx] for k in FIELDS}, band)
    num = np.zeros(C)
    leave = np.zeros(C)
    for r, i in enumerate(idx):
        cs = np.unique(cand[r])
        if cs.size > 1:
            for c in cs:
                num[c] += abs(u[i] - mean[c])
            leave[cell[i]] += 1
    left = n - leave
    dev = np.where(left > 0, num / np.maximum(left, 1), np.inf)
    dev = np.where(n > 0, dev, np.inf)
    lo = mean[cell] - dev[cell]
    hi = mean[cell] + dev[cell]
    for r, i in enumerate(idx):
        cs = np.unique(cand[r])
        lo[i] = np.min(mean[cs] - dev[cs])
        hi[i] = np.max(mean[cs] + dev[cs])
    return lo, hi


def assert_priors_within(uh, lo, hi, rtol, what=""):
    """Every particle's prior inside its bounds (widened by rtol); returns the
    fraction of particles with an unbounded prior (a cell that may empty)."""
    uh = np.asarray(uh, dtype=np.float64)
    fin = np.isfinite(lo) & np.isfinite(hi)
    bad = fin & ((uh < lo - rtol * np.abs(lo)) | (uh > hi + rtol * np.abs(hi)))
    assert not bad.any(), (f"{what}: {int(bad.sum())} priors out of bounds; first at "
                           f"{int(np.argmax(bad))}: {uh[bad][0]} not in [{lo[bad][0]}, {hi[bad][0]}]")
    return float((~fin).mean())
