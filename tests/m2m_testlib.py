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


def clean_of_cell_edges(P, cell, E, xc, band_e, band_x):
    """Particles whose prior cell is certain in a comparison of cell means:
    not in a cell that holds a particle within the band of a cell edge (in E
    or in x = L/L_c), nor in the cell across that edge, where such a particle
    may land when its coordinates are rounded differently. Cells linear in E,
    without the L_z split."""
    import numpy as np
    dE = (P["E_hi"] - P["E_lo"]) / P["n_E"]
    te = (E - P["E_lo"]) / dE
    tx = xc * P["n_x"]
    amb_e = np.abs(te - np.round(te)) * dE <= band_e
    amb_x = np.abs(tx - np.round(tx)) <= band_x * P["n_x"]
    k, l = np.divmod(cell, P["n_x"])
    k_o = np.where(te >= np.round(te), np.round(te) - 1, np.round(te)).astype(int)
    l_o = np.where(tx >= np.round(tx), np.round(tx) - 1, np.round(tx)).astype(int)
    k2 = np.where(amb_e, np.clip(k_o, 0, P["n_E"] - 1), k)
    l2 = np.where(amb_x, np.clip(l_o, 0, P["n_x"] - 1), l)
    amb = amb_e | amb_x
    dirty = np.zeros(P["n_E"] * P["n_x"], bool)
    for kk, ll in ((k, l), (k2, l), (k, l2), (k2, l2)):
        dirty[(kk * P["n_x"] + ll)[amb]] = True
    return ~dirty[cell]
