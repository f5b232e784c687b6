"""Potential scan on the GPU: fits of one data set in potentials of
different mass-to-light ratio, stepped as one batch, rank the candidates."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def test_upsilon_scan_recovers_the_mass_to_light_ratio_of_the_targets():
    """Targets from an isotropic model in the potential with upsilon = 1.2;
    every fit starts from the isotropic model of its own potential, so the
    candidates differ only in upsilon (an anisotropic target would bring in
    the mass-anisotropy degeneracy, which a short fit does not resolve)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_2355_amd.fit import Fit
    from paper_1202_2355_amd.scan import best_of, scan
    from workloads import make_layout, make_params, make_potential, make_targets
    from workloads.configs import Workload
    from workloads.device import om_model_device

    ups_true = 1.2
    pot_t = make_potential(upsilon=ups_true, M200=10.0, c=8.0)
    lay = make_layout(30, 0.05, 20.0, 20, 0.05, 20.0, "v2")
    wl = Workload("scan_target", 20_000, "f32", pot_t, lay, make_params(pot_t, n_E=20, n_x=10),
                  300, "iso_in_pot", float("inf"), 0.02, 1 << 18, seed=31)
    tp = om_model_device(wl.n_target, pot_t, wl.target_ra, seed=311)
    tf = Fit(pot_t, lay, wl.params, tp, dtype="f32")
    T = make_targets(lambda V, S: tf.observe(V, S), wl)
    tf.close()
    ups = [0.8, 1.0, 1.2, 1.4, 1.6]
    pots = [make_potential(upsilon=u, M200=10.0, c=8.0) for u in ups]
    _say("scan", ups, "N", wl.N, "steps", wl.steps)
    chi2 = scan(pots, lay, lambda p: make_params(p, n_E=20, n_x=10), T,
                lambda p: om_model_device(wl.N, p, float("inf"), seed=312), wl.steps)
    best = best_of(ups, chi2)
    _say("scan chi2/J", np.round(chi2 / wl.J, 3), "best", best)
    assert int(np.argmin(chi2)) == ups.index(ups_true)
    assert abs(best - ups_true) < 0.15
