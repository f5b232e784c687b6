"""GPU parity of the self-consistent stellar potential (Sec. 2.1; Sec. 5)
against the FP64 oracle (run on an MI355X).

Criteria
* node table built from one state: |t_gpu - t_ora| <= rel * the largest
  |entry| of its (l, m) column (values and slopes separately); rel = 1e-12
  for FP64 particle state, 2e-5 for FP32 (each term is rounded to float, the
  sums are FP64);
* runs: positions within 1e-9, weights within 1e-10 and chi^2 within 1e-9
  relative for FP64 state; weights within 1e-4 for FP32 state (as the runs in
  the analytic potential), and the node table at the end of the run.
"""

import sys

import numpy as np
import pytest

from m2m_testlib import cast, oracle_targets, random_weights, weight_errors
from workloads import with_scf, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def Fit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1202_2355_amd import _abi
    _abi.lib()
    from paper_1202_2355_amd.fit import Fit
    return Fit


def _assert_table(tab, ref, rel, what):
    assert tab.shape == ref.shape
    for c in (0, 1):
        scale = np.abs(ref[:, :, c]).max(axis=0)  # per (l, m) column
        err = np.abs(tab[:, :, c] - ref[:, :, c]).max(axis=0)
        worst = float(np.max(err / scale))
        _say(what, "value" if c == 0 else "slope", "max err / column scale", worst)
        assert worst <= rel, (what, c, worst)


def _oracle_table(oracle, wl, parts, u):
    pot = dict(wl.potential.as_dict(), **{k: wl.params[k] for k in oracle.SCF_KEYS})
    return oracle.scf_table(pot, parts, u, mass=wl.params["mass"], nthreads=8)


@pytest.mark.parametrize("dtype,l_max,n_nodes", [("f32", 4, 24), ("f64", 4, 24), ("f64", 0, 2),
                                                ("f32", 8, 40)])
def test_table_of_one_state_matches_oracle(oracle, Fit, dtype, l_max, n_nodes):
    """Also the smallest expansion (the monopole on two nodes: one interval
    between the core and the outside) and a large one (l <= 8, 40 nodes)."""
    wl = with_scf(workload(2), l_max=l_max, n_nodes=n_nodes, r_min=0.02, r_max=80.0)
    n = 60_001
    _say("scf table", dtype, l_max, n_nodes, n)
    parts = cast(wl.initial_particles(n=n, seed=41), dtype)
    u = cast({"u": random_weights(n, 43, spread=0.5)}, dtype)["u"]
    T = oracle_targets(oracle, wl)
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype, u=u)
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])  # builds the expansion
    tab = f.potential_table()
    ref = _oracle_table(oracle, wl, parts, u)
    _assert_table(tab, ref, 2e-5 if dtype == "f32" else 1e-12, f"scf table {dtype}")
    f.close()


def _scf_pair(oracle, Fit, wl, n, dtype, band, seed):
    T = oracle_targets(oracle, wl)
    parts = cast(wl.initial_particles(n=n, seed=seed), dtype)
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype)
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    o = oracle.OracleFit(wl.potential, wl.layout, wl.params, parts, T["Y"], T["sigma"], T["V_p"],
                         T["sigma_p"], track_flags=True, band=band, nthreads=8)
    return f, o


@pytest.mark.parametrize("l_max", [2, 3, 4])
def test_scf_run_fp64_matches_oracle(oracle, Fit, l_max):
    """FP64 state, workload 1 in its own multipole potential (16 nodes,
    rebuilt every 5 steps): 40 steps with a prior refresh. l <= 2 and 4 take
    the force with unrolled loops, l <= 3 the one with the degree at run time."""
    wl = with_scf(workload(1), l_max=l_max, n_nodes=16, r_min=0.05, r_max=50.0, every=5)
    wl = wl.with_(params=dict(wl.params, prior_every=20))
    n = 20_003
    _say("scf run fp64", wl.name, l_max, n)
    f, o = _scf_pair(oracle, Fit, wl, n, "f64", 1e-12, seed=45)
    f.step(40)
    hist_o = o.step(40)
    hist_g = f.chi2_history(40)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("scf run fp64: rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(st[k], o.arr[k], rtol=0, atol=1e-9)
    assert r2 <= 1e-10
    assert rmax <= 1e-10
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-9)
    _assert_table(f.potential_table(), o.scf.reshape(f.potential_table().shape), 1e-9,
                  "scf run fp64 table")
    f.close()


def test_scf_run_fp32_matches_oracle(oracle, Fit):
    """FP32 state, workload 2 in its own multipole potential (l <= 4, 32
    nodes, rebuilt every 10 steps): weights after 30 steps."""
    wl = with_scf(workload(2), l_max=4, n_nodes=32, r_min=0.02, r_max=100.0, every=10)
    n = 30_001
    _say("scf run fp32", wl.name, n)
    f, o = _scf_pair(oracle, Fit, wl, n, "f32", 1e-5, seed=47)
    f.step(30)
    hist_o = o.step(30)
    hist_g = f.chi2_history(30)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("scf run fp32: rel2", r2, "max(unflagged)", rmax, "max(all)", rall, "flagged", frac)
    assert r2 <= 1e-4
    assert rmax <= 1e-4
    np.testing.assert_allclose(hist_g, hist_o, rtol=1e-4)
    _assert_table(f.potential_table(), o.scf.reshape(f.potential_table().shape), 1e-4,
                  "scf run fp32 table")
    f.close()


def test_expansion_too_large_for_lds_is_refused(oracle, Fit):
    """l <= 8 on 64 nodes needs more than the 160 KiB of LDS of a CU for its
    interval table and sums: creation fails cleanly."""
    from paper_1202_2355_amd._abi import M2M_EUNSUPPORTED, M2MError
    wl = with_scf(workload(2), l_max=8, n_nodes=64, r_min=0.02, r_max=80.0)
    parts = cast(wl.initial_particles(n=4_096, seed=57), "f32")
    with pytest.raises(M2MError) as e:
        Fit(wl.potential, wl.layout, wl.params, parts, dtype="f32")
    assert e.value.status == M2M_EUNSUPPORTED


def test_monopole_on_two_nodes_run_fp64_matches_oracle(oracle, Fit):
    """The degenerate expansion: l = 0, nodes at r_min and r_max only, so
    most particles sit in the one interval or beyond the last node."""
    wl = with_scf(workload(1), l_max=0, n_nodes=2, r_min=0.3, r_max=3.0, every=3)
    n = 10_007
    _say("scf monopole two nodes fp64", n)
    f, o = _scf_pair(oracle, Fit, wl, n, "f64", 1e-12, seed=55)
    f.step(20)
    hist_o = o.step(20)
    st = f.particles()
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(st[k], o.arr[k], rtol=0, atol=1e-9)
    np.testing.assert_allclose(f.chi2_history(20), hist_o, rtol=1e-9)
    f.close()


def test_refresh_potential_rebuilds_from_the_current_state(oracle, Fit):
    """After 7 steps (last rebuild at step 5) an explicit rebuild gives the
    expansion of the particles and weights as they are now."""
    wl = with_scf(workload(1), l_max=3, n_nodes=20, r_min=0.05, r_max=50.0, every=5)
    n = 12_007
    _say("scf refresh", n)
    f, o = _scf_pair(oracle, Fit, wl, n, "f64", 1e-12, seed=49)
    f.step(7)
    before = f.potential_table()
    f.refresh_potential()
    after = f.potential_table()
    st = f.particles()
    ref = _oracle_table(oracle, wl, st, st["u"])
    _assert_table(after, ref, 1e-12, "scf refresh")
    assert not np.array_equal(before, after)
    f.close()


def test_scf_batch_equals_alone(oracle, Fit):
    """Two fits with the expansion stepped in one batch: the same results as
    each alone (the rebuild runs in the batched finalize)."""
    from paper_1202_2355_amd.batch import Batch
    wl = with_scf(workload(2), l_max=2, n_nodes=16, r_min=0.02, r_max=100.0, every=4)
    T = oracle_targets(oracle, wl)
    sizes, steps = [9_001, 20_011], [12, 9]
    _say("scf batch vs alone", sizes, steps)
    parts = [cast(wl.initial_particles(n=n, seed=50 + k), "f32") for k, n in enumerate(sizes)]
    alone = []
    for k in range(2):
        f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        f.step(steps[k])
        alone.append((f.particles()["u"], f.potential_table()))
        f.close()
    b = Batch(max_fits=4)
    fits = []
    for k in range(2):
        f = Fit(wl.potential, wl.layout, wl.params, parts[k], dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        b.admit(f, steps[k])
        fits.append(f)
    assert len(b.run_to_completion(steps_per_launch=4)) == 2
    for k, f in enumerate(fits):
        np.testing.assert_allclose(f.particles()["u"], alone[k][0], rtol=1e-5)
        _assert_table(f.potential_table(), alone[k][1], 1e-6, "scf batch table")
        f.close()
    b.close()


def test_long_fp32_run_with_mass_beyond_the_last_node_stays_finite(oracle, Fit):
    """l <= 4 with the last node at r = 20 (a tenth of the mass beyond it):
    after 300 steps every particle is finite and chi^2 stays near that of the
    same run in the analytic potential (the expansion decays beyond the last
    node instead of growing like r^l)."""
    base = workload(2)
    wl = with_scf(base, l_max=4, n_nodes=24, r_min=0.02, r_max=20.0, every=5)
    T = oracle_targets(oracle, base)
    n = 100_003
    _say("scf long fp32", n)
    parts = cast(base.initial_particles(n=n, seed=53), "f32")
    chi = {}
    for name, w in (("analytic", base), ("scf", wl)):
        f = Fit(w.potential, w.layout, w.params, parts, dtype="f32")
        f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
        f.step(300)
        st = f.particles()
        assert all(np.all(np.isfinite(st[k])) for k in ("x", "y", "z", "vx", "vy", "vz")), name
        chi[name] = f.observables()["chi2"]
        if name == "scf":
            assert np.all(np.isfinite(f.potential_table()))
        f.close()
    _say("scf long fp32 chi2", chi)
    assert chi["scf"] < 3.0 * chi["analytic"]


def test_checkpoint_resume_keeps_the_expansion(oracle, Fit):
    """The state blob carries the node table: a fit resumed from a state saved
    between two rebuilds continues exactly like the uninterrupted run."""
    wl = with_scf(workload(1), l_max=2, n_nodes=16, r_min=0.05, r_max=50.0, every=5)
    T = oracle_targets(oracle, wl)
    n = 12_011
    _say("scf checkpoint", n)
    parts = cast(wl.initial_particles(n=n, seed=59), "f64")
    f = Fit(wl.potential, wl.layout, wl.params, parts, dtype="f64")
    f.set_targets(T["Y"], T["sigma"], T["V_p"], T["sigma_p"])
    f.step(7)  # last rebuild after step 5: the table is not that of the current particles
    blob = f.get_state()
    mid = f.particles()
    mid_tab = f.potential_table()
    f.step(6)
    end, end_tab = f.particles(), f.potential_table()
    g = Fit(wl.potential, wl.layout, wl.params,
            {k: mid[k] for k in ("x", "y", "z", "vx", "vy", "vz")}, dtype="f64", u=mid["u"],
            u_prior=mid["uh"])
    g.set_state(blob)
    assert np.array_equal(g.potential_table(), mid_tab)
    g.step(6)
    end2 = g.particles()
    for k in ("x", "y", "z", "vx", "vy", "vz", "u"):
        np.testing.assert_allclose(end2[k], end[k], rtol=1e-12, atol=1e-12)
    _assert_table(g.potential_table(), end_tab, 1e-12, "scf checkpoint table")
    f.close()
    g.close()


def test_scf_with_alm_observables_run_fp64_matches_oracle(oracle, Fit):
    """The paper's pairing: spherical-harmonic density observables (l <= 2 on
    30 mesh radii) in a fit whose stellar potential is its own expansion
    (l <= 2, 16 nodes, rebuilt every 4 steps)."""
    from workloads import with_alm
    wl = with_scf(with_alm(workload(1), n_mesh=30, l_max=2), l_max=2, n_nodes=16, r_min=0.05,
                  r_max=50.0, every=4)
    n = 15_013
    _say("scf + alm run fp64", wl.name, n)
    f, o = _scf_pair(oracle, Fit, wl, n, "f64", 1e-12, seed=63)
    f.step(24)
    hist_o = o.step(24)
    st = f.particles()
    r2, rmax, rall, frac = weight_errors(st["u"], o.arr["u"], o.flag)
    _say("scf + alm run fp64: rel2", r2, "max(unflagged)", rmax, "flagged", frac)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(st[k], o.arr[k], rtol=0, atol=1e-9)
    assert r2 <= 1e-10 and rmax <= 1e-10
    np.testing.assert_allclose(f.chi2_history(24), hist_o, rtol=1e-9)
    f.close()
