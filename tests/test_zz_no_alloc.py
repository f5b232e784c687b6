"""The allocation-free observation (m2m_observe_noalloc, its working memory in
the library's static device scratch) against m2m_observe of a context over
the same particles: calls in a row on one GPU, the second with fewer
particles than the first (the scratch keeps the first call's tile rows), then
other kinds of observables and the FP64 state."""

import numpy as np
import pytest
import torch

from paper_1202_2355_amd import _abi as A

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u")


@pytest.fixture(scope="module")
def Fit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A.lib()
    from paper_1202_2355_amd.fit import Fit
    return Fit


def _fit_over(Fit, wl, n, seed, dtype):
    from workloads.device import om_model_device
    tdt = torch.float64 if dtype == "f64" else torch.float32
    parts = om_model_device(n, wl.potential, 1.0, seed=seed, dtype=tdt)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed + 7)
    u = (0.25 + 1.5 * torch.rand(n, generator=g, device="cuda", dtype=torch.float64)).to(tdt)
    fit = Fit(wl.potential, wl.layout, wl.params, parts, dtype=dtype, u=u)
    torch.cuda.synchronize()
    return fit


def _gh_centres(layout):
    n_R = layout["n_R"]
    return np.linspace(-0.05, 0.05, n_R), np.linspace(0.2, 0.6, n_R)


def _noalloc(fit, wl, dtype, V=None, S=None):
    ptrs = [fit.t[k].data_ptr() for k in FIELDS]
    torch.cuda.synchronize()
    return A.m2m_observe_noalloc(wl.layout, wl.params["mass"], fit.n, dtype, ptrs, V, S)


def _assert_same(y, ref, what):
    # the same kernels; tiles may differ (no prior cells), so the FP64 sums
    # may differ in their last bits
    assert y.shape == ref.shape, what
    assert np.all(np.isfinite(y)), what
    scale = np.max(np.abs(ref))
    assert scale > 0, what
    err = np.abs(y - ref)
    bound = 1e-12 * np.abs(ref) + 1e-13 * scale
    assert np.all(err <= bound), (what, float(np.max(err / (np.abs(ref) + scale))))


def test_noalloc_observation_matches_the_context_twice_in_a_row(Fit):
    from workloads import workload
    wl = workload(2)                         # Gauss-Hermite, FP32 state
    V, S = _gh_centres(wl.layout)
    for n, seed in ((300_001, 11), (70_001, 12)):
        print(f"[noalloc] GH f32 n={n} seed={seed}", flush=True)
        fit = _fit_over(Fit, wl, n, seed, "f32")
        ref = fit.observe(V, S)
        y = _noalloc(fit, wl, "f32", V, S)
        _assert_same(y, ref, f"gh n={n}")
        fit.close()


def test_noalloc_observation_other_layouts_and_fp64(Fit):
    from workloads import workload
    cases = (
        (workload(3), 150_001, "f32", 21),    # LOSVD, 2610 observables
        (workload(1), 20_001, "f64", 22),     # v^2 moments, FP64 state
        (workload(2), 1, "f32", 23),          # a single particle
    )
    for wl, n, dtype, seed in cases:
        print(f"[noalloc] {wl.name} {dtype} n={n}", flush=True)
        V, S = _gh_centres(wl.layout) if wl.layout["kin"] == "gh" else (None, None)
        fit = _fit_over(Fit, wl, n, seed, dtype)
        ref = fit.observe(V, S)
        y = _noalloc(fit, wl, dtype, V, S)
        if n == 1:
            assert np.array_equal(y, ref), wl.name
        else:
            _assert_same(y, ref, wl.name)
        fit.close()


def test_noalloc_observation_refuses_more_than_its_scratch(Fit):
    from workloads import workload
    wl = workload(3)
    n_big = 8_000_000
    # real arrays of n_big particles, so that nothing could read out of bounds
    big = torch.zeros(7, n_big, dtype=torch.float32, device="cuda")
    big[6].fill_(1.0)
    torch.cuda.synchronize()
    before = A.m2m_get_launch()
    try:
        A.m2m_set_launch(1024, 16)   # 4096 tile rows of 2612 doubles: 86 MB
        with pytest.raises(A.M2MError, match="static scratch"):
            A.m2m_observe_noalloc(wl.layout, wl.params["mass"], n_big, "f32",
                                  [big[i].data_ptr() for i in range(7)])
    finally:
        A.m2m_set_launch(*before)
    del big
    # the next call still works
    fit = _fit_over(Fit, wl, 200_001, 31, "f32")
    ref = fit.observe()
    _assert_same(_noalloc(fit, wl, "f32"), ref, "after a refusal")
    fit.close()
