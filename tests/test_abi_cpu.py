"""The C-ABI library loads and exports every function the header declares;
host-only entry points answer without a GPU."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "m2m.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(m2m_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("m2m_create", "m2m_set_targets", "m2m_step", "m2m_update_priors",
              "m2m_get_weights", "m2m_destroy", "m2m_batch_run"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_1202_2355_amd import _abi
    lib = _abi.lib()
    for n in _declared():
        assert hasattr(lib, n), n
        assert isinstance(getattr(lib, n), ctypes._CFuncPtr)
    assert set(_abi.SIGNATURES) == set(_declared())


def test_host_only_entry_points():
    from paper_1202_2355_amd import _abi
    from workloads import workload
    wl = workload(3)
    assert _abi.m2m_num_observables(wl.layout) == 50 + 40 * 64
    bad = dict(wl.layout, n_r=0)
    assert _abi.m2m_num_observables(bad) == 0
    assert _abi.m2m_workspace_bytes(wl.layout, wl.params, wl.N) > 0
    assert _abi.m2m_workspace_bytes(wl.layout, wl.params, 0) == 0
    # prior smoothing: grids of at most 128 cells per side
    assert _abi.m2m_workspace_bytes(wl.layout, dict(wl.params, smooth=1), wl.N) > 0
    assert _abi.m2m_workspace_bytes(wl.layout, dict(wl.params, smooth=1, n_E=200, n_x=2),
                                    wl.N) == 0
    assert _abi.m2m_workspace_bytes(wl.layout, dict(wl.params, smooth=2), wl.N) == 0
    # spherical-harmonic density observables: (l_max + 1)^2 per mesh radius
    alm = dict(wl.layout, n_r=60, dens="alm", l_max=4)
    assert _abi.m2m_num_observables(alm) == 60 * 25 + 40 * 64
    assert _abi.m2m_num_observables(dict(alm, l_max=9)) == 0
    assert _abi.m2m_num_observables(dict(alm, l_max=-1)) == 0
    assert _abi.m2m_num_observables(dict(alm, n_r=1)) == 0
    assert _abi.m2m_num_observables(dict(alm, dens=2)) == 0
    assert _abi.m2m_num_observables(dict(alm, n_r=200, l_max=8)) == 0  # J > 16384
    # self-consistent potential: 2..64 nodes, degree 0..8, 0 < r_min < r_max,
    # rebuilt every >= 1 steps; its interval sums and node table add to the
    # workspace
    scf = dict(wl.params, scf_lmax=4, scf_nr=32, scf_rmin=0.02, scf_rmax=100.0, scf_every=10)
    w0 = _abi.m2m_workspace_bytes(wl.layout, wl.params, wl.N)
    assert _abi.m2m_workspace_bytes(wl.layout, scf, wl.N) > w0
    for bad in (dict(scf_nr=1), dict(scf_nr=65), dict(scf_lmax=9), dict(scf_lmax=-1),
                dict(scf_rmin=0.0), dict(scf_rmax=0.01), dict(scf_every=0),
                dict(scf_rmin=float("nan"))):
        assert _abi.m2m_workspace_bytes(wl.layout, dict(scf, **bad), wl.N) == 0, bad
    assert _abi.m2m_workspace_bytes(wl.layout, dict(scf, scf_nr=0, scf_lmax=99), wl.N) == w0
    b0 = _abi.m2m_get_launch()
    with pytest.raises(_abi.M2MError):
        _abi.m2m_set_launch(300, 4)
    _abi.m2m_set_launch(512, 2)
    assert _abi.m2m_get_launch() == (512, 2)
    _abi.m2m_set_launch(*b0)


def test_create_rejects_bad_arguments_without_touching_memory():
    import ctypes as C
    from paper_1202_2355_amd import _abi
    from workloads import workload
    wl = workload(1)
    ctx = C.c_void_p()
    ptrs = [C.c_void_p(0)] * 8   # NULL arrays are rejected before any device call
    st = _abi.lib().m2m_create(C.byref(_abi.potential(wl.potential)),
                               C.byref(_abi.obs_layout(wl.layout)), C.byref(_abi.params(wl.params)),
                               100, 0, *ptrs, None, 0, None, C.byref(ctx))
    assert st == _abi.M2M_EINVAL and not ctx.value
    bad = dict(wl.params, dt=-1.0)
    st = _abi.lib().m2m_create(C.byref(_abi.potential(wl.potential)),
                               C.byref(_abi.obs_layout(wl.layout)), C.byref(_abi.params(bad)),
                               100, 0, *([C.c_void_p(4096)] * 8), None, 0, None, C.byref(ctx))
    assert st == _abi.M2M_EINVAL
    # an empty fit, an unknown dtype and a misaligned array are refused before
    # the pointers are used (4096 and 4104 are never dereferenced)
    for n, dtype, ptrs in ((0, 0, [C.c_void_p(4096)] * 8), (100, 7, [C.c_void_p(4096)] * 8),
                           (100, 0, [C.c_void_p(4096)] * 7 + [C.c_void_p(4104)])):
        ctx = C.c_void_p()
        st = _abi.lib().m2m_create(C.byref(_abi.potential(wl.potential)),
                                   C.byref(_abi.obs_layout(wl.layout)), C.byref(_abi.params(wl.params)),
                                   n, dtype, *ptrs, None, 0, None, C.byref(ctx))
        assert st == _abi.M2M_EINVAL and not ctx.value, (n, dtype)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built HIP library every entry point raises."""
    from paper_1202_2355_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB", str(tmp_path / "libm2m.so"))
    with pytest.raises(ImportError, match="missing"):
        _abi.lib()


def test_observe_noalloc_rejects_before_touching_memory():
    """The allocation-free observation refuses bad arguments, and layouts and
    particle counts beyond its static scratch, before any device call (the
    addresses 4096... are never dereferenced)."""
    from paper_1202_2355_amd import _abi
    from workloads import workload
    wl = workload(3)
    fake = [4096 * (k + 1) for k in range(7)]
    with pytest.raises(_abi.M2MError, match="16-byte aligned"):
        _abi.m2m_observe_noalloc(wl.layout, 1.0, 100, "f32", fake[:6] + [0])
    with pytest.raises(_abi.M2MError, match="mass"):
        _abi.m2m_observe_noalloc(wl.layout, -1.0, 100, "f32", fake)
    with pytest.raises(_abi.M2MError, match="n_r"):
        _abi.m2m_observe_noalloc(dict(wl.layout, n_r=0), 1.0, 100, "f32", fake)
    gh = workload(2)
    with pytest.raises(_abi.M2MError, match="V_p and sigma_p"):
        _abi.m2m_observe_noalloc(gh.layout, 1.0, 100, "f32", fake)
    before = _abi.m2m_get_launch()
    try:
        # 4096 tile rows of 2612 doubles (86 MB) do not fit the 32 MiB scratch
        _abi.m2m_set_launch(1024, 16)
        with pytest.raises(_abi.M2MError, match="static scratch") as e:
            _abi.m2m_observe_noalloc(wl.layout, 1.0, 8_000_000, "f32", fake)
        assert e.value.status == _abi.M2M_ENOMEM
    finally:
        _abi.m2m_set_launch(*before)
