"""Host-side admission rules of the serving loop, without a GPU: a request
whose footprint exceeds the whole HBM budget, or that the library refuses,
is rejected at once instead of blocking the queue behind it."""

from workloads import make_params, make_potential, workload


def _req(n, rid=0, **par):
    from paper_1202_2355_amd.serve import Request
    wl = workload(3)
    pot = make_potential(upsilon=1.0, M200=10.0, c=8.0)
    p = dict(make_params(pot, n_E=64, n_x=32), **par)
    return Request(rid=rid, arrival=0.0, potential=pot, params=p, layout=wl.layout, n=n,
                   steps=10, dataset=0, seed=0)


def test_footprint_counts_state_and_workspace():
    from paper_1202_2355_amd import _abi
    from paper_1202_2355_amd.serve import footprint_bytes
    r = _req(100_000)
    ws = _abi.m2m_workspace_bytes(r.layout, r.params, r.n, "f32")
    assert ws > 0
    assert footprint_bytes(r, "f32") == 32 * r.n + ws
    assert footprint_bytes(r, "f64") == 64 * r.n + _abi.m2m_workspace_bytes(
        r.layout, r.params, r.n, "f64")


def test_oversized_and_invalid_requests_are_refused():
    from paper_1202_2355_amd.serve import footprint_bytes, refusal
    small, big = _req(100_000, 0), _req(4_000_000, 1)
    budget = footprint_bytes(small, "f32") * 3
    assert refusal(small, "f32", budget) == ""
    assert "exceeds the HBM budget" in refusal(big, "f32", budget)
    # the same request fits a budget that holds it, however tight
    assert refusal(big, "f32", footprint_bytes(big, "f32")) == ""
    # parameters the library refuses (a grid too large to smooth)
    bad = _req(1000, 2, smooth=1, n_E=64, n_x=64)
    assert "invalid" in refusal(bad, "f32", 1 << 40)
