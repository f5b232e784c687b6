"""The library's host-side eigendecomposition of the prior-smoothing penalty
(Sec. 2.3.2, eq. smooth_grid), which the device smoother works in, checked
without a GPU: expanded from its parity blocks it must reproduce the penalty
written as finite differences with array slices, be orthonormal, and filter
a grid at any lambda as the oracle's dense solve does."""

import numpy as np
import pytest

from test_oracle_smoothing import _penalty_matrix


def _axis_basis(n, p):
    """The parity vectors of an axis of n cells (columns)."""
    m = (n + 1) // 2 if p == 0 else n // 2
    T = np.zeros((n, m))
    for i in range(m):
        j = n - 1 - i
        if i == j:
            T[i, i] = 1.0
        else:
            T[i, i] = np.sqrt(0.5)
            T[j, i] = np.sqrt(0.5) * (1 if p == 0 else -1)
    return T


def _expand(basis, nE, nx):
    """Full eigenvalues g (n) and eigenvectors Q (n x n, columns) in cell
    order k n_x + l, from the blocked layout."""
    n = nE * nx
    g = basis[:n]
    off = n
    cols = []
    for b in range(4):
        TE, TX = _axis_basis(nE, b >> 1), _axis_basis(nx, b & 1)
        m = TE.shape[1] * TX.shape[1]
        Z = basis[off:off + m * m].reshape(m, m)
        off += m * m
        if m:
            cols.append(np.kron(TE, TX) @ Z)
    assert off == basis.size
    return g, np.hstack(cols)


@pytest.mark.parametrize("shape", [(16, 8), (9, 6), (3, 7), (1, 5), (2, 2), (20, 10), (13, 1)])
def test_basis_diagonalizes_the_thin_plate_penalty(shape):
    from paper_1202_2355_amd import _abi
    nE, nx = shape
    hE, hx = 0.05, 1.0 / nx
    basis = _abi.m2m_smoothing_basis(nE, nx, hE, hx)
    g, Q = _expand(basis, nE, nx)
    P = _penalty_matrix(nE, nx, hE, hx)
    scale = max(np.abs(P).max(), 1.0)
    np.testing.assert_allclose(Q.T @ Q, np.eye(nE * nx), atol=1e-12)
    np.testing.assert_allclose(Q @ np.diag(g) @ Q.T, P, atol=1e-12 * scale)
    assert np.all(g >= 0)
    # the planes: three zero eigenvalues when both axes have 3+ cells
    if nE >= 2 and nx >= 2:
        assert np.sum(g < 1e-10 * g.max()) == 3


def test_spectral_filter_matches_the_oracle_dense_solve(oracle):
    """At a fixed lambda the smoother in the library's basis,
    Q diag(1/(1 + lambda g)) Q^T w0, equals the oracle's Cholesky solve."""
    from paper_1202_2355_amd import _abi
    from workloads import make_params, make_potential
    nE, nx = 12, 7
    par = make_params(make_potential(), n_E=nE, n_x=nx)
    hE, hx = (par["E_hi"] - par["E_lo"]) / nE, 1.0 / nx
    g, Q = _expand(_abi.m2m_smoothing_basis(nE, nx, hE, hx), nE, nx)
    w0 = np.random.default_rng(4).uniform(0.5, 1.5, nE * nx)
    for lam in (1e-9, 1e-6, 1e-3):
        ws = Q @ ((Q.T @ w0) / (1 + lam * g))
        wo = oracle.smooth_grid_at(par, w0, lam)
        np.testing.assert_allclose(ws, wo, rtol=1e-10)


def test_basis_arguments_are_checked():
    from paper_1202_2355_amd import _abi
    for args in ((0, 4, 0.1, 0.1), (129, 4, 0.1, 0.1), (64, 64, 0.1, 0.1), (4, 4, 0.0, 0.1),
                 (4, 4, 0.1, float("nan"))):
        with pytest.raises(_abi.M2MError) as e:
            _abi.m2m_smoothing_basis(*args)
        assert e.value.status == _abi.M2M_EINVAL
