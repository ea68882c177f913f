"""Pins for the oracle's 1D basis (Sec. 2.1, eqs. 2.1-2.6).

The checks use their own quadrature (fine Gauss rules on sub-cells), not the
construction's matrices, so a wrong sign, index or scale in oracle/basis.py
fails one of them.
"""
import numpy as np
import pytest

from oracle import basis


def _halves(npts=40):
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    xs = np.concatenate([0.5 * x, 0.5 + 0.5 * x])
    ws = np.concatenate([0.5 * w, 0.5 * w])
    return xs, ws


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_alpert_orthonormal_vanishing_moments_sign(k):
    xs, ws = _halves()
    psi = np.array([basis._psi(k, p, xs, False) for p in range(k + 1)])
    gram = (psi * ws) @ psi.T
    assert np.abs(gram - np.eye(k + 1)).max() < 1e-13
    # 0-based p: orthogonal to every polynomial of degree <= k + p on [0,1]
    for p in range(k + 1):
        for deg in range(k + p + 1):
            mom = np.sum(ws * psi[p] * (xs - 0.5) ** deg)
            assert abs(mom) < 1e-13, (p, deg, mom)
        # and not orthogonal to degree k+p+1 (the extra moment is where it stops)
        assert abs(np.sum(ws * psi[p] * (xs - 0.5) ** (k + p + 1))) > 1e-6
    # sign rule: top nonzero Legendre coefficient on the right half is positive
    xr = xs[xs >= 0.5]
    wr = ws[xs >= 0.5]
    for p in range(k + 1):
        pr = psi[p][xs >= 0.5]
        coef = [np.sum(wr * pr * basis.legendre01(q, 2 * xr - 1) * np.sqrt(2)) for q in range(k + 1)]
        top = [c for c in coef if abs(c) > 1e-10][-1]
        assert top > 0


def test_k0_is_haar():
    xs, _ = _halves(4)
    psi = basis._psi(0, 0, xs, False)
    assert np.allclose(psi[xs < 0.5], -1.0) and np.allclose(psi[xs >= 0.5], 1.0)


@pytest.mark.parametrize("N,k", [(4, 1), (3, 2), (3, 3)])
def test_hierarchical_basis_orthonormal(N, k):
    # independent fine rule on level-(N+1) cells
    x, w = np.polynomial.legendre.leggauss(k + 3)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    h = 2.0 ** (-(N + 1))
    xs = ((np.arange(2 ** (N + 1))[:, None] + x[None, :]) * h).ravel()
    ws = np.tile(w * h, 2 ** (N + 1))
    funcs = basis.hier_list_1d(N, k)
    V = np.array([basis.hier(k, lev, j, p, xs) for (lev, j, p) in funcs])
    G = (V * ws) @ V.T
    assert np.abs(G - np.eye(len(funcs))).max() < 1e-12
    # level-l function j is supported on the level-(l-1) cell j  (reading of eq. 2.6)
    for r, (lev, j, p) in enumerate(funcs):
        if lev >= 1:
            a, b = j * 2.0 ** (1 - lev), (j + 1) * 2.0 ** (1 - lev)
            outside = (xs < a) | (xs > b)
            assert np.all(V[r, outside] == 0.0)


@pytest.mark.parametrize("N,k", [(3, 1), (4, 2)])
def test_transform_is_orthogonal(N, k):
    T = basis.to_cell_legendre(N, k)
    assert np.abs(T @ T.T - np.eye(T.shape[0])).max() < 1e-12


def test_level_layout():
    k = 2
    assert [basis.level_offset(l, k) for l in range(5)] == [0, 3, 6, 12, 24]
    assert basis.hier_index_1d(3, 1, 2, k) == 12 + 1 * 3 + 2
    assert len(basis.hier_list_1d(4, k)) == (k + 1) * 2 ** 4
