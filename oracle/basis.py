"""1D bases on [0,1]: scaled Legendre polynomials and Alpert multiwavelets.

Paper: Sec. 2.1, nested partition (2.1), spaces V_n^k (2.2)-(2.3), wavelet
spaces W_n^k (2.4)-(2.5) and the orthonormal hierarchical basis (2.6).

Readings taken here (the paper leaves them open):

* (2.6) prints the dilation as ``2^l x - (2j+1)`` inside a level-n function;
  the exponent is read as ``n``.  With f_p living on [-1,1] the level-n,
  cell-j function is then supported on the level-(n-1) cell j, i.e.
  ``v_{p,n}^j(x) = 2^{(n-1)/2} psi_p(2^{n-1} x - j)`` with
  ``psi_p(t) = sqrt(2) f_p(2t - 1)`` on [0,1].
* W_n^k fixes its basis only up to an orthogonal rotation.  The basis is
  pinned by Alpert's extra vanishing moments: the (1-based) p-th function is
  orthogonal to all polynomials of degree <= k+p-1 on its support, which fixes
  it up to sign; the sign makes the highest-degree Legendre coefficient (that
  is not zero) of f_p on the right half (0,1) positive.

Level 0 (W_0 = V_0) uses ``phi_p(x) = sqrt(2p+1) P_p(2x-1)``, p = 0..k.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss01(n: int):
    """n-point Gauss-Legendre rule on [0,1] (nodes, weights)."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def legendre01(p: int, x):
    """Orthonormal Legendre polynomial of degree p on [0,1]: sqrt(2p+1) P_p(2x-1)."""
    c = np.zeros(p + 1)
    c[p] = 1.0
    return np.sqrt(2 * p + 1) * npleg.legval(2.0 * np.asarray(x, dtype=np.float64) - 1.0, c)


def dlegendre01(p: int, x):
    """d/dx of legendre01(p, x)."""
    c = np.zeros(p + 1)
    c[p] = 1.0
    dc = npleg.legder(c)
    return 2.0 * np.sqrt(2 * p + 1) * npleg.legval(2.0 * np.asarray(x, dtype=np.float64) - 1.0, dc)


@functools.lru_cache(maxsize=None)
def alpert(k: int):
    """Alpert multiwavelets psi_p on [0,1], p = 0..k (0-based; the paper's p-1).

    Returns ``(cL, cR)``, each (k+1, k+1): psi_p restricted to the left half
    [0,1/2) is ``sum_q cL[p,q] * sqrt(2) * phi_q(2t)`` and to the right half
    [1/2,1] is ``sum_q cR[p,q] * sqrt(2) * phi_q(2t-1)`` (phi_q = legendre01),
    i.e. coefficients in the orthonormal half-interval Legendre bases.

    Construction (Sec. 2.1, (2.4) and the Alpert basis cited under (2.6)):
    psi_p is the unit vector of the piecewise-P^k space on the two halves that
    is orthogonal to every polynomial of degree <= k+p (0-based p) on [0,1]
    and to psi_{p+1..k}.
    """
    nb = 2 * (k + 1)
    xg, wg = gauss01(3 * k + 4)
    # constraint rows: <psi, phi_i> over [0,1] for i = 0..2k, computed half by half
    C = np.zeros((2 * k + 1, nb))
    for i in range(2 * k + 1):
        for q in range(k + 1):
            # left half: t = u/2, dt = du/2 ; right half: t = (u+1)/2
            C[i, q] = np.sum(wg * 0.5 * np.sqrt(2.0) * legendre01(q, xg) * legendre01(i, 0.5 * xg))
            C[i, k + 1 + q] = np.sum(
                wg * 0.5 * np.sqrt(2.0) * legendre01(q, xg) * legendre01(i, 0.5 * (xg + 1.0))
            )
    found = {}
    for p in range(k, -1, -1):
        rows = [C[: k + p + 1]] + [found[q][None, :] for q in range(p + 1, k + 1)]
        S = np.concatenate(rows, axis=0)
        _, s, vt = np.linalg.svd(S)
        assert S.shape[0] == nb - 1 and s[-1] > 1e-8, "constraint rows must have full rank"
        f = vt[-1]
        f = f / np.linalg.norm(f)
        right = f[k + 1 :]
        top = [q for q in range(k + 1) if abs(right[q]) > 1e-10]
        if right[top[-1]] < 0:
            f = -f
        found[p] = f
    cL = np.array([found[p][: k + 1] for p in range(k + 1)])
    cR = np.array([found[p][k + 1 :] for p in range(k + 1)])
    return cL, cR


def _psi(k: int, p: int, t, deriv: bool):
    """psi_p(t) (or its derivative) on [0,1]; zero outside [0,1)."""
    cL, cR = alpert(k)
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    left = (t >= 0.0) & (t < 0.5)
    right = (t >= 0.5) & (t < 1.0)
    for q in range(k + 1):
        if deriv:
            out[left] += cL[p, q] * np.sqrt(2.0) * 2.0 * dlegendre01(q, 2.0 * t[left])
            out[right] += cR[p, q] * np.sqrt(2.0) * 2.0 * dlegendre01(q, 2.0 * t[right] - 1.0)
        else:
            out[left] += cL[p, q] * np.sqrt(2.0) * legendre01(q, 2.0 * t[left])
            out[right] += cR[p, q] * np.sqrt(2.0) * legendre01(q, 2.0 * t[right] - 1.0)
    return out


def hier(k: int, level: int, j: int, p: int, x, deriv: bool = False):
    """1D hierarchical basis function v_{p,level}^j at points x (eq. 2.6).

    Points must not sit on a breakpoint of the function (one-sided limits are
    never needed by the oracle: traces are taken on the full grid instead).
    Level 0 is defined on the periodic unit interval [0,1).
    """
    x = np.asarray(x, dtype=np.float64)
    if level == 0:
        inside = (x >= 0.0) & (x < 1.0)
        val = dlegendre01(p, x) if deriv else legendre01(p, x)
        return np.where(inside, val, 0.0)
    s = 2.0 ** (level - 1)
    t = s * x - j
    if deriv:
        return s ** 1.5 * _psi(k, p, t, True)
    return np.sqrt(s) * _psi(k, p, t, False)


def level_count(level: int) -> int:
    """Number of cells (translates j) at a 1D level: 1 for level 0, 2^(l-1) otherwise."""
    return 1 if level == 0 else 2 ** (level - 1)


def level_offset(level: int, k: int) -> int:
    """Index of the first level-`level` function in the 1D hierarchical ordering."""
    return 0 if level == 0 else (k + 1) * 2 ** (level - 1)


def hier_index_1d(level: int, j: int, p: int, k: int) -> int:
    """Position r = offset(level) + j(k+1) + p of (level, j, p) among levels 0..N."""
    return level_offset(level, k) + j * (k + 1) + p


def hier_list_1d(N: int, k: int):
    """All 1D hierarchical functions up to level N, in index order: list of (level, j, p)."""
    out = []
    for lev in range(N + 1):
        for j in range(level_count(lev)):
            for p in range(k + 1):
                out.append((lev, j, p))
    return out


def to_cell_legendre(N: int, k: int):
    """Dense orthogonal T: row r = coefficients of 1D hierarchical function r
    (levels 0..N) in the level-N cell-Legendre basis, column c*(k+1)+q for
    cell c and degree q.  Cell basis: 2^{N/2} phi_q(2^N x - c).

    Both families span V_N^k (eq. 2.5), so T is square and orthogonal; its
    entries are inner products computed cell by cell with an exact Gauss rule.
    """
    n = (k + 1) * 2 ** N
    h = 2.0 ** (-N)
    xg, wg = gauss01(k + 2)
    T = np.zeros((n, n))
    for r, (lev, j, p) in enumerate(hier_list_1d(N, k)):
        if lev == 0:
            cells = range(2 ** N)
        else:
            width = 2 ** (N - lev + 1)  # level-N cells under the level-(lev-1) support cell
            cells = range(j * width, (j + 1) * width)
        for c in cells:
            x = (c + xg) * h
            v = hier(k, lev, j, p, x)
            for q in range(k + 1):
                T[r, c * (k + 1) + q] = np.sum(wg * h * v * legendre01(q, xg) / np.sqrt(h))
    return T
