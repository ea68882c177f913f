"""L2 projection of initial data onto the sparse-grid space, and L2 errors.

Paper: Sec. 2.2, Theorem 2.4 takes u_h(0) = P u, the L2 projection onto
V_N^k.  The paper does not say how it measures the L2 error.

Readings:
* Initial data are sums of separable terms amp * prod_m g_m(x_m).  For an
  orthonormal tensor basis the projection coefficient of a separable term is
  the product of 1D projection coefficients, each computed cell by cell on
  Omega_N with a 16-point Gauss rule (exact to rounding for the trigonometric
  and dyadic-box factors used here).
* L2 error, exact for an orthonormal basis (Parseval):
  ||u - u_h||^2 = ||u||^2 - ||P u||^2 + ||P u - U||^2, with ||u|| analytic.

1D factor descriptors (shared format with the input generator):
  ("cos", f, phi)  -> cos(2 pi f x + phi)
  ("box", a, b)    -> indicator of [a, b)
"""
from __future__ import annotations

import numpy as np

from .basis import gauss01, hier, hier_list_1d
from .sparsegrid import enumerate_dofs


def factor_fn(desc):
    kind = desc[0]
    if kind == "cos":
        f, phi = float(desc[1]), float(desc[2])
        return lambda x: np.cos(2.0 * np.pi * f * x + phi)
    if kind == "box":
        a, b = float(desc[1]), float(desc[2])
        return lambda x: ((x >= a) & (x < b)).astype(np.float64)
    raise ValueError(f"unknown factor {desc!r}")


def project_1d(N: int, k: int, desc, nq: int = 16):
    """c[r] = int_0^1 g(x) v_r(x) dx for every 1D hierarchical function r (levels 0..N)."""
    g = factor_fn(desc)
    h = 2.0 ** (-N)
    xg, wg = gauss01(nq)
    x = ((np.arange(2 ** N)[:, None] + xg[None, :]) * h).ravel()
    w = np.tile(wg * h, 2 ** N)
    gx = g(x) * w
    out = np.zeros((k + 1) * 2 ** N)
    for r, (lev, j, p) in enumerate(hier_list_1d(N, k)):
        out[r] = np.dot(gx, hier(k, lev, j, p, x))
    return out


def project_separable(d: int, N: int, k: int, amp: float, factors):
    """Coefficients (canonical order) of amp * prod_m g_m(x_m)."""
    _, _, _, r1d = enumerate_dofs(d, N, k)
    out = np.full(r1d.shape[0], float(amp))
    for m in range(d):
        out *= project_1d(N, k, factors[m])[r1d[:, m]]
    return out


def project_terms(d: int, N: int, k: int, terms):
    """Sum of separable terms [(amp, [factor_0, ..., factor_{d-1}]), ...]."""
    out = np.zeros(enumerate_dofs(d, N, k)[3].shape[0])
    for amp, factors in terms:
        out += project_separable(d, N, k, amp, factors)
    return out


def l2_error(U, PU, unorm2: float) -> float:
    """||u - u_h|| from the coefficients U of u_h, P u and ||u||^2 (Parseval)."""
    U = np.asarray(U, dtype=np.float64)
    PU = np.asarray(PU, dtype=np.float64)
    e2 = unorm2 - float(PU @ PU) + float((PU - U) @ (PU - U))
    return float(np.sqrt(max(e2, 0.0)))
