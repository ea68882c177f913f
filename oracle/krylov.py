"""Krylov approximation of exp(h A) v.

Paper: Sec. 3, Krylov space (3.7), Arnoldi process producing V_M and the
upper Hessenberg H_M, and the approximation (3.8)
    exp(h A) v  ~  gamma V_M exp(h H_M) e_1,   gamma = ||v||_2,
with exp(h H_M) by Pade approximation with scaling and squaring.

Readings:
* Arnoldi is run with modified Gram-Schmidt (the reference the paper cites
  for Arnoldi states it that way) for exactly M steps, i.e. M products A v_j;
  h_{M+1,M} is kept only as an a-posteriori estimate.
* Happy breakdown: if h_{j+1,j} <= 1e-12 * ||A||_inf the process stops with
  m = j (the Krylov space is invariant; the result is then exact).
* M larger than the number of unknowns is clamped to it; v = 0 gives 0.
* For systems the species are independent blocks of A, so one Arnoldi is run
  per species (exp of a block-diagonal matrix is block-diagonal).

exp(h H) uses scipy.linalg.expm (Pade with scaling and squaring, the
Al-Mohy/Higham form of the algorithm the paper cites); expm_eigh is the
independent cross-check through the symmetric eigendecomposition.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

BREAKDOWN_REL = 1e-12


def arnoldi_mgs(apply, v, M: int, anorm: float):
    """Arnoldi with modified Gram-Schmidt.

    Returns (V, H, m, beta): V is n x (m+1) (last column unused after a
    breakdown), H is (m+1) x m, m the dimension reached, beta = ||v||.
    """
    v = np.asarray(v, dtype=np.float64)
    n = v.shape[0]
    M = min(M, n)
    beta = float(np.linalg.norm(v))
    V = np.zeros((n, M + 1))
    H = np.zeros((M + 1, M))
    if beta == 0.0:
        return V[:, :1], H[:1, :0], 0, beta
    V[:, 0] = v / beta
    m = M
    for j in range(M):
        w = apply(V[:, j])
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= BREAKDOWN_REL * anorm:
            m = j + 1
            break
        V[:, j + 1] = w / H[j + 1, j]
    return V[:, : m + 1], H[: m + 1, :m], m, beta


def expv(A, h: float, v, M: int, anorm: float | None = None, expm=None):
    """gamma V_m exp(h H_m) e_1 (eq. 3.8).  Returns (w, info)."""
    if anorm is None:
        anorm = float(np.abs(A).sum(axis=1).max())
    V, H, m, beta = arnoldi_mgs(lambda x: A @ x, v, M, anorm)
    if m == 0:
        return np.zeros_like(np.asarray(v, dtype=np.float64)), {"m": 0, "h_next": 0.0, "H": H}
    E = (expm or sla.expm)(h * H[:m, :m])
    w = beta * (V[:, :m] @ E[:, 0])
    return w, {"m": m, "h_next": float(H[m, m - 1]), "H": H}


def expm_eigh(X):
    """exp(X) for (numerically) symmetric X via eigh of its symmetric part."""
    S = 0.5 * (X + X.T)
    lam, Q = np.linalg.eigh(S)
    return (Q * np.exp(lam)) @ Q.T


def dense_expv(A, h: float, v):
    """exp(h A) v with a dense exponential (tiny grids only)."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    return sla.expm(h * Ad) @ np.asarray(v, dtype=np.float64)
