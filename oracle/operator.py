"""The sparse-grid interior-penalty diffusion operator A = -B, assembled explicitly.

Paper: Sec. 2.1, semi-discrete scheme (2.10) with the symmetric interior
penalty bilinear form B, jump/average definitions (2.11), penalty sigma = 20,
Gamma = all cell faces of the finest uniform mesh Omega_N; Sec. 4 intro (the
"unidirectional principle": d-dimensional integrals are products of 1D ones).

Route (independent of the library): the 1D full-grid SIPG matrix is assembled
on the 2^N cells of Omega_N in the orthonormal cell-Legendre basis, moved to the
hierarchical basis with the explicit orthogonal transform T of basis.py, and
the d-dimensional A is formed entry by entry from its definition

    A[a, b] = - sum_i D * Bh_i[r_i(a), r_i(b)] * prod_{m != i} delta(r_m(a), r_m(b)),

a and b ranging over the sparse index set only.  Off-axis factors are the
identity because the basis is orthonormal (the 1D mass matrix is I).

Readings:
* h in sigma/h is the finest mesh size h_N = 2^-N on every face (Gamma is the
  set of faces of Omega_N, and the energy norm of Sec. 2.2 uses h_N).
* [q] = q^- - q^+ with '-' the cell to the left of the face; {q} the mean.
* Periodic boundary: the face at x = 0 joins the last and the first cell.
* A diagonal diffusion tensor k_ii(x_i) enters the i-th 1D form: volume
  weight k_ii(x) integrated by a Gauss rule (default 12 points per cell) and
  face weight k_ii(x_face).  Off-diagonal k_ij is out of scope.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import dlegendre01, gauss01, legendre01, to_cell_legendre
from .sparsegrid import enumerate_dofs


def full_grid_sipg(N: int, k: int, sigma: float = 20.0, kappa=None, nquad: int = 12, bc: str = "periodic"):
    """1D SIPG matrix B_full[v, u] = B(u, v) on 2^N cells, cell-Legendre basis.

    Cell c basis: h^{-1/2} phi_q((x - c h)/h), h = 2^-N.
    bc = "periodic": the face at x = 0 joins the last and the first cell.
    bc = "dirichlet" (zero boundary values): on a boundary face the jump is
    the one-sided trace times the outward normal and the average of the
    flux is its one-sided value (the convention stated after eq. 2.11), so the
    face at x = 0 acts on cell 0 with [u] = -u(0+), {u'} = u'(0+), and the face
    at x = 1 on the last cell with [u] = u(1-), {u'} = u'(1-).
    """
    nc = 2 ** N
    h = 2.0 ** (-N)
    n = nc * (k + 1)
    B = np.zeros((n, n))
    xg, wg = gauss01(nquad)
    kap = (lambda x: np.ones_like(x)) if kappa is None else kappa
    # volume: int_cell kappa u' v'
    dphi = np.array([dlegendre01(q, xg) for q in range(k + 1)])  # on reference cell
    for c in range(nc):
        kv = kap((c + xg) * h)
        loc = (dphi * (wg * kv)) @ dphi.T / h ** 2  # h^{-3/2}*h^{-3/2}*h
        s = slice(c * (k + 1), (c + 1) * (k + 1))
        B[s, s] += loc
    # traces on the reference cell
    v0 = np.array([legendre01(q, 0.0) for q in range(k + 1)])
    v1 = np.array([legendre01(q, 1.0) for q in range(k + 1)])
    d0 = np.array([dlegendre01(q, 0.0) for q in range(k + 1)])
    d1 = np.array([dlegendre01(q, 1.0) for q in range(k + 1)])
    if bc == "dirichlet":
        for xe, c, jump, der in ((0.0, 0, -v0 / np.sqrt(h), d0 / h ** 1.5), (1.0, nc - 1, v1 / np.sqrt(h), d1 / h ** 1.5)):
            ke = float(kap(np.array([xe]))[0])
            loc = -ke * np.outer(jump, der) - ke * np.outer(der, jump) + (sigma / h) * np.outer(jump, jump)
            s = slice(c * (k + 1), (c + 1) * (k + 1))
            B[s, s] += loc
    elif bc != "periodic":
        raise ValueError(bc)
    for e in range(1 if bc == "dirichlet" else 0, nc):
        L, R = (e - 1) % nc, e
        xe = e * h
        ke = float(kap(np.array([xe]))[0])
        # for each local function f in {L_q, R_q}: jump [f] = f^- - f^+, mean of derivative
        jump = np.concatenate([v1, -v0]) / np.sqrt(h)
        mder = 0.5 * np.concatenate([d1, d0]) / h ** 1.5
        loc = (
            -ke * np.outer(jump, mder)  # row = test v: -{k u'}[v]
            - ke * np.outer(mder, jump)  # -{k v'}[u]
            + (sigma / h) * np.outer(jump, jump)
        )
        idx = np.concatenate([np.arange(L * (k + 1), (L + 1) * (k + 1)), np.arange(R * (k + 1), (R + 1) * (k + 1))])
        # unbuffered accumulation: with one cell (N = 0) the periodic face joins the cell to itself
        np.add.at(B, (idx[:, None], idx[None, :]), loc)
    return B


def hier_operator_1d(N: int, k: int, sigma: float = 20.0, kappa=None, drop_rel: float = 1e-13, bc: str = "periodic"):
    """1D operator in the hierarchical basis (levels 0..N): Bh = T B_full T^T.

    Entries below drop_rel * max|Bh| are rounding noise of exact zeros (a
    function's vanishing moments cancel every term unless the other function
    jumps on its support) and are set to zero.
    """
    T = to_cell_legendre(N, k)
    Bh = T @ full_grid_sipg(N, k, sigma, kappa, bc=bc) @ T.T
    Bh[np.abs(Bh) < drop_rel * np.abs(Bh).max()] = 0.0
    return Bh


def assemble_A(d: int, N: int, k: int, sigma: float = 20.0, kappas=None, D: float = 1.0, bc: str = "periodic"):
    """Explicit sparse A (scipy CSR, canonical DOF order) for one species.

    kappas: None (k_ii = 1) or a list of d callables k_ii(x); bc: "periodic" or
    "dirichlet" (zero boundary values on every face of the cube).
    """
    _, _, _, r1d = enumerate_dofs(d, N, k)
    n1 = (k + 1) * 2 ** N
    ndof = r1d.shape[0]
    weights = n1 ** np.arange(d - 1, -1, -1, dtype=np.int64)
    keys = r1d @ weights
    order = np.argsort(keys)
    skeys = keys[order]
    rows, cols, vals = [], [], []
    cache = {}
    for i in range(d):
        kap = None if kappas is None else kappas[i]
        ck = id(kap) if kap is not None else None
        if ck not in cache:
            cache[ck] = hier_operator_1d(N, k, sigma, kap, bc=bc)
        Bh = cache[ck]
        ri = r1d[:, i]
        for r in np.unique(ri):
            a_idx = np.nonzero(ri == r)[0]
            nzc = np.nonzero(Bh[r])[0]
            for c in nzc:
                target = keys[a_idx] + (c - r) * weights[i]
                pos = np.searchsorted(skeys, target)
                pos = np.minimum(pos, ndof - 1)
                ok = skeys[pos] == target
                rows.append(a_idx[ok])
                cols.append(order[pos[ok]])
                vals.append(np.full(int(ok.sum()), -D * Bh[r, c]))
    A = sp.csr_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(ndof, ndof)
    )
    A.sum_duplicates()
    return A


def inf_norm(A) -> float:
    """max_i sum_j |A_ij| (used only for the Krylov breakdown threshold)."""
    return float(np.abs(A).sum(axis=1).max())
