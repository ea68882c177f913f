"""Reaction term F(U) by quadrature at the Gauss points of the finest mesh.

Paper: Sec. 3, semi-discrete system (3.1) dU/dt = A U + F(U); Sec. 5 states
how F is evaluated: the numerical solution is reconstructed at the Gaussian
points of the finest-level mesh Omega_N and the integral int f(u_h) v dx is
done by the quadrature rule there.

    R : coefficients -> values of u_h at every Gauss point of Omega_N
    P : point values g -> coefficients  sum_q W_q g_q v_a(x_q)   (P = R^T diag(W))
    F(U) = P f(R U)

Reading (the paper does not give the number of points): nq = k+1
Gauss-Legendre points per dimension in each finest cell, so P R = I on the
sparse space (integrands of degree 2k are exact).

Both transforms are written as the literal sums over level blocks: a block l
contributes the tensor product of its 1D basis functions, contracted one axis
at a time (numpy tensordot), which is the definition u_h(x) = sum_a U_a v_a(x).

Reaction polynomials: f_s(u0, u1) = sum_{a,b} c[s, a, b] u0^a u1^b, c of shape
(species, 4, 4) covering every reaction used (degree <= 3).
"""
from __future__ import annotations

import numpy as np

from .basis import gauss01, hier, hier_list_1d, level_count, level_offset
from .sparsegrid import block_offsets


class Quadrature:
    """Gauss points of Omega_N and the 1D basis table V1[r, q] = v_r(x_q)."""

    def __init__(self, d: int, N: int, k: int, nq: int | None = None):
        self.d, self.N, self.k = d, N, k
        self.nq = k + 1 if nq is None else nq
        h = 2.0 ** (-N)
        xg, wg = gauss01(self.nq)
        self.x1 = ((np.arange(2 ** N)[:, None] + xg[None, :]) * h).ravel()
        self.w1 = np.tile(wg * h, 2 ** N)
        self.V1 = np.array([hier(k, lev, j, p, self.x1) for (lev, j, p) in hier_list_1d(N, k)])
        self.blocks, self.starts, self.sizes = block_offsets(d, N, k)
        self.npts1 = self.x1.shape[0]

    def _rows(self, lev):
        o = level_offset(lev, self.k)
        return slice(o, o + level_count(lev) * (self.k + 1))

    def R(self, U):
        """Point values of u_h, array of shape (npts1,)*d."""
        U = np.asarray(U, dtype=np.float64)
        out = np.zeros((self.npts1,) * self.d)
        for l, s, n in zip(self.blocks, self.starts, self.sizes):
            ext = [level_count(lm) * (self.k + 1) for lm in l]
            T = U[s : s + n].reshape(ext)
            for lm in l:
                T = np.tensordot(T, self.V1[self._rows(lm)], axes=([0], [0]))
            out += T
        return out

    def weights(self):
        W = self.w1
        for _ in range(self.d - 1):
            W = np.multiply.outer(W, self.w1)
        return W

    def P(self, g):
        """Coefficients sum_q W_q g_q v_a(x_q), canonical order."""
        gw = np.asarray(g, dtype=np.float64) * self.weights()
        out = np.zeros(int(self.sizes.sum()))
        for l, s, n in zip(self.blocks, self.starts, self.sizes):
            T = gw
            for lm in l:
                T = np.tensordot(T, self.V1[self._rows(lm)], axes=([0], [1]))
            out[s : s + n] = T.ravel()
        return out


def f_eval(c, u):
    """f_s(u0, u1) for every species s; u is a list of point-value arrays."""
    c = np.asarray(c, dtype=np.float64)
    u0 = u[0]
    u1 = u[1] if len(u) > 1 else np.zeros_like(u0)
    out = []
    for s in range(len(u)):
        acc = np.zeros_like(u0)
        for a in range(4):
            for b in range(4):
                if c[s, a, b] != 0.0:
                    acc = acc + c[s, a, b] * u0 ** a * u1 ** b
        out.append(acc)
    return out


def f_jac(c, u):
    """J[s][t] = d f_s / d u_t at every point."""
    c = np.asarray(c, dtype=np.float64)
    u0 = u[0]
    u1 = u[1] if len(u) > 1 else np.zeros_like(u0)
    S = len(u)
    J = [[np.zeros_like(u0) for _ in range(S)] for _ in range(S)]
    for s in range(S):
        for a in range(4):
            for b in range(4):
                cc = c[s, a, b]
                if cc == 0.0:
                    continue
                if a > 0:
                    J[s][0] = J[s][0] + cc * a * u0 ** (a - 1) * u1 ** b
                if b > 0 and S > 1:
                    J[s][1] = J[s][1] + cc * b * u0 ** a * u1 ** (b - 1)
    return J


def F(quad: Quadrature, c, U):
    """F(U) = P f(R U) per species; U has shape (species, ndof)."""
    uq = [quad.R(U[s]) for s in range(U.shape[0])]
    fq = f_eval(c, uq)
    return np.array([quad.P(fq[s]) for s in range(U.shape[0])])
