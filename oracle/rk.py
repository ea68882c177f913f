"""Explicit Runge-Kutta comparators and their stability limits (Sec. 4, Table 1).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper uses explicit second- and third-order Runge-Kutta methods (RK2,
RK3) to show the step-size limit the stiff diffusion operator imposes, and
reports it as CFL = k d dt / h_N^2 (k the diffusion coefficient, d the
dimension).  It does not say which RK2/RK3.  Reading: the strong-stability-
preserving forms of Shu and Osher,

    RK2:  U1 = U + dt L(U);  U^{n+1} = 1/2 U + 1/2 (U1 + dt L(U1)),
    RK3:  U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));
          U^{n+1} = 1/3 U + 2/3 (U2 + dt L(U2)),

with L(U) = A U + F(U).  For a linear problem every s-stage method of order
s (s = 2, 3) has the stability function R(z) = sum_{j<=s} z^j / j!, so the
limit on a symmetric negative semi-definite A is dt <= z_s / |lambda_0(A)|
with z_s the length of the stability interval on the negative real axis
(z_2 = 2, z_3 = 2.5127...), whichever RK2/RK3 the paper used.
"""
from __future__ import annotations

import math

import numpy as np


def rk_step(prob, U, dt, order):
    """One SSP-RK step of order 2 or 3 for dU/dt = A U + F(U) (prob: iif.Problem)."""

    def L(V):
        return np.array([prob.A[s] @ V[s] for s in range(prob.S)]) + prob.F(V)

    U = np.asarray(U, dtype=np.float64)
    U1 = U + dt * L(U)
    if order == 2:
        return 0.5 * U + 0.5 * (U1 + dt * L(U1))
    if order == 3:
        U2 = 0.75 * U + 0.25 * (U1 + dt * L(U1))
        return U / 3.0 + (2.0 / 3.0) * (U2 + dt * L(U2))
    raise ValueError("order must be 2 or 3")


def stability_function(order, z):
    """R(z) = sum_{j=0}^{order} z^j / j! (any explicit RK with s = order stages)."""
    return sum(z ** j / math.factorial(j) for j in range(order + 1))


def real_stability_limit(order):
    """Largest z_s with |R(-x)| <= 1 for all x in [0, z_s], by bisection on the
    first crossing of |R| = 1 past the origin."""
    lo, hi = 1e-6, 10.0
    # bracket: scan for the first x where |R(-x)| > 1
    xs = np.linspace(lo, hi, 100001)
    bad = np.nonzero(np.abs(stability_function(order, -xs)) > 1.0)[0]
    hi = xs[bad[0]]
    lo = xs[bad[0] - 1]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if abs(stability_function(order, -mid)) > 1.0:
            hi = mid
        else:
            lo = mid
    return lo


def cfl_limit(lambda0, d, N, order, kcoef=1.0):
    """Largest stable CFL = k d dt / h_N^2 for an operator with extreme eigenvalue lambda0."""
    dt = real_stability_limit(order) / abs(lambda0)
    return kcoef * d * dt / (2.0 ** -N) ** 2
