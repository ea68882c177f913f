"""IIF2 and IIF3 time stepping with the implicit reaction stage.

Paper: Sec. 3, integrating-factor form (3.2), the r-th order family (3.3)
with Lagrange coefficients (3.4), and IIF2 (3.5):

    U^{n+1} = exp(A dt) (U^n + dt/2 F(U^n)) + dt/2 F(U^{n+1}).

The implicit stage solves  G(U) = U - dt/2 F(U) - W = 0,  W = exp(A dt)(...),
a system of the size of the unknowns (Sec. 5: the sparse basis is global, so
the "local implicit property" is lost and Newton iterations are needed).

Readings:
* The stage is solved by a pointwise quasi-Newton iteration with the same
  root as Newton on G:
      U <- U - P[(I_s - dt/2 J_f(u_q))^{-1} (R G)_q],
  with a species-by-species Jacobian inverse at every quadrature point q.
  `implicit_stage_newton_dense` is the exact-Jacobian Newton on tiny grids
  that pins the root.
* Initial guess U^0 = W + dt/2 F(U^n); stop when ||G||_2 <= tol * max(1, ||W||_2)
  (tol = 1e-13 unless given), at most 50 corrections.
* F(U^{n+1}) of the accepted iterate is reused as F(U^n) of the next step
  (same input, same value).
* One Krylov exponential per species (the diffusion operator of a system is
  block diagonal, species s scaled by D_s).
* A forcing term of (1.1) (Examples 2 and 3) enters F as its L2 projection
  S(t) evaluated at the time level of each F (F^{n+1} = P f(R U^{n+1}) +
  S(t^{n+1}) in the stage).
* Local implicit stage (variant, not the paper's scheme): the stage solved
  pointwise at the Gauss points, u - c f(u) = R W, then U = P u; Newton per
  point from u = w, stop at |g| <= 1e-15 max(1, |w|) or 30 corrections.
* IIF3 (3.6): terms under one exponential share a Krylov evaluation, the
  stage coefficient is alpha_1 dt = 5 dt / 12 with initial guess
  W + alpha_1 dt F(U^n), and the first step is one IIF2 step (start-up).
"""
from __future__ import annotations

import numpy as np

from . import krylov, reaction
from .operator import assemble_A, inf_norm

TOL_DEFAULT = 1e-13
MAX_ITER_DEFAULT = 50


def iif_alpha(r: int):
    """Lagrange coefficients of (3.4): alpha_i for i = -1 .. r-2 (returns a dict).

    alpha_{-i} = (1/dt) int_0^dt prod_{k=-1..r-2, k != i} (tau + k dt)/((k - i) dt) dtau,
    evaluated with dt = 1 by exact polynomial integration.
    """
    from numpy.polynomial import polynomial as P

    out = {}
    for i in range(-1, r - 1):
        poly = np.array([1.0])
        for kk in range(-1, r - 1):
            if kk == i:
                continue
            poly = P.polymul(poly, np.array([kk, 1.0]) / (kk - i))
        integ = P.polyint(poly)
        out[i] = float(P.polyval(1.0, integ) - P.polyval(0.0, integ))
    return out


class Problem:
    """One instance: operator, quadrature, reaction and step parameters."""

    def __init__(self, d, N, k, D, rx, dt, M, sigma=20.0, kappas=None, nq=None, bc="periodic"):
        self.d, self.N, self.k = d, N, k
        self.D = list(D)
        self.S = len(self.D)
        self.rx = np.asarray(rx, dtype=np.float64)
        self.dt, self.M = float(dt), int(M)
        self.bc = bc
        A1 = assemble_A(d, N, k, sigma, kappas, 1.0, bc)
        self.A = [Ds * A1 for Ds in self.D]
        self.anorm = [inf_norm(a) for a in self.A]
        self.quad = reaction.Quadrature(d, N, k, nq)
        self.ndof = A1.shape[0]

    def F(self, U):
        return reaction.F(self.quad, self.rx, U)


def implicit_stage(prob: Problem, W, Fn, tol=TOL_DEFAULT, max_iter=MAX_ITER_DEFAULT, coef=None, S=None):
    """Pointwise quasi-Newton solve of U - c (F(U) + S) = W, c = coef (default
    dt/2, the IIF2 stage; IIF3 uses c = alpha_1 dt = 5 dt / 12), S a source
    vector at the new time level (projection of a forcing term, or None).
    Initial guess W + c F^n, F^n the full right-hand side of the old level.

    Returns (U, F(U) + S, info) with info = {iters, residual, converged}.
    """
    dt2 = 0.5 * prob.dt if coef is None else float(coef)
    if S is not None:
        U, FU, info = implicit_stage(prob, W + dt2 * np.asarray(S), Fn, tol, max_iter, coef=dt2)
        return U, FU + S, info
    S = prob.S
    U = W + dt2 * Fn
    wnorm = float(np.linalg.norm(W))
    it = 0
    while True:
        uq = [prob.quad.R(U[s]) for s in range(S)]
        fq = reaction.f_eval(prob.rx, uq)
        FU = np.array([prob.quad.P(fq[s]) for s in range(S)])
        G = U - dt2 * FU - W
        res = float(np.linalg.norm(G))
        if res <= tol * max(1.0, wnorm):
            return U, FU, {"iters": it, "residual": res, "converged": True}
        if it == max_iter:
            return U, FU, {"iters": it, "residual": res, "converged": False}
        Gq = [prob.quad.R(G[s]) for s in range(S)]
        J = reaction.f_jac(prob.rx, uq)
        if S == 1:
            dq = [Gq[0] / (1.0 - dt2 * J[0][0])]
        else:
            a, b = 1.0 - dt2 * J[0][0], -dt2 * J[0][1]
            c, d = -dt2 * J[1][0], 1.0 - dt2 * J[1][1]
            det = a * d - b * c
            dq = [(d * Gq[0] - b * Gq[1]) / det, (a * Gq[1] - c * Gq[0]) / det]
        U = U - np.array([prob.quad.P(dq[s]) for s in range(S)])
        it += 1


LOCAL_TOL = 1e-15
LOCAL_MAX_ITER = 30


def solve_pointwise(rx, wq, coef, tol=LOCAL_TOL, max_iter=LOCAL_MAX_ITER):
    """Solve u - c f(u) = w independently at every point (s x s Newton, s <= 2),
    from u = w, until |u - c f(u) - w| <= tol * max(1, |w|) at the point (max
    norm over species) or max_iter corrections.  wq: list over species of
    point arrays.  Returns the list of solutions."""
    S = len(wq)
    u = [np.array(w, dtype=np.float64) for w in wq]
    wmag = np.maximum(1.0, np.max(np.abs(np.array(wq)), axis=0))
    active = np.ones(u[0].shape, dtype=bool)
    for it in range(max_iter + 1):
        f = reaction.f_eval(rx, u)
        g = [u[s] - coef * f[s] - wq[s] for s in range(S)]
        gmax = np.max(np.abs(np.array(g)), axis=0)
        active &= ~(gmax <= tol * wmag)
        if not active.any() or it == max_iter:
            break
        J = reaction.f_jac(rx, u)
        if S == 1:
            du = [g[0] / (1.0 - coef * J[0][0])]
        else:
            a, b = 1.0 - coef * J[0][0], -coef * J[0][1]
            c, d = -coef * J[1][0], 1.0 - coef * J[1][1]
            det = a * d - b * c
            du = [(d * g[0] - b * g[1]) / det, (a * g[1] - c * g[0]) / det]
        for s in range(S):
            u[s] = np.where(active, u[s] - du[s], u[s])
    return u


def implicit_stage_local(prob: Problem, W, coef=None, S=None):
    """Local implicit stage (the "local implicit property" of IIF schemes that
    Sec. 5 names as future work for the sparse-grid method): instead of the
    Galerkin root of U - c P f(R U) = W, solve the reaction problem
    u - c f(u) = R W independently at every Gauss point of Omega_N and project,
    U = P u.  A different scheme (collocation of the stage): equal to the
    Galerkin stage for linear f, close to it (at quadrature-error level) for
    nonlinear f.  Returns (U, F(U) + S)."""
    c = 0.5 * prob.dt if coef is None else float(coef)
    W = np.asarray(W, dtype=np.float64)
    if S is not None:
        W = W + c * np.asarray(S)
    wq = [prob.quad.R(W[s]) for s in range(prob.S)]
    uq = solve_pointwise(prob.rx, wq, c)
    U = np.array([prob.quad.P(uq[s]) for s in range(prob.S)])
    F = prob.F(U) + (S if S is not None else 0.0)
    return U, F


def iif2_step_local(prob: Problem, U, Fn, dense=False, S_next=None):
    """IIF2 (3.5) with the local implicit stage.  Returns (U^{n+1}, F^{n+1}, info)."""
    v = U + 0.5 * prob.dt * Fn
    W, kinfo = expv_species(prob, v, dense)
    U1, F1 = implicit_stage_local(prob, W, 0.5 * prob.dt, S_next)
    return U1, F1, {"krylov": kinfo}


def iif2_run_local(prob: Problem, U0, steps: int, dense=False, source=None):
    """`steps` IIF2 steps with the local implicit stage.  Returns (U, F(U), infos)."""
    U = np.array(U0, dtype=np.float64).reshape(prob.S, prob.ndof)
    Fn = prob.F(U) + (source(0.0) if source else 0.0)
    infos = []
    for n in range(steps):
        Sn = source((n + 1) * prob.dt) if source else None
        U, Fn, info = iif2_step_local(prob, U, Fn, dense, S_next=Sn)
        infos.append(info)
    return U, Fn, infos


def implicit_stage_newton_dense(prob: Problem, W, Fn, tol=1e-14, max_iter=30):
    """Exact-Jacobian Newton on G(U) = U - dt/2 P f(R U) - W (tiny grids only).

    J_G = I - dt/2 P diag(J_f) R, with R and P formed as explicit matrices.
    """
    S, n = prob.S, prob.ndof
    dt2 = 0.5 * prob.dt
    Rm = np.stack([prob.quad.R(e).ravel() for e in np.eye(n)], axis=1)  # npts x n
    Wq = prob.quad.weights().ravel()
    Pm = (Rm * Wq[:, None]).T  # n x npts
    U = W + dt2 * Fn
    for _ in range(max_iter):
        uq = [Rm @ U[s] for s in range(S)]
        fq = reaction.f_eval(prob.rx, uq)
        G = U - dt2 * np.array([Pm @ fq[s] for s in range(S)]) - W
        if np.linalg.norm(G) <= tol * max(1.0, np.linalg.norm(W)):
            break
        J = reaction.f_jac(prob.rx, uq)
        JG = np.eye(S * n)
        for s in range(S):
            for t in range(S):
                JG[s * n : (s + 1) * n, t * n : (t + 1) * n] -= dt2 * (Pm * J[s][t][None, :]) @ Rm
        U = U - np.linalg.solve(JG, G.ravel()).reshape(S, n)
    return U


def expv_species(prob: Problem, v, dense: bool = False, h=None):
    """exp(A_s h) v_s for every species (Krylov with M, or dense); h = dt by default."""
    h = prob.dt if h is None else float(h)
    out, infos = [], []
    for s in range(prob.S):
        if dense:
            out.append(krylov.dense_expv(prob.A[s], h, v[s]))
            infos.append({"m": -1})
        else:
            w, info = krylov.expv(prob.A[s], h, v[s], prob.M, prob.anorm[s])
            out.append(w)
            infos.append(info)
    return np.array(out), infos


def iif2_step(prob: Problem, U, Fn, dense=False, tol=TOL_DEFAULT, max_iter=MAX_ITER_DEFAULT, S_next=None):
    """One IIF2 step (3.5).  Fn: the right-hand side at the old level (reaction
    plus source); S_next: source vector at the new level or None.
    Returns (U^{n+1}, F(U^{n+1}) + S_next, info)."""
    v = U + 0.5 * prob.dt * Fn
    W, kinfo = expv_species(prob, v, dense)
    U1, F1, ninfo = implicit_stage(prob, W, Fn, tol, max_iter, S=S_next)
    ninfo["krylov"] = kinfo
    return U1, F1, ninfo


def iif2_run(prob: Problem, U0, steps: int, dense=False, tol=TOL_DEFAULT, max_iter=MAX_ITER_DEFAULT, source=None):
    """`steps` IIF2 steps from U0 (species, ndof); source(t) -> (species, ndof)
    array or None (time-dependent forcing, F = P f(R U) + source(t)).
    Returns (U, F(U), infos)."""
    U = np.array(U0, dtype=np.float64).reshape(prob.S, prob.ndof)
    Fn = prob.F(U) + (source(0.0) if source else 0.0)
    infos = []
    for n in range(steps):
        Sn = source((n + 1) * prob.dt) if source else None
        U, Fn, info = iif2_step(prob, U, Fn, dense, tol, max_iter, S_next=Sn)
        infos.append(info)
    return U, Fn, infos


def iif3_step(prob: Problem, U, Fn, Fnm1, dense=False, tol=TOL_DEFAULT, max_iter=MAX_ITER_DEFAULT, S_next=None):
    """One IIF3 step (3.6), the r = 3 member of (3.3) with the coefficients (3.4):

        U^{n+1} = e^{A dt} U^n + dt (alpha_1 F(U^{n+1}) + alpha_0 e^{A dt} F(U^n)
                                     + alpha_{-1} e^{2 A dt} F(U^{n-1})),
        alpha_1 = 5/12, alpha_0 = 2/3, alpha_{-1} = -1/12.

    Reading: terms under the same exponential share one Krylov evaluation (as
    in IIF2, (3.5)): W = exp(A dt)(U^n + alpha_0 dt F^n) + exp(2 A dt)(alpha_{-1}
    dt F^{n-1}), each by its own Arnoldi process with h = dt and h = 2 dt; the
    implicit stage solves U - alpha_1 dt F(U) = W.
    Returns (U^{n+1}, F(U^{n+1}), info)."""
    al = iif_alpha(3)
    dt = prob.dt
    W, kinfo = expv_species(prob, U + al[0] * dt * Fn, dense, h=dt)
    W2, kinfo2 = expv_species(prob, al[1] * dt * Fnm1, dense, h=2.0 * dt)
    U1, F1, ninfo = implicit_stage(prob, W + W2, Fn, tol, max_iter, coef=al[-1] * dt, S=S_next)
    ninfo["krylov"] = kinfo
    ninfo["krylov2"] = kinfo2
    return U1, F1, ninfo


def iif3_run(prob: Problem, U0, steps: int, dense=False, tol=TOL_DEFAULT, max_iter=MAX_ITER_DEFAULT, source=None):
    """`steps` steps of IIF3 from U0; the first step, which has no F(U^{n-1}),
    is one IIF2 step (reading: the paper does not state its start-up).
    Returns (U, F(U), F(U^{n-1}) of the last step, infos)."""
    U = np.array(U0, dtype=np.float64).reshape(prob.S, prob.ndof)
    Fn = prob.F(U) + (source(0.0) if source else 0.0)
    Fp = None
    infos = []
    for n in range(steps):
        Sn = source((n + 1) * prob.dt) if source else None
        if n == 0:
            U1, F1, info = iif2_step(prob, U, Fn, dense, tol, max_iter, S_next=Sn)
        else:
            U1, F1, info = iif3_step(prob, U, Fn, Fp, dense, tol, max_iter, S_next=Sn)
        U, Fp, Fn = U1, Fn, F1
        infos.append(info)
    return U, Fn, Fp, infos
