"""Pins for IIF2 and its implicit reaction stage (Sec. 3, eqs. 3.3-3.6; Sec. 5)."""
import json
import os

import numpy as np
import pytest

from oracle import iif, krylov, project, sparsegrid
from paper_1810_11111_amd import inputs as I


def test_lagrange_coefficients_give_iif2_iif3(golden_dir):
    with open(os.path.join(golden_dir, "paper_values.json")) as fh:
        g = json.load(fh)["iif_alpha"]
    a2 = iif.iif_alpha(2)
    assert np.allclose([a2[-1], a2[0]], g["r2"], atol=1e-15)
    a3 = iif.iif_alpha(3)
    assert np.allclose([a3[-1], a3[0], a3[1]], g["r3"], atol=1e-15)


def test_pointwise_stage_has_newton_root():
    d, N, k = 2, 3, 1
    prob = iif.Problem(d, N, k, [0.01, 1.0], I.rx_schnakenberg(0.1, 0.9), 0.2, 10)
    n = prob.ndof
    rng = np.random.default_rng(0)
    W = np.zeros((2, n))
    W[0, 0], W[1, 0] = 1.0, 0.9
    W += rng.uniform(-0.05, 0.05, W.shape)
    Fn = prob.F(W)
    U1, _, info = iif.implicit_stage(prob, W, Fn, tol=1e-15)
    U2 = iif.implicit_stage_newton_dense(prob, W, Fn)
    assert info["converged"]
    assert np.abs(U1 - U2).max() <= 1e-13 * np.abs(U2).max()
    G = U1 - 0.1 * prob.F(U1) - W
    assert np.linalg.norm(G) < 1e-13


def test_linear_stage_closed_form():
    d, N, k = 2, 3, 1
    prob = iif.Problem(d, N, k, [1.0], I.rx_linear(-1.0), 0.01, 10)
    W = np.random.default_rng(1).uniform(-1, 1, (1, prob.ndof))
    U, _, info = iif.implicit_stage(prob, W, prob.F(W), tol=1e-15)
    assert np.abs(U - W / 1.005).max() < 1e-15 and info["iters"] <= 2


def test_constant_state_with_linear_decay():
    d, N, k = 2, 4, 1
    dt = 0.05
    prob = iif.Problem(d, N, k, [1.0], I.rx_linear(-1.0), dt, 10)
    U0 = np.zeros((1, prob.ndof))
    U0[0, 0] = 0.7
    U, _, infos = iif.iif2_run(prob, U0, 6)
    assert infos[0]["krylov"][0]["m"] == 1
    ref = 0.7 * ((1 - dt / 2) / (1 + dt / 2)) ** 6
    assert abs(U[0, 0] - ref) < 1e-15 and np.abs(U[0, 1:]).max() < 1e-15


def test_zero_reaction_is_repeated_exponential():
    d, N, k = 2, 4, 1
    prob = iif.Problem(d, N, k, [0.1], I.rx_zeros(1), 0.01, 12)
    U0 = np.random.default_rng(2).uniform(-1, 1, (1, prob.ndof))
    U, _, _ = iif.iif2_run(prob, U0, 3)
    v = U0[0]
    for _ in range(3):
        v, _ = krylov.expv(prob.A[0], prob.dt, v, 12, prob.anorm[0])
    assert np.abs(U[0] - v).max() < 1e-14


def test_mean_trapezoid_identity_with_dense_exponential():
    """Periodic: exp(A dt) keeps the mean coefficient, so U_0^{n+1} = U_0^n + dt/2 (F_0^n + F_0^{n+1})."""
    d, N, k = 2, 3, 1
    prob = iif.Problem(d, N, k, [1.0], I.rx_quadratic(-1.0), 0.01, 10)
    U0 = project.project_terms(d, N, k, [(0.5, [I.SIN, I.SIN]), (0.3, [I.ONE, I.ONE])])[None]
    F0 = prob.F(U0)
    U1, F1, _ = iif.iif2_step(prob, U0, F0, dense=True, tol=1e-15)
    assert abs(U1[0, 0] - (U0[0, 0] + 0.005 * (F0[0, 0] + F1[0, 0]))) < 1e-14


@pytest.mark.slow
def test_example4_matches_table7(golden_dir):
    """Example 4 (stiff linear 2-species system): the IIF2 error is dominated by the
    time discretisation, so its magnitude is pinned, not only its order.
    Initial v is read as (b - c) prod cos(2 pi x_i), the value of the exact solution at t=0."""
    with open(os.path.join(golden_dir, "paper_values.json")) as fh:
        g = json.load(fh)["example4_table7"]
    d, k, T, M = g["d"], g["k"], g["T"], g["M"]
    a, b, c = g["a"], g["b"], g["c"]
    kk = 1.0 / (4 * d * np.pi ** 2)
    uerr, verr = [], []
    for N in (5, 6, 7):
        dt = 2.0 ** -N
        prob = iif.Problem(d, N, k, [kk * a, kk * a], I.rx_stiff_linear_system(b, c), dt, M)
        P = project.project_terms(d, N, k, [(1.0, [I.COS] * d)])
        U, _, _ = iif.iif2_run(prob, np.array([2 * P, (b - c) * P]), int(round(T / dt)))
        fu = np.exp(-(b + a) * T) + np.exp(-(c + a) * T)
        fv = (b - c) * np.exp(-(c + a) * T)
        uerr.append(project.l2_error(U[0], fu * P, fu ** 2 * 0.25))
        verr.append(project.l2_error(U[1], fv * P, fv ** 2 * 0.25))
    for i in range(3):
        assert abs(uerr[i] / g["u_error"][i] - 1) < 0.15, (uerr, g["u_error"])
        assert abs(verr[i] / g["v_error"][i] - 1) < 0.15, (verr, g["v_error"])
        assert abs(verr[i] / uerr[i] / (b - c) - 1) < 0.02
    assert all(1.7 < np.log2(uerr[i] / uerr[i + 1]) < 2.3 for i in range(2))


def _ode_error(scheme, dt, T=1.0, u0=0.8):
    """Spatially constant state, f = -u^2: A keeps constants (exp(A dt) is the
    identity on them, Krylov breaks down at m = 1), so the scheme reduces to
    its scalar form for u' = -u^2, u(t) = u0 / (1 + u0 t)."""
    prob = iif.Problem(2, 3, 1, [1.0], I.rx_quadratic(-1.0), dt, 8)
    U0 = np.zeros((1, prob.ndof))
    U0[0, 0] = u0
    steps = int(round(T / dt))
    if scheme == 2:
        U, _, _ = iif.iif2_run(prob, U0, steps, tol=1e-15)
    else:
        U, _, _, _ = iif.iif3_run(prob, U0, steps, tol=1e-15)
    assert np.abs(U[0, 1:]).max() < 1e-14
    return abs(U[0, 0] - u0 / (1.0 + u0 * T))


def test_iif3_is_third_order_and_iif2_second_order_in_time():
    """(3.3)-(3.6): IIF3 (with one IIF2 start-up step) converges at order 3 and
    IIF2 at order 2; a wrong coefficient or exponential shift in the IIF3
    combination drops its order."""
    e3 = [_ode_error(3, dt) for dt in (0.1, 0.05, 0.025)]
    e2 = [_ode_error(2, dt) for dt in (0.1, 0.05, 0.025)]
    r3 = [np.log2(e3[i] / e3[i + 1]) for i in range(2)]
    r2 = [np.log2(e2[i] / e2[i + 1]) for i in range(2)]
    assert all(2.8 < r < 3.3 for r in r3), r3
    assert all(1.8 < r < 2.2 for r in r2), r2
    assert e3[-1] < e2[-1] / 10


def test_iif3_zero_reaction_is_repeated_exponential():
    d, N, k = 2, 4, 1
    prob = iif.Problem(d, N, k, [0.1], I.rx_zeros(1), 0.01, 12)
    U0 = np.random.default_rng(3).uniform(-1, 1, (1, prob.ndof))
    U, _, _, infos = iif.iif3_run(prob, U0, 3)
    v = U0[0]
    for _ in range(3):
        v, _ = krylov.expv(prob.A[0], prob.dt, v, 12, prob.anorm[0])
    assert np.abs(U[0] - v).max() < 1e-14
    assert infos[1]["krylov2"][0]["m"] == 0  # exp(2 A dt) of the zero vector


def test_iif3_stage_root_with_dense_exponentials():
    """The IIF3 stage solves U - (5/12) dt F(U) = W with W from the two
    exponentials; with dense exponentials the result satisfies (3.6) exactly."""
    from scipy.linalg import expm

    d, N, k = 2, 3, 1
    dt = 0.02
    prob = iif.Problem(d, N, k, [0.5], I.rx_quadratic(-1.0), dt, 10)
    U0 = project.project_terms(d, N, k, [(0.5, [I.SIN, I.SIN]), (0.3, [I.ONE, I.ONE])])[None]
    Um1 = 0.9 * U0
    Fn, Fm1 = prob.F(U0), prob.F(Um1)
    U1, F1, info = iif.iif3_step(prob, U0, Fn, Fm1, dense=True, tol=1e-15)
    E = expm(dt * prob.A[0].toarray() if hasattr(prob.A[0], "toarray") else dt * prob.A[0])
    rhs = E @ U0[0] + dt * (5 / 12 * F1[0] + 2 / 3 * (E @ Fn[0]) - 1 / 12 * (E @ (E @ Fm1[0])))
    assert info["converged"]
    assert np.abs(U1[0] - rhs).max() < 1e-13 * max(1.0, np.abs(rhs).max())


def test_local_stage_equals_galerkin_for_linear_reaction():
    """f = lambda u: pointwise u = w / (1 - c lambda), and P R = I on the sparse
    space, so the local stage is the Galerkin stage W / (1 - c lambda)."""
    prob = iif.Problem(2, 3, 1, [1.0], I.rx_linear(-2.0), 0.05, 10)
    W = np.random.default_rng(7).uniform(-1, 1, (1, prob.ndof))
    U, _ = iif.implicit_stage_local(prob, W)
    assert np.abs(U - W / (1 + 0.05)).max() < 1e-14


def test_local_stage_solves_the_pointwise_problem():
    prob = iif.Problem(2, 3, 2, [0.01, 1.0], I.rx_schnakenberg(0.1, 0.9), 0.2, 10)
    rng = np.random.default_rng(8)
    W = np.zeros((2, prob.ndof))
    W[0, 0], W[1, 0] = 1.0, 0.9
    W += rng.uniform(-0.05, 0.05, W.shape)
    c = 0.1
    wq = [prob.quad.R(W[s]) for s in range(2)]
    uq = iif.solve_pointwise(prob.rx, wq, c)
    f = iif.reaction.f_eval(prob.rx, uq)
    for s in range(2):
        assert np.abs(uq[s] - c * f[s] - wq[s]).max() < 1e-14
    # close to, but not equal to, the Galerkin root (a different scheme)
    Ul, _ = iif.implicit_stage_local(prob, W, c)
    Ug, _, _ = iif.implicit_stage(prob, W, prob.F(W), tol=1e-15, coef=c)
    diff = np.abs(Ul - Ug).max()
    assert 1e-10 < diff < 1e-3, diff


def test_local_stage_example3_second_order():
    """Example 3 (zero Dirichlet, u^2, forcing) with the local stage, P1 IIF2:
    still second order in the L2 error."""
    import math

    errs = []
    for N in (3, 4, 5):
        wl = I.example3(2, N, 1)
        inst = wl.instances[0]
        prob = iif.Problem(inst.d, N, 1, inst.D, inst.rx, wl.dt, wl.M, bc="dirichlet")
        U0 = project.project_terms(2, N, 1, [(1.0, [I.SIN, I.SIN])])[None]
        S0 = sum(project.project_separable(2, N, 1, a, f) for a, f, _ in wl.sources)
        U, _, _ = iif.iif2_run_local(prob, U0, wl.steps, source=lambda t: (math.exp(-2 * t) * S0)[None])
        T = wl.steps * wl.dt
        errs.append(project.l2_error(U[0], math.exp(-T) * U0[0], math.exp(-2 * T) * 0.25))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.05 and all(1.4 < r < 2.8 for r in rates), (errs, rates)
