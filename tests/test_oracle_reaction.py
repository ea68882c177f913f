"""Pins for the reaction transforms R, P and F(U) = P f(R U) (Sec. 3 eq. 3.1; Sec. 5)."""
import numpy as np
import pytest

from oracle import basis, reaction, sparsegrid
from paper_1810_11111_amd import inputs as I


@pytest.mark.parametrize("d,N,k", [(2, 3, 1), (2, 3, 2), (3, 2, 1)])
def test_P_R_is_identity(d, N, k):
    q = reaction.Quadrature(d, N, k)
    U = np.random.default_rng(0).uniform(-1, 1, sparsegrid.dof_count(d, N, k))
    assert np.abs(q.P(q.R(U)) - U).max() < 1e-13


def test_R_matches_pointwise_definition():
    d, N, k = 2, 3, 2
    q = reaction.Quadrature(d, N, k)
    lev, cell, deg, _ = sparsegrid.enumerate_dofs(d, N, k)
    U = np.random.default_rng(1).uniform(-1, 1, lev.shape[0])
    vals = q.R(U)
    rng = np.random.default_rng(2)
    for _ in range(6):
        i0, i1 = rng.integers(0, q.npts1, size=2)
        x0, x1 = q.x1[i0], q.x1[i1]
        direct = 0.0
        for a in range(lev.shape[0]):
            direct += U[a] * basis.hier(k, lev[a, 0], cell[a, 0], deg[a, 0], np.array([x0]))[0] * basis.hier(
                k, lev[a, 1], cell[a, 1], deg[a, 1], np.array([x1])
            )[0]
        assert abs(vals[i0, i1] - direct) < 1e-12


def test_linear_reaction_is_exact():
    d, N, k = 2, 3, 1
    q = reaction.Quadrature(d, N, k)
    U = np.random.default_rng(3).uniform(-1, 1, (1, sparsegrid.dof_count(d, N, k)))
    F = reaction.F(q, I.rx_linear(-2.5), U)
    assert np.abs(F + 2.5 * U).max() < 1e-13


def test_quadratic_exact_for_k1():
    """k=1, f=-u^2: u_h^2 v has degree 3 per axis, so the 2-point rule is the exact
    Galerkin projection; a 4-point rule must give the same coefficients."""
    d, N, k = 2, 3, 1
    U = np.random.default_rng(4).uniform(-1, 1, (1, sparsegrid.dof_count(d, N, k)))
    F2 = reaction.F(reaction.Quadrature(d, N, k, 2), I.rx_quadratic(), U)
    F4 = reaction.F(reaction.Quadrature(d, N, k, 4), I.rx_quadratic(), U)
    assert np.abs(F2 - F4).max() < 1e-13
    # and a cubic (u^3, degree 4 per axis) is not exact with 2 points
    F2c = reaction.F(reaction.Quadrature(d, N, k, 2), I.rx_allen_cahn(), U)
    F4c = reaction.F(reaction.Quadrature(d, N, k, 4), I.rx_allen_cahn(), U)
    assert np.abs(F2c - F4c).max() > 1e-6


def test_homogeneous_steady_states():
    d, N, k = 2, 3, 2
    q = reaction.Quadrature(d, N, k)
    n = sparsegrid.dof_count(d, N, k)
    a, b = 0.1, 0.9
    U = np.zeros((2, n))
    U[0, 0], U[1, 0] = a + b, b / (a + b) ** 2
    assert np.abs(reaction.F(q, I.rx_schnakenberg(a, b), U)).max() < 1e-14
    U = np.zeros((2, n))
    U[0, 0] = 1.0
    assert np.abs(reaction.F(q, I.rx_gray_scott(0.04, 0.06), U)).max() < 1e-14
    U = np.zeros((1, n))
    U[0, 0] = 1.0
    assert np.abs(reaction.F(q, I.rx_allen_cahn(), U)).max() < 1e-14


def test_jacobian_matches_finite_difference():
    rx = I.rx_gray_scott(0.04, 0.06)
    u = [np.array([0.3, 0.7]), np.array([0.2, 0.1])]
    J = reaction.f_jac(rx, u)
    eps = 1e-7
    for t in range(2):
        up = [x.copy() for x in u]
        um = [x.copy() for x in u]
        up[t] += eps
        um[t] -= eps
        fp, fm = reaction.f_eval(rx, up), reaction.f_eval(rx, um)
        for s in range(2):
            assert np.allclose((fp[s] - fm[s]) / (2 * eps), J[s][t], atol=1e-7)
