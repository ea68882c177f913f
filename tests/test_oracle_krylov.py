"""Pins for the Krylov exponential (Sec. 3, eqs. 3.7-3.8) and exp(h H_M)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import iif, krylov, operator, project
from paper_1810_11111_amd import inputs as I


@pytest.fixture(scope="module")
def small():
    A = operator.assemble_A(2, 4, 1)
    return A, operator.inf_norm(A)


def test_hessenberg_symmetric_tridiagonal(small):
    A, an = small
    v = np.random.default_rng(1).uniform(-1, 1, A.shape[0])
    V, H, m, beta = krylov.arnoldi_mgs(lambda x: A @ x, v, 20, an)
    Hm = H[:m, :m]
    assert m == 20
    assert np.abs(np.triu(Hm, 2)).max() <= 1e-10 * np.abs(Hm).max()
    assert np.abs(Hm - Hm.T).max() <= 1e-10 * np.abs(Hm).max()
    assert np.abs(V[:, :m].T @ V[:, :m] - np.eye(m)).max() < 1e-10


def test_contraction(small):
    A, an = small
    for seed in range(3):
        v = np.random.default_rng(seed).uniform(-1, 1, A.shape[0])
        w, _ = krylov.expv(A, 1e-3, v, 15, an)
        assert np.linalg.norm(w) <= np.linalg.norm(v) * (1 + 1e-14)


def test_eigenvector_gives_m1_and_exact_result(small):
    A, an = small
    lam, Q = np.linalg.eigh(A.toarray())
    for idx in (0, len(lam) // 2, len(lam) - 2):
        v = Q[:, idx]
        w, info = krylov.expv(A, 1e-4, v, 20, an)
        assert info["m"] == 1
        assert np.linalg.norm(w - np.exp(1e-4 * lam[idx]) * v) <= 1e-12


def test_zero_vector_and_clamp(small):
    A, an = small
    w, info = krylov.expv(A, 0.1, np.zeros(A.shape[0]), 10, an)
    assert info["m"] == 0 and not np.any(w)
    A1 = operator.assemble_A(2, 2, 1)
    v = np.random.default_rng(5).uniform(-1, 1, A1.shape[0])
    w, info = krylov.expv(A1, 1e-3, v, 10 * A1.shape[0], operator.inf_norm(A1))
    assert info["m"] <= A1.shape[0]


def test_full_dimension_equals_dense_exponential():
    A = operator.assemble_A(2, 2, 1)
    an = operator.inf_norm(A)
    v = np.random.default_rng(2).uniform(-1, 1, A.shape[0])
    h = 2e-4
    w, info = krylov.expv(A, h, v, A.shape[0], an)
    ref = krylov.dense_expv(A, h, v)
    lam, Q = np.linalg.eigh(A.toarray())
    ref2 = Q @ (np.exp(h * lam) * (Q.T @ v))
    assert np.linalg.norm(ref - ref2) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(w - ref) <= 1e-10 * np.linalg.norm(ref)


def test_expm_pade_vs_eigh_on_hessenberg(small):
    A, an = small
    v = np.random.default_rng(3).uniform(-1, 1, A.shape[0])
    V, H, m, _ = krylov.arnoldi_mgs(lambda x: A @ x, v, 25, an)
    for h in (1e-5, 1e-4, 1e-3):
        E1 = sla.expm(h * H[:m, :m])[:, 0]
        E2 = krylov.expm_eigh(h * H[:m, :m])[:, 0]
        assert np.linalg.norm(E1 - E2) <= 1e-13 * max(1.0, h * an) * np.linalg.norm(E1)


def test_table3_plateau_for_m_at_least_25(golden_dir):
    """Table 3: at N=7, T=0.6 in one step the error does not change for M >= 25."""
    with open(os.path.join(golden_dir, "paper_values.json")) as fh:
        g = json.load(fh)["table3_krylov_plateau"]
    d, N, k, T = g["d"], g["N"], g["k"], g["T"]
    A = operator.assemble_A(d, N, k, D=1.0 / (8 * np.pi ** 2))
    an = operator.inf_norm(A)
    U0 = project.project_terms(d, N, k, [(1.0, [I.SIN] * d)])
    fac = np.exp(-T)
    errs = []
    for M in (25, 100):
        w, _ = krylov.expv(A, T, U0, M, an)
        errs.append(project.l2_error(w, fac * U0, fac ** 2 * 0.25))
    paper = g["error_dt06"]
    assert abs(paper[0] / paper[1] - 1) < 0.02
    assert abs(errs[0] / errs[1] - 1) < 0.02


@pytest.mark.slow
def test_example1_orders_match_table4(golden_dir):
    """Table 4: P1 2D orders close to 2 (printed 1.81, 1.96, 2.00 for N = 4..7)."""
    d, k = 2, 1
    errs = []
    for N in (4, 5, 6):
        kk = 1.0 / (4 * d * np.pi ** 2)
        prob = iif.Problem(d, N, k, [kk], I.rx_zeros(1), 2.0 ** -N, 25)
        U0 = project.project_terms(d, N, k, [(1.0, [I.SIN] * d)])[None]
        U, _, _ = iif.iif2_run(prob, U0, 2 ** (N + 1))
        fac = np.exp(-2.0)
        errs.append(project.l2_error(U[0], fac * U0[0], fac ** 2 * 0.25))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.75 < o < 2.35 for o in orders), orders
