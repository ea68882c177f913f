"""Pins for the zero-Dirichlet operator and forced problems (Sec. 2.1 boundary
convention after eq. 2.11; Sec. 4, Examples 2 and 3)."""
import math

import numpy as np
import pytest

from oracle import iif, operator, project
from paper_1810_11111_amd import inputs as I


@pytest.mark.parametrize("k", [1, 2])
def test_dirichlet_1d_operator_spectrum(k):
    """Symmetric positive definite (no constant null space), and its smallest
    eigenvalues converge to those of -d^2/dx^2 with zero ends, (pi m)^2."""
    errs = []
    for N in (3, 4, 5):
        B = operator.full_grid_sipg(N, k, bc="dirichlet")
        assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
        ev = np.sort(np.linalg.eigvalsh(B))
        assert ev[0] > 0
        errs.append(max(abs(ev[m - 1] / (math.pi * m) ** 2 - 1.0) for m in (1, 2, 3)))
    # O(h^{2k}) eigenvalue convergence: two refinements gain about 2^{4k}
    assert errs[-1] < 1e-2 and errs[0] / errs[2] > 0.75 * 2 ** (4 * k), errs


def test_dirichlet_reduces_to_periodic_away_from_the_boundary():
    """Only the two boundary faces differ: rows of interior cells not touching
    the boundary agree with the periodic operator."""
    N, k = 4, 1
    Bd = operator.full_grid_sipg(N, k, bc="dirichlet")
    Bp = operator.full_grid_sipg(N, k)
    K1, nc = k + 1, 2 ** N
    inner = slice(2 * K1, (nc - 2) * K1)
    assert np.abs(Bd[inner] - Bp[inner]).max() == 0.0
    assert np.abs(Bd[:K1] - Bp[:K1]).max() > 1.0


def test_sparse_dirichlet_operator_is_negative_definite():
    A = operator.assemble_A(2, 4, 1, bc="dirichlet").toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    ev = np.sort(np.linalg.eigvalsh(A))
    assert ev[-1] < 0
    # smoothest mode sin(pi x) sin(pi y): -2 pi^2 up to discretisation
    assert abs(ev[-1] / (-2.0 * math.pi ** 2) - 1.0) < 0.02


def _run_example(wl, scheme=2):
    inst = wl.instances[0]
    prob = iif.Problem(inst.d, inst.N, inst.k, inst.D, inst.rx, wl.dt, wl.M,
                       bc="dirichlet" if inst.bc else "periodic")
    U0 = project.project_terms(inst.d, inst.N, inst.k, [(1.0, [I.SIN] * inst.d)])[None]
    S0 = np.zeros(prob.ndof)
    for a, f, _ in wl.sources:
        S0 += project.project_separable(inst.d, inst.N, inst.k, a, f)
    rates = [r for _, _, r in wl.sources]
    assert len(set(rates)) == 1
    src = lambda t: (math.exp(-rates[0] * t) * S0)[None]  # noqa: E731
    run = iif.iif2_run if scheme == 2 else iif.iif3_run
    res = run(prob, U0, wl.steps, tol=1e-13, source=src)
    U = res[0]
    T = wl.steps * wl.dt
    PU = math.exp(-T) * U0[0]
    return project.l2_error(U[0], PU, math.exp(-2 * T) * 0.5 ** inst.d)


@pytest.mark.parametrize("example", [I.example2, I.example3])
def test_examples_2_3_p1_iif2_second_order(example):
    """P1 with IIF2, dt = h_N, T = 1: errors fall at about second order (Tables 5
    and 6 print 1.5-2.1; magnitudes are not pinned)."""
    errs = [_run_example(example(2, N, 1)) for N in (3, 4, 5)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.05 and all(1.4 < r < 2.8 for r in rates), (errs, rates)


def test_example3_p2_iif3_third_order():
    """P2 with IIF3 (Tables 5-6 pair them): about third order."""
    errs = [_run_example(I.example3(2, N, 2), scheme=3) for N in (3, 4)]
    rate = math.log2(errs[0] / errs[1])
    assert errs[-1] < 5e-3 and 2.3 < rate < 3.8, (errs, rate)
