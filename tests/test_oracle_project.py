"""Pins for the L2 projection of initial data and the Parseval error (Sec. 2.2, Thm. 2.4)."""
import math

import numpy as np

from oracle import project, sparsegrid
from paper_1810_11111_amd import inputs as I


def test_constant_projects_to_first_coefficient():
    U = project.project_terms(2, 4, 1, [(2.5, [I.ONE, I.ONE])])
    assert abs(U[0] - 2.5) < 1e-14 and np.abs(U[1:]).max() < 1e-14


def test_dyadic_box_is_represented_exactly():
    # [3/8, 5/8) is a union of level-3 cells: in V_N for N >= 3, so ||P chi||^2 = ||chi||^2
    box = ("box", 0.375, 0.625)
    U = project.project_terms(2, 6, 1, [(1.0, [box, box])])
    assert abs(U @ U - 0.25 ** 2) < 1e-14
    U1 = project.project_terms(1, 3, 1, [(1.0, [box])])
    assert abs(U1 @ U1 - 0.25) < 1e-14


def test_sine_projection_norm_and_error_identity():
    gaps = []
    for N in (4, 5, 6):
        U = project.project_terms(2, N, 1, [(1.0, [I.SIN, I.SIN])])
        # ||u||^2 = 1/4 and ||u - Pu||^2 = ||u||^2 - ||Pu||^2 >= 0, shrinking with N
        gaps.append(0.25 - U @ U)
    assert 0.0 <= gaps[2] < gaps[1] < gaps[0] < 1e-3
    assert gaps[1] / gaps[2] > 8.0  # ||u - Pu|| = O(h^2) up to log factors for P1
    assert project.l2_error(U, U, 0.25) == math.sqrt(max(0.25 - U @ U, 0.0))


def test_fourier_mode_expansion_is_pointwise_exact():
    rng = np.random.default_rng(0)
    freqs, phase, amp = np.array([2, -1, 3]), 0.7, 1.3
    terms = I.fourier_mode_terms(amp, freqs, phase)
    for _ in range(5):
        x = rng.uniform(0, 1, 3)
        tot = 0.0
        for a, fac in terms:
            val = a
            for m, (_, f, ph) in enumerate(fac):
                val *= math.cos(2 * math.pi * f * x[m] + ph)
            tot += val
        assert abs(tot - amp * math.cos(2 * math.pi * freqs @ x + phase)) < 1e-13


def test_separable_projection_is_product_of_1d():
    d, N, k = 3, 3, 1
    U = project.project_separable(d, N, k, 1.0, [I.SIN, I.COS, I.ONE])
    c0, c1 = project.project_1d(N, k, I.SIN), project.project_1d(N, k, I.COS)
    _, _, _, r1d = sparsegrid.enumerate_dofs(d, N, k)
    assert np.allclose(U, c0[r1d[:, 0]] * c1[r1d[:, 1]] * (r1d[:, 2] == 0), atol=1e-15)
