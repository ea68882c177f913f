"""Pins for the explicit RK comparator and the CFL study (Sec. 4, Tables 1-2)."""
import json
import os

import numpy as np
import pytest

from oracle import iif, operator, rk
from paper_1810_11111_amd import inputs as I


def _table(golden_dir, key):
    with open(os.path.join(golden_dir, "paper_values.json")) as fh:
        return json.load(fh)[key]


def test_real_stability_limits():
    """|R(-x)| <= 1 on [0, z_s]: z_2 = 2 exactly; z_3 is the real root of
    1 - x + x^2/2 - x^3/6 = -1 (about 2.5127)."""
    assert abs(rk.real_stability_limit(2) - 2.0) < 1e-9
    z3 = rk.real_stability_limit(3)
    assert abs(1 - z3 + z3 ** 2 / 2 - z3 ** 3 / 6 + 1.0) < 1e-9
    assert 2.5127 < z3 < 2.5128


def test_table1_rk3_over_rk2_is_the_stability_ratio(golden_dir):
    """Every row of Table 1: CFL(RK3) / CFL(RK2) = z_3 / z_2 (same operator)."""
    t = _table(golden_dir, "cfl_table1")
    want = rk.real_stability_limit(3) / rk.real_stability_limit(2)
    pairs = [tuple(t["full"][p].values()) for p in ("P1", "P2")]
    pairs += [tuple(r[p]) for key in ("sparse2d", "sparse3d") for r in t[key] for p in ("P1", "P2")]
    for rk2, rk3 in pairs:
        assert abs(rk3 / rk2 / want - 1.0) < 0.015, (rk2, rk3)


def test_table1_follows_from_table2_eigenvalues(golden_dir):
    """The paper's own lambda_0 (Table 2) with z_2 gives its RK2 CFL (Table 1):
    CFL = d z_2 / (|lambda_0| h_N^2), which fixes the reading of the CFL number."""
    t1 = _table(golden_dir, "cfl_table1")
    for r in _table(golden_dir, "lambda0_table2")["rows"]:
        d, k, N = r["d"], r["k"], r["N"]
        if d != 2:
            continue
        p = f"P{k}"
        row = [x for x in t1["sparse2d"] if x["N"] == N][0]
        assert abs(rk.cfl_limit(r["sparse"], d, N, 2) / row[p][0] - 1.0) < 0.02, (r, row)
        assert abs(rk.cfl_limit(r["full"], d, N, 2) / t1["full"][p]["RK2"] - 1.0) < 0.02, r


@pytest.mark.parametrize("d,k,N", [(2, 1, 3), (2, 1, 4), (2, 1, 5), (2, 2, 3), (2, 2, 4), (3, 1, 3), (3, 1, 4)])
def test_sparse_over_full_cfl_matches_table1(golden_dir, d, k, N):
    """Our operator's CFL ratio sparse/full (= lambda_0 full / lambda_0 sparse)
    against Table 1's; absolute CFL values are not pinned (penalty reading)."""
    t = _table(golden_dir, "cfl_table1")
    row = [x for x in t[f"sparse{d}d"] if x["N"] == N][0]
    paper = row[f"P{k}"][0] / t["full"][f"P{k}"]["RK2"]
    A = operator.assemble_A(d, N, k).toarray()
    lam_sparse = np.linalg.eigvalsh(A).min()
    lam_full = d * np.linalg.eigvalsh(-operator.full_grid_sipg(N, k)).min()
    ours = rk.cfl_limit(lam_sparse, d, N, 2) / rk.cfl_limit(lam_full, d, N, 2)
    assert abs(ours / paper - 1.0) < 0.03, (ours, paper)


@pytest.mark.parametrize("order", [2, 3])
def test_rk_step_is_the_stability_polynomial_for_linear_problems(order):
    """f = c u: one step multiplies by R(dt (A + c I)) exactly."""
    prob = iif.Problem(2, 3, 1, [0.5], I.rx_linear(-0.7), 0.001, 10)
    U = np.random.default_rng(5).uniform(-1, 1, (1, prob.ndof))
    A = prob.A[0].toarray() - 0.7 * np.eye(prob.ndof)
    Z = 0.001 * A
    R = sum(np.linalg.matrix_power(Z, j) / np.prod(range(1, j + 1)) for j in range(order + 1))
    got = rk.rk_step(prob, U, 0.001, order)
    assert np.abs(got[0] - R @ U[0]).max() < 1e-13


@pytest.mark.parametrize("order", [2, 3])
def test_rk_stable_below_limit_unstable_above(order):
    """dt just below z_s / |lambda_0| stays bounded; just above grows (Sec. 4)."""
    prob = iif.Problem(2, 4, 1, [1.0], I.rx_zeros(1), 1.0, 10)
    lam0 = np.linalg.eigvalsh(prob.A[0].toarray()).min()
    dt0 = rk.real_stability_limit(order) / abs(lam0)
    U0 = np.random.default_rng(6).uniform(-1, 1, (1, prob.ndof))
    for fac, grows in ((0.98, False), (1.03, True)):
        U = U0.copy()
        for _ in range(400):
            U = rk.rk_step(prob, U, fac * dt0, order)
        ratio = np.linalg.norm(U) / np.linalg.norm(U0)
        assert (ratio > 10.0) == grows, (fac, ratio)
