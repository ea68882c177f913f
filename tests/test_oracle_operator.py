"""Pins for the explicit operator A = -B (Sec. 2.1, eqs. 2.10-2.11; Lemmas 2.1-2.2)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import basis, operator, sparsegrid


def _bilinear_brute(N, k, sigma, kappa, a, b):
    """B(v_b, v_a) straight from the definition, with hier() evaluations only."""
    (la, ja, pa), (lb, jb, pb) = a, b
    h = 2.0 ** (-N)
    xg, wg = np.polynomial.legendre.leggauss(10)
    xg, wg = 0.5 * (xg + 1), 0.5 * wg
    kap = (lambda x: np.ones_like(x)) if kappa is None else kappa
    tot = 0.0
    for c in range(2 ** N):
        x = (c + xg) * h
        tot += np.sum(wg * h * kap(x) * basis.hier(k, la, ja, pa, x, True) * basis.hier(k, lb, jb, pb, x, True))
    eps = 1e-9 * h

    def tr(lev, j, p, x, der):
        # periodic one-sided limits through points just inside each side
        xl = (x - eps) % 1.0
        xr = (x + eps) % 1.0
        return (basis.hier(k, lev, j, p, np.array([xl]), der)[0], basis.hier(k, lev, j, p, np.array([xr]), der)[0])

    for e in range(2 ** N):
        xe = e * h
        ke = float(kap(np.array([xe]))[0])
        ua, ua_ = tr(la, ja, pa, xe, False)
        ub, ub_ = tr(lb, jb, pb, xe, False)
        da, da_ = tr(la, ja, pa, xe, True)
        db, db_ = tr(lb, jb, pb, xe, True)
        ja_, jb_ = ua - ua_, ub - ub_
        tot += -ke * 0.5 * (db + db_) * ja_ - ke * 0.5 * (da + da_) * jb_ + sigma / h * ja_ * jb_
    return tot


@pytest.mark.parametrize("k,kappa", [(1, None), (2, None), (1, "sin")])
def test_hier_operator_entries_brute_force(k, kappa):
    N = 3
    kf = None if kappa is None else (lambda x: 1.0 + 0.5 * np.sin(2 * np.pi * x))
    Bh = operator.hier_operator_1d(N, k, 20.0, kf)
    funcs = basis.hier_list_1d(N, k)
    rng = np.random.default_rng(0)
    picks = [(r, c) for r in range(len(funcs)) for c in range(len(funcs))]
    rng.shuffle(picks)
    scale = np.abs(Bh).max()
    for r, c in picks[:120]:
        ref = _bilinear_brute(N, k, 20.0, kf, funcs[r], funcs[c])
        assert abs(Bh[r, c] - ref) <= 2e-7 * scale, (funcs[r], funcs[c], Bh[r, c], ref)


@pytest.mark.parametrize("d,N,k", [(2, 4, 1), (2, 3, 2), (3, 3, 1)])
def test_symmetric_negative_semidefinite_one_zero_mode(d, N, k):
    A = operator.assemble_A(d, N, k)
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() <= 1e-12 * np.abs(Ad).max()
    const = np.zeros(A.shape[0])
    const[0] = 1.0  # the constant function: level-0, degree-0 in every axis
    assert np.abs(A @ const).max() <= 1e-12 * np.abs(Ad).max()
    ev = np.linalg.eigvalsh(Ad)
    assert ev[-1] <= 1e-9 * abs(ev[0])
    assert abs(ev[-1]) <= 1e-9 * abs(ev[0]) and ev[-2] < -1.0  # exactly one zero eigenvalue


def test_kron_sum_restriction_matches_assembly():
    """A equals -(Bh (x) I + I (x) Bh) on the full tensor index set, restricted to S."""
    d, N, k = 2, 4, 1
    Bh = sp.csr_matrix(operator.hier_operator_1d(N, k))
    n1 = Bh.shape[0]
    full = -(sp.kron(Bh, sp.eye(n1)) + sp.kron(sp.eye(n1), Bh)).tocsr()
    _, _, _, r1d = sparsegrid.enumerate_dofs(d, N, k)
    idx = r1d[:, 0] * n1 + r1d[:, 1]
    ref = full[idx][:, idx].toarray()
    A = operator.assemble_A(d, N, k).toarray()
    assert np.abs(A - ref).max() <= 1e-13 * np.abs(ref).max()


def test_sparse_full_lambda0_ratio_matches_table2(golden_dir):
    with open(os.path.join(golden_dir, "paper_values.json")) as fh:
        rows = json.load(fh)["lambda0_table2"]["rows"]
    for r in rows:
        d, k, N = r["d"], r["k"], r["N"]
        A = operator.assemble_A(d, N, k).toarray()
        lam_sparse = np.linalg.eigvalsh(A).min()
        lam_full = d * np.linalg.eigvalsh(-operator.full_grid_sipg(N, k)).min()
        ratio, paper = lam_sparse / lam_full, r["sparse"] / r["full"]
        tol = 0.015 if k == 1 else 0.035
        assert abs(ratio / paper - 1.0) < tol, (r, ratio, paper)


def test_smooth_eigenvalue_converges_to_minus_4pi2():
    errs = []
    for N in (3, 4, 5):
        ev = np.sort(np.linalg.eigvalsh(operator.full_grid_sipg(N, 1)))
        errs.append(abs(ev[1] - 4 * np.pi ** 2))
    assert errs[0] > 3 * errs[1] > 9 * errs[2]


def test_single_periodic_cell_by_hand():
    """N = 0, k = 1: one cell whose two ends meet at the periodic face.  For
    phi_1 = sqrt(3)(2x-1): int phi_1'^2 = 12, jump 2 sqrt(3), mean derivative
    2 sqrt(3), so B = 12 - 2*12 + 20*12 = 228; phi_0 = 1 has no jump and no slope."""
    B = operator.full_grid_sipg(0, 1)
    assert np.allclose(B, [[0.0, 0.0], [0.0, 228.0]], atol=1e-12)


def test_inf_norm():
    A = operator.assemble_A(2, 3, 1)
    assert operator.inf_norm(A) == pytest.approx(np.abs(A.toarray()).sum(axis=1).max(), rel=1e-15)
