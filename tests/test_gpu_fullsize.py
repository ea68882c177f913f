"""GPU parity of iif2_step at the full sizes of the high-dimensional and batched workloads.

The expected states are the oracle's (Sec. 3, eq. 3.5 with the Krylov
exponential of eqs. 3.7-3.8 and the implicit stage on F(U) = P f(R U) of
Sec. 5), two IIF2 steps from the oracle's own projection of the initial data,
written by ``tests/golden/make_fullsize.py`` (which calls only the oracle and
the seeded input descriptions) and committed as ``tests/golden/fullsize_*.npz``:

    c3   Allen-Cahn, d=3 N=7 k=1, variable k_ii (13,568 DOF; 16.8M Gauss points per field)
    c5   u_t = Lap u - u^2, d=4 N=6 k=1 (24,320 DOF; 268M Gauss points per field),
         amplitude 0.5, and right-hand sides 0 and 15 of the batch of 16
    c4   64 Gray-Scott instances, d=2, N 5-8, k 1-2 (462,592 DOF)

These shapes select reaction line kernels, LDS layouts and sweep tiers that
the reduced-size tests never reach.

FP64 tolerance per species: the sum over the two steps of 1e-12 ||v_s^n||,
v^n = U^n + dt/2 F(U^n) the Krylov input of step n (the FP64 parity bound of
test_gpu_krylov applied to each step's exponential; the implicit stage that
follows is a contraction).  Reduced-precision
sweeps: relative L2 error against the FP64 oracle within the stated bound
(FP32 1e-4, BF16 3e-2), printed with its margin.
"""
import os

import numpy as np
import pytest

from paper_1810_11111_amd import inputs as I

from _gpu_common import fp64_bound, lib, note, say, to_dev

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(case):
    return np.load(os.path.join(GOLD, f"fullsize_{case}.npz"), allow_pickle=False)


def _ws(plan, M, nrhs=1):
    import torch

    _, ib = plan.workspace_size(M, nrhs)
    return torch.empty(ib, dtype=torch.uint8, device="cuda")


def _run(plan, wl, U0, nrhs, tol, newton_max=12):
    """Two IIF2 steps from U0 (nrhs x total); returns the state and the
    statistics after each step."""
    import torch

    sg = lib()
    U = to_dev(np.ascontiguousarray(U0.reshape(nrhs, -1)))
    F = torch.zeros_like(U)
    ws = _ws(plan, wl.M, nrhs)
    st = torch.zeros(nrhs * len(plan.instances) * 2 * sg.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    plan.reaction(U, F, ws, nrhs=nrhs)
    per_step = []
    for _ in range(2):
        plan.iif2_step(wl.dt, wl.M, U, F, ws, newton_tol=tol, newton_max=newton_max, stats=st, nrhs=nrhs)
        torch.cuda.synchronize()
        per_step.append(sg.stats_array(st).copy())
    out = U.cpu().numpy()
    del ws
    return out, per_step


def _fp64_tol(g, j, s, dt):
    """Summed per-step bound for problem j (golden row), species s."""
    b = fp64_bound(dt, float(g["anorm"][j][s]))
    return sum(b * float(g["vnorm"][j][n][s]) for n in range(2))


def _check_problem(label, got, ref, g, j, nd, S, dt, stats, slot, fp64=True, rel_tol=None):
    for s in range(S):
        seg = slice(s * nd, (s + 1) * nd)
        err = float(np.linalg.norm(got[seg] - ref[seg]))
        if fp64:
            tol = _fp64_tol(g, j, s, dt)
            note(f"{label} species {s}", err, tol, float(g["vnorm"][j][0][s]))
            assert err <= tol, f"{label} species {s}: err {err:.3e} > {tol:.3e}"
        else:
            rel = err / float(np.linalg.norm(ref[seg]))
            note(f"{label} species {s} (relative L2)", rel, rel_tol)
            assert rel <= rel_tol, f"{label} species {s}: relative L2 error {rel:.3e} > {rel_tol:.1e}"
        for n in range(2):
            e = stats[n][slot + s]
            assert e["status"] == 0, (label, n, s, e["status"])
            if fp64:
                assert e["krylov_m"] == int(g["m"][j][n][s]), (label, n, s, e["krylov_m"])
    if fp64:
        for n in range(2):  # corrections per step: the oracle's count, up to one near the threshold
            assert abs(int(stats[n][slot]["newton_iters"]) - int(g["iters"][j][n])) <= 1, (label, n)


@pytest.mark.parametrize("prec,rel_tol", [("fp64", None), ("bf16", 3e-2)])
def test_allen_cahn_d3_full_size(prec, rel_tol):
    """c3 at its full size: d=3 N=7 k=1, k_ii = 1 + 0.5 sin(2 pi x_i); FP64 and BF16 sweeps."""
    sg = lib()
    g = _golden("c3")
    wl = I.allen_cahn_d3()
    say("full size allen_cahn_d3", prec)
    plan = sg.Plan(wl.instances, prec)
    nd = plan.info(0)[0]
    U0, ref = g["U0"][0], g["U2"][0]
    assert U0.size == nd
    got, stats = _run(plan, wl, U0, 1, float(g["newton_tol"]))
    _check_problem(f"c3 {prec}", got[0], ref, g, 0, nd, 1, wl.dt, stats, 0, fp64=prec == "fp64", rel_tol=rel_tol)
    plan.close()


@pytest.mark.parametrize("prec,rel_tol", [("fp64", None), ("fp32", 1e-4)])
def test_quadratic_d4_full_size(prec, rel_tol):
    """c5 at its full size: d=4 N=6 k=1, f = -u^2, amplitude 0.5; FP64 and FP32 sweeps."""
    sg = lib()
    g = _golden("c5")
    wl = I.quadratic_d4()
    say("full size quadratic_d4", prec)
    plan = sg.Plan(wl.instances, prec)
    nd = plan.info(0)[0]
    assert g["U0"][0].size == nd
    got, stats = _run(plan, wl, g["U0"][0], 1, float(g["newton_tol"]))
    _check_problem(f"c5 {prec}", got[0], g["U2"][0], g, 0, nd, 1, wl.dt, stats, 0, fp64=prec == "fp64",
                   rel_tol=rel_tol)
    plan.close()


def test_quadratic_d4_sixteen_rhs_full_size():
    """c5 as a batch of 16 right-hand sides of one plan (nrhs = 16): right-hand
    sides 0 and 15 against their oracle states; the others start from the
    library's projection and are checked for convergence only."""
    sg = lib()
    g0, g15 = _golden("c5_rhs0"), _golden("c5_rhs15")
    wl = I.quadratic_d4(nrhs=16)
    say("full size quadratic_d4, 16 right-hand sides")
    plan = sg.Plan(wl.instances[:1], "fp64")
    nd = plan.info(0)[0]
    U0 = np.zeros((16, nd))
    for r in range(16):
        (terms, _, _), = wl.initial_condition(r, nd)
        U0[r] = sum(plan.project(0, a, f) for a, f in terms)
    # the library's projection of these two agrees with the oracle's to rounding
    for r, g in ((0, g0), (15, g15)):
        assert np.abs(U0[r] - g["U0"][0]).max() <= 1e-14
        U0[r] = g["U0"][0]
    got, stats = _run(plan, wl, U0, 16, float(g0["newton_tol"]))
    for r, g in ((0, g0), (15, g15)):
        _check_problem(f"c5 rhs {r}", got[r], g["U2"][0], g, 0, nd, 1, wl.dt, stats, r * 2)
    for n in range(2):
        assert np.all(stats[n]["status"][0::2] == 0)
    plan.close()


@pytest.mark.parametrize("prec,rel_tol", [("fp64", None), ("fp32", 1e-4)])
def test_gray_scott_batch_full_size(prec, rel_tol):
    """c4 at its full size: all 64 Gray-Scott instances (N 5-8, k 1-2) in one plan,
    every instance and species against its own oracle state."""
    sg = lib()
    g = _golden("c4")
    wl = I.gray_scott_batch()
    say("full size gray_scott_batch 64", prec)
    plan = sg.Plan(wl.instances, prec)
    assert g["U0"].size == plan.total
    got, stats = _run(plan, wl, g["U0"], 1, float(g["newton_tol"]), newton_max=6)
    got = got[0]
    for i in range(len(wl.instances)):
        nd, off, _ = plan.info(i)
        seg = slice(off, off + 2 * nd)
        _check_problem(f"c4 {prec} instance {i}", got[seg], g["U2"][seg], g, i, nd, 2, wl.dt, stats, i * 2,
                       fp64=prec == "fp64", rel_tol=rel_tol)
    plan.close()
