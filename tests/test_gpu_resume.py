"""Checkpoint and resume of the time stepping.

An IIF2 step (Sec. 3, eq. 3.5) carries the state (U^n, F(U^n)): F from the
accepted Newton iterate is the next step's F^n, and F(U^{n+1}) from the
final iterate is what the step leaves in the cache.  An IIF3 step (eq. 3.6)
also carries F(U^{n-1}).  Running 2K steps in one go must give the same
bits as K steps, a save of that state to host files, a load into a fresh
plan and workspace, and K more steps.
"""
import numpy as np
import pytest

from paper_1810_11111_amd import inputs as I

from _gpu_common import lib, say, to_dev

pytestmark = pytest.mark.gpu


def _ws(plan, M, nrhs):
    import torch

    _, ib = plan.workspace_size(M, nrhs)
    return torch.empty(ib, dtype=torch.uint8, device="cuda")


def _initial(plan, wl, nrhs):
    """The workload's initial data (projected by the library), right-hand
    side r taking instance r's data (instance 0's for a one-instance plan)."""
    x = np.zeros((nrhs, plan.total))
    for r in range(nrhs):
        src = min(r, len(wl.instances) - 1)
        nd, off, _ = plan.info(0)
        for s, (terms, mults, add) in enumerate(wl.initial_condition(src, nd)):
            v = np.zeros(nd)
            for (amp, fac), mult in zip(terms, mults):
                pr = plan.project(0, amp, fac)
                v += pr * (1.0 + mult) if mult is not None else pr
            if add is not None:
                v += add
            x[r, off + s * nd : off + (s + 1) * nd] = v
    return x


@pytest.mark.parametrize("case", ["schnakenberg_d2_iif2", "quadratic_d4_rhs2_iif2", "schnakenberg_d2_iif3"])
def test_resume_from_saved_state_is_bitwise(case, tmp_path):
    import torch

    sg = lib()
    wl, nrhs, iif3 = {
        "schnakenberg_d2_iif2": (I.schnakenberg_d2(N=5, k=2), 1, False),
        "quadratic_d4_rhs2_iif2": (I.quadratic_d4(N=3, nrhs=2), 2, False),
        "schnakenberg_d2_iif3": (I.schnakenberg_d2(N=5, k=2), 1, True),
    }[case]
    insts, dt, M = wl.instances[:1], wl.dt, wl.M
    K = 3
    say("resume", case)

    def start(plan, U0):
        U = to_dev(U0)
        F = torch.zeros_like(U)
        ws = _ws(plan, M, nrhs)
        plan.reaction(U, F, ws, nrhs=nrhs)
        Fp = None
        if iif3:  # IIF3 starts from one IIF2 step (F at two levels)
            Fp = F.clone()
            plan.iif2_step(dt, M, U, F, ws, newton_tol=1e-14, newton_max=8, nrhs=nrhs)
        return U, F, Fp, ws

    def steps(plan, U, F, Fp, ws, n):
        for _ in range(n):
            if iif3:
                plan.iif3_step(dt, M, U, F, Fp, ws, newton_tol=1e-14, newton_max=8, nrhs=nrhs)
            else:
                plan.iif2_step(dt, M, U, F, ws, newton_tol=1e-14, newton_max=8, nrhs=nrhs)
        torch.cuda.synchronize()

    plan = sg.Plan(insts, "fp64")
    U0 = _initial(plan, wl, nrhs)
    # one run of 2K steps
    U, F, Fp, ws = start(plan, U0)
    steps(plan, U, F, Fp, ws, 2 * K)
    ref_U, ref_F = U.cpu().numpy(), F.cpu().numpy()
    # K steps, the state to host files
    U, F, Fp, ws = start(plan, U0)
    steps(plan, U, F, Fp, ws, K)
    np.save(tmp_path / "U.npy", U.cpu().numpy())
    np.save(tmp_path / "F.npy", F.cpu().numpy())
    if iif3:
        np.save(tmp_path / "Fprev.npy", Fp.cpu().numpy())
    plan.close()
    del U, F, Fp, ws
    # a fresh plan and workspace from the files, K more steps
    plan = sg.Plan(insts, "fp64")
    U = to_dev(np.load(tmp_path / "U.npy"))
    F = to_dev(np.load(tmp_path / "F.npy"))
    Fp = to_dev(np.load(tmp_path / "Fprev.npy")) if iif3 else None
    ws = _ws(plan, M, nrhs)
    steps(plan, U, F, Fp, ws, K)
    assert np.all(np.isfinite(ref_U))
    assert np.array_equal(U.cpu().numpy(), ref_U)
    assert np.array_equal(F.cpu().numpy(), ref_F)
    plan.close()
