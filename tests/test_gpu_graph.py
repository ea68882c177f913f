"""A HIP graph of one IIF2 step (Sec. 3, eq. 3.5) replays bit for bit like the eager step.

The benchmark times graph replays of iif2_step; every launch of a step has
fixed arguments (convergence is a device flag, not host control), so a
captured step must reproduce the eager step exactly.  Each replay runs
after eager work and a synchronisation of its own, and every replay is
checked against the eager state of the same step count.
"""
import numpy as np
import pytest

from paper_1810_11111_amd import inputs as I

from _gpu_common import lib, say, to_dev

pytestmark = pytest.mark.gpu


def _ic(plan, wl):
    x = np.zeros(plan.total)
    for i in range(len(wl.instances)):
        nd, off, _ = plan.info(i)
        for s, (terms, mults, add) in enumerate(wl.initial_condition(i, nd)):
            v = np.zeros(nd)
            for (amp, fac), mult in zip(terms, mults):
                pr = plan.project(i, amp, fac)
                v += pr * (1.0 + mult) if mult is not None else pr
            if add is not None:
                v += add
            x[off + s * nd : off + (s + 1) * nd] = v
    return x


@pytest.mark.parametrize("name,prec,tol,nmax", [
    ("schnakenberg_d2", "fp64", 1e-14, 5),
    ("gray_scott_batch", "fp32", 1e-13, 5),
])
def test_graph_replay_equals_eager_step(name, prec, tol, nmax):
    import torch

    sg = lib()
    wl = getattr(I, name)()
    say("graph replay", name, prec)
    plan = sg.Plan(wl.instances, prec)
    U0 = to_dev(_ic(plan, wl))
    _, ib = plan.workspace_size(wl.M, 1)
    ws = torch.empty(ib, dtype=torch.uint8, device="cuda")
    st = torch.zeros(len(wl.instances) * 2 * sg.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    F0 = torch.zeros_like(U0)
    plan.reaction(U0, F0, ws)
    steps = 3
    # eager reference: the state after 1, 2, 3 steps
    U, F = U0.clone(), F0.clone()
    ref = []
    for _ in range(steps):
        plan.iif2_step(wl.dt, wl.M, U, F, ws, newton_tol=tol, newton_max=nmax, stats=st)
        torch.cuda.synchronize()
        ref.append((U.cpu().numpy().copy(), F.cpu().numpy().copy()))
    # capture one step on a side stream (after one eager warm-up step there)
    U, F = U0.clone(), F0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.iif2_step(wl.dt, wl.M, U, F, ws, newton_tol=tol, newton_max=nmax, stats=st)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.iif2_step(wl.dt, wl.M, U, F, ws, newton_tol=tol, newton_max=nmax, stats=st)
    torch.cuda.synchronize()
    # replays from the initial state; eager work and a synchronisation between them
    U.copy_(U0)
    F.copy_(F0)
    torch.cuda.synchronize()
    scratch = torch.empty_like(U0)
    for n in range(steps):
        g.replay()
        torch.cuda.synchronize()
        plan.apply(U0 if prec == "fp64" else U0.float(), scratch if prec == "fp64" else scratch.float())
        torch.cuda.synchronize()
        Ug, Fg = U.cpu().numpy(), F.cpu().numpy()
        assert np.array_equal(Ug, ref[n][0]), f"replay {n + 1}: state differs from the eager step"
        assert np.array_equal(Fg, ref[n][1]), f"replay {n + 1}: F cache differs from the eager step"
    s = sg.stats_array(st)
    assert np.all(s["status"][: 2 * len(wl.instances)] == 0)
    del g
    plan.close()
