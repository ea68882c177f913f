"""iif2_step_noalloc (the fixed-scratch form of iif2_step, Sec. 3 eq. 3.5) through
the C-ABI gives the same result as iif2_step with a caller workspace: two calls
in a row on the shared device scratch, the second with a smaller input, each
equal bit for bit to iif2_step (the same kernels on the same inputs)."""
import ctypes as C

import numpy as np
import pytest

from paper_1810_11111_amd import inputs as I

from _gpu_common import lib, say, to_dev

pytestmark = pytest.mark.gpu


def _ic(plan, wl, nrhs):
    x = np.zeros((nrhs, plan.total))
    for r in range(nrhs):
        nd, off, _ = plan.info(0)
        for s, (terms, mults, add) in enumerate(wl.initial_condition(0, nd)):
            v = sum(plan.project(0, a, f) for a, f in terms)
            x[r, off + s * nd: off + (s + 1) * nd] = v + (add if add is not None else 0.0) * (1.0 + 0.1 * r)
    return x


def _pair(sg, wl, nrhs, steps=2):
    """(U after `steps` steps of iif2_step, the same with iif2_step_noalloc)."""
    import torch

    plan = sg.Plan(wl.instances, "fp64")
    x = _ic(plan, wl, nrhs)
    _, ib = plan.workspace_size(wl.M, nrhs)
    out = []
    for noalloc in (False, True):
        U = to_dev(x.copy())
        F = torch.zeros_like(U)
        ws = torch.empty(ib, dtype=torch.uint8, device="cuda")
        st = torch.zeros(nrhs * 2 * sg.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        plan.reaction(U, F, ws, nrhs=nrhs)
        for _ in range(steps):
            if noalloc:
                # straight through the C-ABI: no workspace argument
                rc = sg._lib.iif2_step_noalloc(plan._h, nrhs, float(wl.dt), wl.M, C.c_void_p(U.data_ptr()),
                                               C.c_void_p(F.data_ptr()), None, 1e-14, 12, C.c_void_p(st.data_ptr()),
                                               C.c_void_p(torch.cuda.current_stream().cuda_stream))
                assert rc == 0, sg._lib.sgdg_last_error()
            else:
                plan.iif2_step(wl.dt, wl.M, U, F, ws, newton_tol=1e-14, newton_max=12, stats=st, nrhs=nrhs)
        torch.cuda.synchronize()
        assert np.all(sg.stats_array(st)["status"] == 0)
        out.append(U.cpu().numpy())
    plan.close()
    return out


def test_noalloc_matches_workspace_form_twice():
    sg = lib()
    say("iif2_step_noalloc: Schnakenberg N=5 k=2, 2 right-hand sides")
    a, b = _pair(sg, I.schnakenberg_d2(N=5, k=2), nrhs=2)
    assert np.array_equal(a, b)
    say("iif2_step_noalloc: Schnakenberg N=4 k=1, 1 right-hand side (smaller)")
    a, b = _pair(sg, I.schnakenberg_d2(N=4, k=1), nrhs=1)
    assert np.array_equal(a, b)


def test_noalloc_rejects_plans_beyond_the_scratch():
    import torch

    sg = lib()
    wl = I.quadratic_d4()  # the d=4 N=6 workspace is several GB
    say("iif2_step_noalloc: size refusal d=4 N=6")
    plan = sg.Plan(wl.instances, "fp64")
    U = torch.zeros(plan.total, dtype=torch.float64, device="cuda")
    F = torch.zeros_like(U)
    rc = sg._lib.iif2_step_noalloc(plan._h, 1, 0.005, 40, C.c_void_p(U.data_ptr()), C.c_void_p(F.data_ptr()), None,
                                   1e-14, 5, None, None)
    assert rc == 4 and b"fixed device scratch" in sg._lib.sgdg_last_error()
    plan.close()
