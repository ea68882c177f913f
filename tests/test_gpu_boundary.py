"""Error behaviour of the C-ABI with a real plan (the contract of include/sgdg.h):
argument errors return SGDG_ERR_ARG before any device work and leave the
outputs untouched; a request outside the reaction transforms' range
((k+1) 2^N > 2048 per axis) returns SGDG_ERR_UNSUPPORTED while the sweep and
the Krylov exponential still serve the plan."""
import numpy as np
import pytest

from paper_1810_11111_amd import inputs as I

from _gpu_common import lib, say, to_dev

pytestmark = pytest.mark.gpu


def _status(fn, *a, **kw):
    sg = lib()
    try:
        fn(*a, **kw)
    except sg.SgdgError as e:
        return e.status
    return 0


def test_argument_errors_leave_outputs_untouched():
    import torch

    sg = lib()
    inst = I.Instance(2, 4, 1, [1.0, 0.5], I.rx_zeros(2))
    say("boundary errors d=2 N=4 k=1")
    plan = sg.Plan([inst], "fp64")
    M = 10
    kb, ib = plan.workspace_size(M, 1)
    x = to_dev(I.smooth_random(plan.total, 3, 1)[0])
    y = torch.full_like(x, 7.0)
    ws = torch.empty(ib, dtype=torch.uint8, device="cuda")
    small = torch.empty(kb - 1, dtype=torch.uint8, device="cuda")
    # M out of range, workspace too small, aliasing, non-finite h
    assert _status(plan.krylov_expv, 0.1, 0, x, y, ws) == 1
    assert _status(plan.krylov_expv, 0.1, 49, x, y, ws) == 1
    assert _status(plan.krylov_expv, 0.1, M, x, y, small) == 1
    assert _status(plan.krylov_expv, float("nan"), M, x, y, ws) == 1
    assert _status(plan.apply, x, x) == 1
    assert _status(plan.apply, x, y, nrhs=0) == 1
    assert _status(plan.reaction, x, x, ws) == 1
    U = x.clone()
    assert _status(plan.iif2_step, -0.1, M, U, y, ws) == 1
    assert _status(plan.iif2_step, 0.1, M, U, y, ws, newton_tol=-1.0) == 1
    assert _status(plan.iif3_step, 0.1, M, U, y, y, ws) == 1
    assert _status(plan.iif2_step, 0.1, M, U, U, ws) == 1  # U aliasing the F cache
    torch.cuda.synchronize()
    assert (y.cpu().numpy() == 7.0).all()
    assert np.array_equal(U.cpu().numpy(), x.cpu().numpy())
    # the plan still works afterwards
    plan.apply(x, y)
    torch.cuda.synchronize()
    assert np.isfinite(y.cpu().numpy()).all() and not (y.cpu().numpy() == 7.0).all()
    plan.close()


def test_reaction_range_is_unsupported_sweep_and_krylov_still_run():
    import torch

    sg = lib()
    inst = I.Instance(2, 11, 1, [1.0], I.rx_quadratic(-1.0))  # (k+1) 2^N = 4096 > 2048
    say("unsupported reaction range d=2 N=11 k=1")
    plan = sg.Plan([inst], "fp64")
    M = 8
    _, ib = plan.workspace_size(M, 1)
    ws = torch.empty(ib, dtype=torch.uint8, device="cuda")
    x = to_dev(0.1 * I.smooth_random(plan.total, 4, 1)[0])
    F = torch.full_like(x, 3.0)
    U = x.clone()
    assert _status(plan.reaction, x, F, ws) == 4
    assert _status(plan.iif2_step, 0.01, M, U, F, ws) == 4
    torch.cuda.synchronize()
    assert (F.cpu().numpy() == 3.0).all()
    y = torch.empty_like(x)
    plan.apply(x, y)
    w = torch.empty_like(x)
    st = torch.zeros(2 * sg.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    # h ||A||_inf = 1e-3: exp(hA) v = v + h A v + r with
    # ||r||_inf <= (h ||A||_inf)^2 / 2 * e^(h ||A||_inf) * ||v||_inf < 6e-7 ||v||_inf
    h = 1e-3 / plan.norm_inf(0, 0)
    plan.krylov_expv(h, M, x, w, ws, stats=st)
    torch.cuda.synchronize()
    s = sg.stats_array(st)
    assert s["status"][0] == 0 and np.isfinite(w.cpu().numpy()).all()
    xv, yv, wv = x.cpu().numpy(), y.cpu().numpy(), w.cpu().numpy()
    dev = np.abs(wv - xv - h * yv).max()
    assert dev <= 6e-7 * np.abs(xv).max(), dev
    plan.close()
