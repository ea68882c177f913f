"""Launch-shape autotuning of the last-axis reaction kernels (sg_dg_tune,
sg_dg_line_shape).

The last axis of F(U) = P f(R U) (Sec. 5, applied axis by axis) runs as tiles
of whole lines; a shape (lines per tile, workgroups per compute unit, and
which of two register budgets the kernel is built with) only decides which
workgroup computes which line and how the compiler keeps its values.  So a
tuned plan, and plans forced to the extreme shapes, must give the default
plan's F and IIF2 steps (Sec. 3, eq. 3.5) bit for bit.
"""
import os

import numpy as np
import pytest

from paper_1810_11111_amd import inputs as I

from _gpu_common import lib, say, to_dev

pytestmark = pytest.mark.gpu


def _ws(plan, M, nrhs):
    import torch

    _, ib = plan.workspace_size(M, nrhs)
    return torch.empty(ib, dtype=torch.uint8, device="cuda")


def _run(plan, U0, nrhs, dt, M, steps=2):
    """F(U0), then `steps` IIF2 steps (F pass, residual and correction passes)."""
    import torch

    U = to_dev(np.ascontiguousarray(U0.reshape(nrhs, -1)))
    F = torch.zeros_like(U)
    ws = _ws(plan, M, nrhs)
    plan.reaction(U, F, ws, nrhs=nrhs)
    torch.cuda.synchronize()
    F0 = F.cpu().numpy().copy()
    for _ in range(steps):
        plan.iif2_step(dt, M, U, F, ws, newton_tol=1e-14, newton_max=8, nrhs=nrhs)
    torch.cuda.synchronize()
    return F0, U.cpu().numpy(), F.cpu().numpy()


def _cases():
    return {
        "quadratic_d4_n4_rhs3": (I.quadratic_d4(N=4).instances, 3, 0.005, 20),
        "gray_scott_8": (I.gray_scott_batch(ninst=8).instances, 1, 1.0, 10),
    }


@pytest.mark.parametrize("name", ["quadratic_d4_n4_rhs3", "gray_scott_8"])
def test_tuned_and_forced_shapes_match_default(name):
    sg = lib()
    insts, nrhs, dt, M = _cases()[name]
    say("tune", name)
    ref_plan = sg.Plan(insts, "fp64")
    total = ref_plan.total
    # near the homogeneous states: 0.5 (u' = -u^2), (1, 0) for Gray-Scott, with 1% noise
    U0 = 0.01 * I.smooth_random(total * nrhs, 41, 1)[0].reshape(nrhs, total)
    for i, inst in enumerate(insts):
        nd, off, _ = ref_plan.info(i)
        U0[:, off] += 0.5 if inst.species == 1 else 1.0  # the constant mode of species 0
    ref = _run(ref_plan, U0, nrhs, dt, M)
    ref_plan.close()

    tuned = sg.Plan(insts, "fp64")
    rep = tuned.tune(_ws(tuned, 1, nrhs), nrhs=nrhs)
    assert len(rep) >= 1
    for r in rep:
        for i in range(2):
            assert 1 <= r["rounds"][i] <= 64 and 1 <= r["wg_per_cu"][i] <= 64 and r["waves"][i] in (0, 3)
            assert r["ms_best"][i] <= r["ms_default"][i]
    got = _run(tuned, U0, nrhs, dt, M)
    for a, b in zip(got, ref):
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b)
    # a second plan of the same shape is served from the process cache
    again = sg.Plan(insts, "fp64")
    rep2 = again.tune(_ws(again, 1, nrhs), nrhs=nrhs)
    assert all(r["from_cache"] == [1, 1] for r in rep2)
    assert [(r["rounds"], r["wg_per_cu"], r["waves"]) for r in rep2] == [
        (r["rounds"], r["wg_per_cu"], r["waves"]) for r in rep]
    again.close()
    tuned.close()

    for rounds, wgcu, waves in ((1, 1, 0), (64, 64, 3), (3, 5, 0), (2, 16, 3)):
        forced = sg.Plan(insts, "fp64")
        for r in rep:
            for nin in (1, 2):
                forced.line_shape(r["class"], nin, rounds, wgcu, waves)
        got = _run(forced, U0, nrhs, dt, M)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (rounds, wgcu, waves)
        forced.close()


def test_tune_cache_file(tmp_path):
    """Choices written to the SGDG_TUNE_CACHE file by one process are read by
    another (a fresh interpreter), which then sets them without timing."""
    import json
    import subprocess
    import sys

    from _gpu_common import ROOT

    path = tmp_path / "tune.txt"
    prog = (
        "import sys, torch; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "from paper_1810_11111_amd import sgdg as sg, inputs as I\n"
        "p = sg.Plan(I.quadratic_d4(N=3).instances, 'fp64'); _, ib = p.workspace_size(1, 2)\n"
        "ws = torch.empty(ib, dtype=torch.uint8, device='cuda')\n"
        "r = p.tune(ws, nrhs=2); import json\n"
        "print(json.dumps({'cache': [c['from_cache'] for c in r],"
        " 'shapes': [c['rounds'] + c['wg_per_cu'] + c['waves'] for c in r]}))\n"
    ) % (ROOT, os.path.join(ROOT, "tests"))
    env = dict(os.environ, SGDG_TUNE_CACHE=str(path))
    say("tune cache file")
    first = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=240)
    assert first.returncode == 0, first.stderr[-2000:]
    assert path.exists() and len(path.read_text().splitlines()) >= 2
    second = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=240)
    assert second.returncode == 0, second.stderr[-2000:]
    f1 = json.loads(first.stdout.strip().splitlines()[-1])
    f2 = json.loads(second.stdout.strip().splitlines()[-1])
    assert all(c == [0, 0] for c in f1["cache"]) and all(c == [1, 1] for c in f2["cache"])
    assert f1["shapes"] == f2["shapes"]
    # lines of the older ten-field form (no register budget) read as waves 0
    lines = path.read_text().splitlines()
    path.write_text("".join(" ".join(ln.split()[:10]) + "\n" for ln in lines))
    third = subprocess.run([sys.executable, "-c", prog], env=env, capture_output=True, text=True, timeout=240)
    assert third.returncode == 0, third.stderr[-2000:]
    f3 = json.loads(third.stdout.strip().splitlines()[-1])
    assert all(c == [1, 1] for c in f3["cache"])
    assert all(s[:4] == t[:4] and s[4:] == [0, 0] for s, t in zip(f3["shapes"], f1["shapes"]))


def test_line_shape_argument_errors():
    sg = lib()
    plan = sg.Plan(I.quadratic_d4(N=3).instances, "fp64")
    with pytest.raises(sg.SgdgError):
        plan.line_shape(0, 3, 1, 1)
    with pytest.raises(sg.SgdgError):
        plan.line_shape(0, 1, 0, 1)
    with pytest.raises(sg.SgdgError):
        plan.line_shape(0, 1, 1, 65)
    with pytest.raises(sg.SgdgError):
        plan.line_shape(99, 1, 1, 1)
    with pytest.raises(sg.SgdgError):
        plan.line_shape(0, 1, 1, 1, waves=2)
    plan.close()
