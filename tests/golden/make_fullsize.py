"""Write the full-size oracle states that the GPU parity tests compare with.

Calls only the CPU oracle (``oracle/``) and the seeded input descriptions
(``paper_1810_11111_amd/inputs.py``, which hold no method arithmetic).  Each
case takes the workload at its full size, projects its initial data with the
oracle, runs two IIF2 steps (Sec. 3, eq. 3.5; Krylov eqs. 3.7-3.8; the
implicit stage on F(U) = P f(R U) of Sec. 5) and stores

    U0      the projected initial coefficients, shape (rhs, species, ndof)
    U2      the state after the two steps, same shape
    iters   implicit-stage corrections per (rhs, step)
    m       Krylov dimension per (rhs, step, species)
    anorm   ||A_s||_inf per species
    vnorm   ||U^n + dt/2 F(U^n)|| per (rhs, step, species) (the Krylov input norm)

in ``fullsize_<case>.npz`` next to this file.

Cases (name: workload, full sizes):
    c3        allen_cahn_d3   d=3 N=7 k=1, variable k_ii          (13,568 DOF)
    c5        quadratic_d4    d=4 N=6 k=1, amplitude 0.5          (24,320 DOF)
    c5_rhs0   quadratic_d4    batch of 16, right-hand side 0
    c5_rhs15  quadratic_d4    batch of 16, right-hand side 15
    c4        gray_scott_batch, all 64 instances (N 5-8, k 1-2)   (462,592 DOF)

Usage:  python tests/golden/make_fullsize.py CASE [CASE ...]
The d=4 cases take about an hour each on 8 cores (the oracle forms the
268M-point field of every R and P pass); c3 takes minutes, c4 about a minute.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import iif, project  # noqa: E402
from paper_1810_11111_amd import inputs as I  # noqa: E402

STEPS = 2
NEWTON_TOL = {"c3": 1e-14, "c5": 1e-14, "c5_rhs0": 1e-14, "c5_rhs15": 1e-14, "c4": 1e-13}


def kappas(inst):
    if inst.kdiag is None:
        return None
    a0, a1, f = inst.kdiag
    return [lambda x, a0=a0, a1=a1, f=f: a0 + a1 * np.sin(2 * np.pi * f * x)] * inst.d


def oracle_ic(wl, i, inst):
    from oracle.sparsegrid import dof_count

    nd = dof_count(inst.d, inst.N, inst.k)
    out = []
    for terms, mults, add in wl.initial_condition(i, nd):
        v = np.zeros(nd)
        for (amp, fac), mult in zip(terms, mults):
            pr = project.project_separable(inst.d, inst.N, inst.k, amp, fac)
            v += pr * (1.0 + mult) if mult is not None else pr
        if add is not None:
            v += add
        out.append(v)
    return np.array(out)


def run_instance(wl, i, inst, tol, log):
    prob = iif.Problem(inst.d, inst.N, inst.k, inst.D, inst.rx, wl.dt, wl.M, kappas=kappas(inst))
    U0 = oracle_ic(wl, i, inst)
    U = U0.copy()
    Fn = prob.F(U)
    iters, ms, vn = [], [], []
    for n in range(STEPS):
        v = U + 0.5 * prob.dt * Fn
        vn.append([float(np.linalg.norm(v[s])) for s in range(prob.S)])
        U, Fn, info = iif.iif2_step(prob, U, Fn, tol=tol)
        assert info["converged"], (i, n, info["residual"])
        iters.append(info["iters"])
        ms.append([kk["m"] for kk in info["krylov"]])
        log(f"  instance {i} step {n + 1}: {info['iters']} corrections, m {ms[-1]}, |G| {info['residual']:.2e}")
    return U0, U, iters, ms, vn, prob.anorm


def make(case):
    t0 = time.time()

    def log(msg):
        print(f"[{case} {time.time() - t0:7.1f}s] {msg}", flush=True)

    tol = NEWTON_TOL[case]
    if case == "c3":
        wl, which = I.allen_cahn_d3(), [0]
    elif case == "c5":
        wl, which = I.quadratic_d4(), [0]
    elif case.startswith("c5_rhs"):
        wl, which = I.quadratic_d4(nrhs=16), [int(case[len("c5_rhs"):])]
    elif case == "c4":
        wl = I.gray_scott_batch()
        which = list(range(len(wl.instances)))
    else:
        raise SystemExit(f"unknown case {case}")
    res = {"U0": [], "U2": [], "iters": [], "m": [], "vnorm": [], "anorm": []}
    for i in which:
        U0, U2, iters, ms, vn, an = run_instance(wl, i, wl.instances[i], tol, log)
        res["U0"].append(U0.ravel())
        res["U2"].append(U2.ravel())
        res["iters"].append(iters)
        res["m"].append(ms)
        res["vnorm"].append(vn)
        res["anorm"].append(an)
    out = os.path.join(HERE, f"fullsize_{case}.npz")
    if case == "c4":  # instances of uneven size: concatenated in instance order
        np.savez_compressed(out, U0=np.concatenate(res["U0"]), U2=np.concatenate(res["U2"]),
                            iters=np.array(res["iters"]), m=np.array(res["m"]), vnorm=np.array(res["vnorm"]),
                            anorm=np.array(res["anorm"]), instances=np.array(which), steps=STEPS,
                            newton_tol=tol)
    else:
        np.savez_compressed(out, U0=np.array(res["U0"]), U2=np.array(res["U2"]), iters=np.array(res["iters"]),
                            m=np.array(res["m"]), vnorm=np.array(res["vnorm"]), anorm=np.array(res["anorm"]),
                            instances=np.array(which), steps=STEPS, newton_tol=tol)
    log(f"wrote {out}")


if __name__ == "__main__":
    for c in sys.argv[1:]:
        make(c)
