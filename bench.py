#!/usr/bin/env python3
"""Benchmark: IIF2 steps of sparse-grid Krylov IIF DG on one MI355X.

Workload (default): the 2-species Schnakenberg system on the periodic unit
square, d=2, sparse level N=7, P2 (k=2), 5184 DOFs per species, IIF2 with
dt=0.05 and Krylov dimension M=30, initial data (a+b, b/(a+b)^2) plus seeded
uniform +-0.01 noise on every coefficient.  One step = one iif2_step call
(two Krylov exponentials, the implicit reaction stage) replayed from a
captured HIP graph; inputs are resident in HBM before timing starts.

Prints ONE JSON line with the IIF2 throughput in DOF-steps/s (FP64 path),
the FP32- and BF16-sweep variants with their L2 difference to the FP64
result, the roofline of the dominant kernel, the out-of-cache sweep, a
64-instance batched run (FP64 and FP32 sweeps), and the CPU oracle baseline
with the L2 error of each precision against the oracle after the same steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IIF2 DOF-steps/sec and operator-apply GB/s; mixed/batched vs FP64 at stated L2 err"
HBM_PEAK_GBS = 8000.0
NEWTON_TOL = 1e-14
NEWTON_MAX = 5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_ic(plan, wl):
    """Initial plan vector from the workload description (library projection)."""
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
            x[off + s * nd: off + (s + 1) * nd] = v
    return x


def dof_per_step(plan, wl):
    return sum(plan.info(i)[0] * inst.species for i, inst in enumerate(wl.instances))


def run_steps(sg, torch, wl, prec, U0, steps, warmup, graph=True, local=False):
    """Returns (seconds for `steps` steps, final U (numpy), stats).  local: the
    stage solved pointwise (iif2_step_local) instead of the Galerkin stage."""
    plan = sg.Plan(wl.instances, prec)
    Ud = torch.from_numpy(U0.copy()).cuda()
    F = torch.zeros_like(Ud)
    _, ib = plan.workspace_size(wl.M, 1)
    ws = torch.empty(ib, dtype=torch.uint8, device="cuda")
    st = torch.zeros(len(wl.instances) * 2 * sg.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    plan.reaction(Ud, F, ws)

    def step():
        if local:
            plan.iif2_step_local(wl.dt, wl.M, Ud, F, ws, stats=st)
        else:
            plan.iif2_step(wl.dt, wl.M, Ud, F, ws, newton_tol=NEWTON_TOL, newton_max=NEWTON_MAX, stats=st)

    torch.cuda.synchronize()
    g = None
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()  # first step eager (warm caches / code objects)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        done = 2  # one eager step and the captured step
    else:
        step()
        done = 1
    run = g.replay if graph else step
    for _ in range(max(0, warmup - done)):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    stats = sg.stats_array(st)
    U = Ud.cpu().numpy()
    del g
    plan.close()
    return secs, U, stats, done + max(0, warmup - done)


def run_steps_iif3(sg, torch, wl, U0, steps, warmup):
    """IIF3 (Sec. 3, eq. 3.6) on the workload: one IIF2 start-up step, then
    IIF3 steps replayed from a captured graph.  Returns (seconds, stats)."""
    plan = sg.Plan(wl.instances, "fp64")
    Ud = torch.from_numpy(U0.copy()).cuda()
    Fc = torch.zeros_like(Ud)
    _, ib = plan.workspace_size(wl.M, 1)
    ws = torch.empty(ib, dtype=torch.uint8, device="cuda")
    st = torch.zeros(len(wl.instances) * 2 * sg.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    plan.reaction(Ud, Fc, ws)
    Fp = Fc.clone()
    plan.iif2_step(wl.dt, wl.M, Ud, Fc, ws, newton_tol=NEWTON_TOL, newton_max=NEWTON_MAX, stats=st)

    def step():
        plan.iif3_step(wl.dt, wl.M, Ud, Fc, Fp, ws, newton_tol=NEWTON_TOL, newton_max=NEWTON_MAX, stats=st)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for _ in range(max(0, warmup - 2)):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    stats = sg.stats_array(st)
    del g
    plan.close()
    return secs, stats


def kernel_source_hash():
    """Hash of the sweep kernel sources and of the plan builder that lays out its
    chunks and task lists (traffic counters are only valid for this code)."""
    h = hashlib.sha256()
    for f in ("apply.hip", "kernels.h", "internal.h", "host_plan.cpp"):
        with open(os.path.join(ROOT, "paper_1810_11111_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_sweep(sg, torch, insts, prec, reps, seed=7):
    """Average duration of one sweep launch (sg_dg_apply, nrhs=1), measured with HIP
    events around a captured graph of `reps` back-to-back launches on the same stream."""
    from paper_1810_11111_amd import inputs as I

    plan = sg.Plan(insts, prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    x = torch.from_numpy(I.smooth_random(plan.total, seed, 1)[0]).to(dt).cuda()
    y = torch.empty_like(x)
    plan.apply(x, y)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            plan.apply(x, y)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    avg = e0.elapsed_time(e1) / 1e3 / reps
    elem = 8 if prec == "fp64" else 4
    total = plan.total
    del g
    plan.close()
    return avg, 2 * total * elem, total


def traffic_record(kernel, workload):
    """Measured HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(wl, budget_s=20.0):
    """The oracle (numpy/scipy FP64) on the same workload: as many steps as fit in
    the budget, from the oracle's own projection of the initial data.  Returns
    the record, that initial state and the oracle state after the steps run."""
    from oracle import iif, project
    from threadpoolctl import threadpool_info

    inst = wl.instances[0]
    prob = iif.Problem(inst.d, inst.N, inst.k, inst.D, inst.rx, wl.dt, wl.M)
    U0 = []
    for terms, mults, add in wl.initial_condition(0, prob.ndof):
        v = np.zeros(prob.ndof)
        for (amp, fac), mult in zip(terms, mults):
            pr = project.project_separable(inst.d, inst.N, inst.k, amp, fac)
            v += pr * (1.0 + mult) if mult is not None else pr
        U0.append(v + add if add is not None else v)
    U0 = np.array(U0)
    U = U0.copy()
    Fn = prob.F(U)
    t0 = time.perf_counter()
    n = 0
    while n < wl.steps and time.perf_counter() - t0 < budget_s:
        U, Fn, _ = iif.iif2_step(prob, U, Fn, tol=NEWTON_TOL)
        n += 1
    secs = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    rec = {"value": prob.ndof * inst.species * n / secs, "unit": "DOF-steps/s", "cores": int(threads),
           "kind": "oracle", "sample": f"first {n} of {wl.steps} IIF2 steps of the same workload ({secs:.1f} s)"}
    return rec, U0.ravel(), n, U.ravel()


def gpu_trajectory(sg, torch, wl, prec, U0, steps):
    """`steps` eager IIF2 steps of the library from U0 (untimed)."""
    plan = sg.Plan(wl.instances, prec)
    Ud = torch.from_numpy(U0.copy()).cuda()
    F = torch.zeros_like(Ud)
    _, ib = plan.workspace_size(wl.M, 1)
    ws = torch.empty(ib, dtype=torch.uint8, device="cuda")
    plan.reaction(Ud, F, ws)
    for _ in range(steps):
        plan.iif2_step(wl.dt, wl.M, Ud, F, ws, newton_tol=NEWTON_TOL, newton_max=NEWTON_MAX)
    torch.cuda.synchronize()
    U = Ud.cpu().numpy()
    plan.close()
    return U


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32/BF16 legs")
    ap.add_argument("--eager", action="store_true", help="launch steps eagerly instead of replaying a graph")
    ap.add_argument("--no-big", action="store_true", help="skip the out-of-cache sweep measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance Gray-Scott batch")
    ap.add_argument("--no-iif3", action="store_true", help="skip the IIF3 leg")
    ap.add_argument("--no-local", action="store_true", help="skip the local-stage variant")
    ap.add_argument("--batched-steps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (--gpus {args.gpus} requested); "
              "independent instances would shard one per GPU with no communication", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_11111_amd import inputs as I
    from paper_1810_11111_amd import sgdg as sg

    wl = I.schnakenberg_d2()
    plan0 = sg.Plan(wl.instances, "fp64")
    U0 = build_ic(plan0, wl)
    ndps = dof_per_step(plan0, wl)
    plan0.close()

    log(f"[bench] fp64: {args.steps} steps, warmup {args.warmup}")
    secs, U64, st64, _ = run_steps(sg, torch, wl, "fp64", U0, args.steps, args.warmup, graph=not args.eager)
    if np.any(st64["status"][: 2 * len(wl.instances)] != 0):
        log("[bench] warning: step status", st64)
    value = ndps * args.steps / secs
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "d": 2, "N": 7, "k": 2, "species": 2, "dof_per_species": ndps // 2,
                   "dt": wl.dt, "M": wl.M, "newton_tol": NEWTON_TOL, "newton_max": NEWTON_MAX,
                   "graph": not args.eager},
        "newton_iters_last_step": int(st64["newton_iters"][0]),
    }
    if not args.no_mixed:
        mixed = {}
        for prec in ("fp32", "bf16"):
            log(f"[bench] {prec}")
            s2, Up, stp, _ = run_steps(sg, torch, wl, prec, U0, args.steps, args.warmup, graph=not args.eager)
            rel = float(np.linalg.norm(Up - U64) / np.linalg.norm(U64))
            mixed[prec] = {"value": ndps * args.steps / s2, "ms_per_step": 1e3 * s2 / args.steps,
                           "rel_l2_vs_fp64": rel, "status_ok": bool(np.all(stp["status"][:2] == 0))}
        out["mixed"] = mixed
    if not args.no_local:
        log("[bench] local stage")
        sl, Ul, stl, _ = run_steps(sg, torch, wl, "fp64", U0, args.steps, args.warmup, graph=not args.eager,
                                   local=True)
        out["iif2_local_stage"] = {
            "value": ndps * args.steps / sl, "ms_per_step": 1e3 * sl / args.steps,
            "status_ok": bool(np.all(stl["status"][: 2 * len(wl.instances)] == 0)),
            "rel_l2_vs_galerkin_stage": float(np.linalg.norm(Ul - U64) / np.linalg.norm(U64)),
            "note": "variant: implicit stage solved pointwise at the Gauss points (local implicit property)"}
    if not args.no_iif3:
        log("[bench] iif3")
        s3, st3 = run_steps_iif3(sg, torch, wl, U0, args.steps, args.warmup)
        out["iif3"] = {"value": ndps * args.steps / s3, "ms_per_step": 1e3 * s3 / args.steps,
                       "status_ok": bool(np.all(st3["status"][: 2 * len(wl.instances)] == 0)),
                       "note": "same workload with IIF3 (eq. 3.6): two Krylov exponentials per step"}
    # roofline of the dominant kernel: the operator sweep (the same kernel the
    # step launches for every Krylov vector), timed live on the workload plan
    log("[bench] sweep timing")
    avg, nbytes, _ = time_sweep(sg, torch, wl.instances, "fp64", reps=100)
    achieved = nbytes / avg / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": traffic_record("apply_kernel_lds", wl.name),
                       "kernel": "apply_kernel_lds<2,2,PrecF64,true,void,1> (operator sweep, y = A x)",
                       "avg_us": avg * 1e6, "bytes_per_launch": nbytes,
                       "launches_per_step": wl.M * 1,
                       "note": "algorithmic bytes = read x + write y, 8 B each per DOF; the working set "
                               "(166 KB) is cache resident, so this launch is latency bound; traffic = "
                               "FETCH_SIZE + WRITE_SIZE per launch scaled by a 256 MiB copy (each XCD's L2 "
                               "fetches the staged operator tables once)"}
    if not args.no_big:
        log("[bench] out-of-cache sweep d=3 N=16 k=1")
        big = [I.Instance(3, 16, 1, [1.0], I.rx_zeros(1))]
        avg_b, nbytes_b, tot_b = time_sweep(sg, torch, big, "fp64", reps=10)
        out["apply_out_of_cache"] = {"workload": "sweep d=3 N=16 k=1 (24.6M DOF, 197 MB per FP64 vector)",
                                     "kernel": "apply_kernel<3,1,PrecF64,void> (global gathers)",
                                     "dof": tot_b, "avg_ms": avg_b * 1e3, "achieved_gbs": nbytes_b / avg_b / 1e9,
                                     "frac_of_peak": nbytes_b / avg_b / 1e9 / HBM_PEAK_GBS,
                                     "bytes_per_launch": nbytes_b,
                                     "traffic": traffic_record("apply_kernel", "sweep_d3_n16_k1")}
    if not args.no_batched:
        # 64 independent Gray-Scott instances (levels 5-8, k 1-2) in one plan: every
        # launch of the step covers all of them; FP64 and FP32 sweeps
        bw = I.gray_scott_batch()
        bplan = sg.Plan(bw.instances, "fp64")
        bU0 = build_ic(bplan, bw)
        bdofs = dof_per_step(bplan, bw)
        bplan.close()
        batched = {"workload": f"{bw.name} ({len(bw.instances)} instances, d=2, N 5-8, k 1-2, M={bw.M}, "
                               f"dt={bw.dt})", "dof_per_step": bdofs, "steps": args.batched_steps}
        ref = None
        for prec in ("fp64", "fp32"):
            log(f"[bench] batched {prec}")
            s2, Ub, stb, _ = run_steps(sg, torch, bw, prec, bU0, args.batched_steps, 3, graph=not args.eager)
            ent = {"value": bdofs * args.batched_steps / s2, "ms_per_step": 1e3 * s2 / args.batched_steps,
                   "status_ok": bool(np.all(stb["status"][: 2 * len(bw.instances)] == 0))}
            if ref is None:
                ref = Ub
            else:
                ent["rel_l2_vs_fp64"] = float(np.linalg.norm(Ub - ref) / np.linalg.norm(ref))
            batched[prec] = ent
        out["batched"] = batched
    if not args.no_cpu:
        log("[bench] cpu oracle")
        rec, U0o, n, Uo = cpu_baseline(wl)
        out["cpu_baseline"] = rec
        # the same steps on the GPU from the oracle's initial state: L2 error of
        # each precision against the FP64 oracle
        err = {"steps": n, "ic_rel_diff_library_vs_oracle": float(np.linalg.norm(U0 - U0o) / np.linalg.norm(U0o))}
        for prec in ("fp64", "fp32", "bf16"):
            Ug = gpu_trajectory(sg, torch, wl, prec, U0o, n)
            err[prec] = float(np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo))
        out["rel_l2_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
