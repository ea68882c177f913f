"""Launch driver for hardware-counter runs of the operator sweep.

Runs `--reps` eager sg_dg_apply launches (nrhs=1, FP64) on a named workload,
then one device-to-device copy of `--copy-mib` MiB.  The copy moves a known
number of bytes, so the FETCH_SIZE / WRITE_SIZE that a counter pass reports
for it calibrates the counters read for the sweep in the same run.

    python -m paper_1810_11111_amd.profile_sweep --workload schnakenberg_d2 --reps 20
"""
from __future__ import annotations

import argparse
import sys

import torch

from . import inputs as I
from . import sgdg as sg

WORKLOADS = {
    "schnakenberg_d2": lambda: I.schnakenberg_d2().instances,
    "sweep_d3_n16_k1": lambda: [I.Instance(3, 16, 1, [1.0], I.rx_zeros(1))],
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="schnakenberg_d2")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=256)
    args = ap.parse_args()
    insts = WORKLOADS[args.workload]()
    plan = sg.Plan(insts, "fp64")
    x = torch.from_numpy(I.smooth_random(plan.total, 7, 1)[0]).cuda()
    y = torch.empty_like(x)
    for _ in range(args.reps):
        plan.apply(x, y)
    torch.cuda.synchronize()
    n = args.copy_mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"[profile_sweep] {args.workload}: {args.reps} sweeps of {plan.total} DOF "
          f"({16 * plan.total} algorithmic bytes each); copy of {n * 8} bytes", flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
