"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*args):
    """Name the case on stdout before each GPU step (flushed)."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def lib():
    """Load the HIP binding, building the library first if nothing is built."""
    so = os.path.join(ROOT, "paper_1810_11111_amd", "libsgdg.so")
    if not os.path.exists(so):
        from paper_1810_11111_amd import build

        build.build()
    from paper_1810_11111_amd import sgdg

    return sgdg


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def bf16_bits(a):
    """float64 array -> bfloat16 bit patterns (uint16, round to nearest even) via torch."""
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16), t.to(torch.float64).numpy()


def note(label, err, tol, scale=None):
    """Print a parity margin: the error, its tolerance, their ratio and (given
    the norm of the input) the error relative to that norm, so that a run's log
    shows how close each case runs to its bound."""
    rel = "" if scale is None else f" rel {err / max(scale, 1e-300):.3e}"
    print(f"[parity] {label}: err {err:.3e} tol {tol:.3e} ratio {err / max(tol, 1e-300):.4f}{rel}", flush=True)


# FP64 parity bound per Krylov exponential (and per IIF step), relative to the
# norm of its input: 1e-12, except for the stiff Schnakenberg v species
# (h ||A||_inf = 6.5e5, the stiffest of every workload), where it is five
# times the oracle's own spread under a reordering of its sums (at most 6e-13,
# pinned by tests/test_oracle_noise_floor.py).
FP64_BOUND = 1e-12
FP64_STIFF_BOUND = 3e-12
STIFF_H_ANORM = 1e5


def fp64_bound(h, anorm):
    return FP64_STIFF_BOUND if h * anorm > STIFF_H_ANORM else FP64_BOUND
