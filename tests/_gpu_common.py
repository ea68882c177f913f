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
