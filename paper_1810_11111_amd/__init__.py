"""Sparse-grid Krylov IIF discontinuous Galerkin on MI355X (gfx950).

The compute path lives in the HIP shared library built from ``csrc/`` and is
reached through :mod:`paper_1810_11111_amd.sgdg` (a thin ctypes binding over
the C ABI declared in ``include/sgdg.h``).  Importing this package does not
load the library; importing ``sgdg`` does and fails loudly if it is missing.
"""

__all__ = ["inputs"]
