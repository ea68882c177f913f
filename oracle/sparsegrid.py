"""Sparse-grid index set and the canonical ordering of degrees of freedom.

Paper: Sec. 2.1, tensor-product wavelet spaces W_l (2.7), basis (2.8) and the
sparse space  V_N^k = sum over |l|_1 <= N of W_l  (2.9).  The paper states the
DOF count only asymptotically, O((k+1)^d 2^N N^(d-1)); the exact count used here
is the size of the index set itself, pinned against every DOF the tables print.

Canonical ordering (an interface shared with the HIP library, which builds its
own copy of it independently):

* level blocks l (multi-indices with |l|_1 <= N) sorted by |l|_1, then
  lexicographically in (l_1, ..., l_d);
* inside a block, a row-major d-dimensional tensor whose axis m has extent
  c(l_m)(k+1), c(0) = 1, c(l) = 2^(l-1), and index t_m = j_m (k+1) + p_m
  (cell j_m, 0-based degree / wavelet index p_m).
"""
from __future__ import annotations

import itertools

import numpy as np

from .basis import level_count, level_offset


def level_blocks(d: int, N: int):
    """All level multi-indices l in N_0^d with |l|_1 <= N, in canonical order."""
    blocks = [l for l in itertools.product(range(N + 1), repeat=d) if sum(l) <= N]
    blocks.sort(key=lambda l: (sum(l), l))
    return blocks


def dof_count(d: int, N: int, k: int) -> int:
    """Exact number of DOFs: (k+1)^d * sum_{|l|<=N} prod_m c(l_m)."""
    return (k + 1) ** d * sum(int(np.prod([level_count(lm) for lm in l])) for l in level_blocks(d, N))


def enumerate_dofs(d: int, N: int, k: int):
    """Per-DOF (level, cell, degree) arrays of shape (ndof, d) in canonical order,
    plus the 1D hierarchical index r_m = offset(l_m) + j_m (k+1) + p_m per axis."""
    lev, cell, deg = [], [], []
    for l in level_blocks(d, N):
        ranges = []
        for lm in l:
            ranges.append([(j, p) for j in range(level_count(lm)) for p in range(k + 1)])
        for combo in itertools.product(*ranges):
            lev.append(l)
            cell.append([c[0] for c in combo])
            deg.append([c[1] for c in combo])
    lev = np.array(lev, dtype=np.int64).reshape(-1, d)
    cell = np.array(cell, dtype=np.int64).reshape(-1, d)
    deg = np.array(deg, dtype=np.int64).reshape(-1, d)
    offs = np.array([level_offset(int(x), k) for x in range(N + 1)], dtype=np.int64)
    r1d = offs[lev] + cell * (k + 1) + deg
    return lev, cell, deg, r1d


def block_offsets(d: int, N: int, k: int):
    """(blocks, start offsets, sizes) of the level blocks in the canonical vector."""
    blocks = level_blocks(d, N)
    sizes = [int(np.prod([level_count(lm) * (k + 1) for lm in l])) for l in blocks]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return blocks, starts, np.array(sizes, dtype=np.int64)
