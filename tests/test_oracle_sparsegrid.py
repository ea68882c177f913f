"""Pins for the sparse index set (Sec. 2.1, eqs. 2.7-2.9) against the paper's DOF tables."""
import csv
import os

import numpy as np

from oracle import basis, sparsegrid


def _rows(golden_dir):
    with open(os.path.join(golden_dir, "dof_table.csv")) as fh:
        lines = [ln for ln in fh if not ln.startswith("#")]
    return list(csv.DictReader(lines))


def test_dof_counts_match_paper_tables(golden_dir):
    rows = _rows(golden_dir)
    assert len(rows) >= 30
    for r in rows:
        d, k, N, dof = int(r["d"]), int(r["k"]), int(r["N"]), int(r["dof"])
        if r["grid"] == "sparse":
            assert sparsegrid.dof_count(d, N, k) == dof, r
        else:
            # full tensor grid: ((k+1) 2^N)^d, i.e. the sparse set without the |l|_1 bound
            assert ((k + 1) * 2 ** N) ** d == dof, r


def test_enumeration_size_and_order():
    for d, N, k in [(2, 5, 1), (3, 4, 2), (4, 3, 1)]:
        lev, cell, deg, r1d = sparsegrid.enumerate_dofs(d, N, k)
        assert lev.shape[0] == sparsegrid.dof_count(d, N, k)
        assert np.all(lev.sum(axis=1) <= N)
        # every (l, j, p) appears once
        keys = {tuple(a) for a in np.concatenate([lev, cell, deg], axis=1)}
        assert len(keys) == lev.shape[0]
        blocks, starts, sizes = sparsegrid.block_offsets(d, N, k)
        assert starts[-1] + sizes[-1] == lev.shape[0]
        for b, s, n in zip(blocks, starts, sizes):
            assert np.all(lev[s : s + n] == np.array(b))
        # block order: by |l|_1 then lexicographic
        assert blocks == sorted(blocks, key=lambda l: (sum(l), l))
        # row-major tensor inside a block: last axis fastest
        b, s = blocks[-1], starts[-1]
        t = cell[s : s + 2] * (k + 1) + deg[s : s + 2]
        assert t[1, -1] == t[0, -1] + 1


def test_d1_sparse_equals_full():
    for N, k in [(5, 1), (4, 2)]:
        _, _, _, r1d = sparsegrid.enumerate_dofs(1, N, k)
        assert np.array_equal(r1d[:, 0], np.arange((k + 1) * 2 ** N))
        assert len(basis.hier_list_1d(N, k)) == r1d.shape[0]
