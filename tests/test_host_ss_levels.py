"""Host logic of the fibre form of the sweep (no GPU).

build_ss_levels (csrc/host_operator.cpp) gives, for every level b, the 1D
SIPG operator of Sec. 2.1 (eq. 2.10) restricted to the piecewise polynomials
on the level-b cells, in their cell-Legendre basis.  Since the hierarchical
basis of levels 0..b is an orthonormal basis of the same space, the
hierarchical operator restricted to levels 0..b must equal Q^T Bs_b Q (Q: the
synthesis by the two-scale relation).  The check compiles the library's host
code with g++ and compares both for degrees 1..3, periodic and zero
Dirichlet boundaries, constant and variable k(x), N = 5 (every b = 0..5,
including the levels where a cell is its own periodic neighbour).  Bound:
1e-13 relative to the largest entry (measured 6e-16); a wrong block, a
transposed block or a missed periodic wrap gives O(1).
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_11111_amd", "csrc")


def test_single_scale_levels_match_hierarchical_operator(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path / "check_ss_levels")
    src = [os.path.join(ROOT, "tests", "host", "check_ss_levels.cpp"), os.path.join(CSRC, "host_operator.cpp"),
           os.path.join(CSRC, "host_basis.cpp")]
    subprocess.run([gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC, *src,
                    "-o", exe], check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=300).stdout
    m = re.search(r"worst relative ([0-9.eE+-]+)", out)
    assert m, out
    assert float(m.group(1)) < 1e-13, out
