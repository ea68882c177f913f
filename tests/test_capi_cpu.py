"""The C-ABI library loads, exports every symbol of include/sgdg.h, and rejects bad
arguments on the host before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from _gpu_common import ROOT, lib


def _declared():
    with open(os.path.join(ROOT, "include", "sgdg.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^(?:sgdg_status|const char\*)\s+(\w+)\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    sg = lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(sg._lib, n), n
    assert set(names) == set(sg.EXPORTED)


def test_argument_errors_return_before_device_work():
    sg = lib()
    L = sg._lib
    h = C.c_void_p()
    assert L.sg_dg_build(None, 1, 0, C.byref(h)) == 1
    d = sg.Desc()
    d.d, d.n, d.k, d.nspecies, d.D[0] = 7, 3, 1, 1, 1.0
    assert L.sg_dg_build(C.byref(d), 1, 0, C.byref(h)) == 1
    assert b"d must be in 1..6" in L.sgdg_last_error()
    d.d, d.k = 2, 0
    assert L.sg_dg_build(C.byref(d), 1, 0, C.byref(h)) == 1
    d.k, d.nspecies = 1, 3
    assert L.sg_dg_build(C.byref(d), 1, 0, C.byref(h)) == 1
    d.nspecies, d.D[0] = 1, -1.0
    assert L.sg_dg_build(C.byref(d), 1, 0, C.byref(h)) == 1
    d.D[0] = 1.0
    assert L.sg_dg_build(C.byref(d), 1, 9, C.byref(h)) == 1
    kd = (sg.Kdiag * 2)(sg.Kdiag(1.0, 1.5, 1.0, 0.0), sg.Kdiag(1.0, 0.0, 0.0, 0.0))
    d.kdiag = C.cast(kd, C.POINTER(sg.Kdiag))
    assert L.sg_dg_build(C.byref(d), 1, 0, C.byref(h)) == 1
    assert h.value is None
    # null plans everywhere
    n = C.c_int64()
    assert L.sg_dg_info(None, 0, C.byref(n), None, None) == 1
    assert L.sg_dg_total(None, C.byref(n)) == 1
    assert L.sg_dg_apply(None, 1, None, None, None) == 1
    assert L.sg_dg_sweep_form(None, 2) == 1
    assert L.krylov_expv(None, 1, 0.1, 10, None, None, None, 0, None, None) in (1, 4)
    assert L.iif2_step(None, 1, 0.1, 10, None, None, None, 1e-14, 5, None, 0, None, None) in (1, 4)
    assert L.iif3_step(None, 1, 0.1, 10, None, None, None, None, 1e-14, 5, None, 0, None, None) in (1, 4)
    assert L.rk_step(None, 1, 0.1, 2, None, None, 0, None) in (1, 4)
    assert L.iif2_step_local(None, 1, 0.1, 10, None, None, None, None, 0, None, None) in (1, 4)
    assert L.sg_dg_tune(None, 1, None, 0, None, None) == 1
    assert L.sg_dg_line_shape(None, 0, 1, 1, 1, 0) == 1
    assert L.sg_dg_destroy(None) == 1


def test_binding_refuses_to_load_without_library(tmp_path, monkeypatch):
    """The product path has no fallback: a missing library is an ImportError."""
    import importlib.util

    src = os.path.join(ROOT, "paper_1810_11111_amd", "sgdg.py")
    dst = tmp_path / "sgdg.py"
    dst.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("sgdg_copy", dst)
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)
