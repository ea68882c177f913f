"""ctypes binding of the C ABI in include/sgdg.h (argument marshalling only).

Every computation runs in libsgdg.so (HIP kernels for gfx950, host plan
builder).  Device buffers are torch CUDA tensors; the binding passes their
data pointers and the current torch stream.  Importing this module without a
built library raises ImportError -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  -- must load first: its HIP runtime is the one libsgdg binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgdg.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1810_11111_amd.build` "
        "(the HIP library is the only implementation)"
    )
_lib = C.CDLL(LIB_PATH)

FP64, FP32_SWEEP, BF16_SWEEP = 0, 1, 2
PREC = {"fp64": FP64, "fp32": FP32_SWEEP, "bf16": BF16_SWEEP}
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_ALLOC", 3: "ERR_HIP", 4: "ERR_UNSUPPORTED", 5: "ERR_NOCONV", 6: "ERR_NONFINITE"}


class Kdiag(C.Structure):
    _fields_ = [("a0", C.c_double), ("a1", C.c_double), ("freq", C.c_double), ("phase", C.c_double)]


class Desc(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("nspecies", C.c_int32),
        ("sigma", C.c_double), ("D", C.c_double * 2), ("kdiag", C.POINTER(Kdiag)),
        ("rx", C.c_double * 32), ("bc", C.c_int32), ("pad", C.c_int32),
    ]


class Factor1D(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("a", C.c_double), ("b", C.c_double)]


TUNE_MAXCLASS = 16


class TuneReport(C.Structure):
    _fields_ = [("nclass", C.c_int32), ("k", C.c_int32 * TUNE_MAXCLASS), ("n", C.c_int32 * TUNE_MAXCLASS),
                ("nspecies", C.c_int32 * TUNE_MAXCLASS), ("cls", C.c_int32 * TUNE_MAXCLASS),
                ("rounds", (C.c_int32 * 2) * TUNE_MAXCLASS), ("wgcu", (C.c_int32 * 2) * TUNE_MAXCLASS),
                ("waves", (C.c_int32 * 2) * TUNE_MAXCLASS),
                ("ms_default", (C.c_float * 2) * TUNE_MAXCLASS), ("ms_best", (C.c_float * 2) * TUNE_MAXCLASS),
                ("from_cache", (C.c_int32 * 2) * TUNE_MAXCLASS)]


class Stats(C.Structure):
    _fields_ = [("krylov_m", C.c_int32), ("newton_iters", C.c_int32), ("h_next", C.c_double),
                ("residual", C.c_double), ("status", C.c_int32), ("pad", C.c_int32)]


STATS_DTYPE = np.dtype([("krylov_m", "<i4"), ("newton_iters", "<i4"), ("h_next", "<f8"),
                        ("residual", "<f8"), ("status", "<i4"), ("pad", "<i4")])
assert STATS_DTYPE.itemsize == C.sizeof(Stats)

_vp, _i32, _i64, _f64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
_sigs = {
    "sgdg_last_error": ([], C.c_char_p),
    "sg_dg_build": ([C.POINTER(Desc), _i32, _i32, C.POINTER(_vp)], C.c_int),
    "sg_dg_destroy": ([_vp], C.c_int),
    "sg_dg_info": ([_vp, _i32, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)], C.c_int),
    "sg_dg_total": ([_vp, C.POINTER(_i64)], C.c_int),
    "sg_dg_workspace_size": ([_vp, _i32, _i32, C.POINTER(_sz), C.POINTER(_sz)], C.c_int),
    "sg_dg_layout": ([_vp, _i32, _vp, _vp, _vp], C.c_int),
    "sg_dg_project": ([_vp, _i32, _f64, C.POINTER(Factor1D), _vp], C.c_int),
    "sg_dg_norm_inf": ([_vp, _i32, _i32, C.POINTER(_f64)], C.c_int),
    "sg_dg_apply": ([_vp, _i32, _vp, _vp, _vp], C.c_int),
    "sg_dg_sweep_form": ([_vp, _i32], C.c_int),
    "krylov_expv": ([_vp, _i32, _f64, _i32, _vp, _vp, _vp, _sz, _vp, _vp], C.c_int),
    "sgdg_reaction": ([_vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp], C.c_int),
    "sgdg_reaction_timed": ([_vp, _i32, _vp, _vp, _vp, _sz, _vp, _vp, C.POINTER(_i32), _vp], C.c_int),
    "iif2_step": ([_vp, _i32, _f64, _i32, _vp, _vp, _vp, _f64, _i32, _vp, _sz, _vp, _vp], C.c_int),
    "iif2_step_noalloc": ([_vp, _i32, _f64, _i32, _vp, _vp, _vp, _f64, _i32, _vp, _vp], C.c_int),
    "iif3_step": ([_vp, _i32, _f64, _i32, _vp, _vp, _vp, _vp, _f64, _i32, _vp, _sz, _vp, _vp], C.c_int),
    "rk_step": ([_vp, _i32, _f64, _i32, _vp, _vp, _sz, _vp], C.c_int),
    "iif2_step_local": ([_vp, _i32, _f64, _i32, _vp, _vp, _vp, _vp, _sz, _vp, _vp], C.c_int),
    "sg_dg_tune": ([_vp, _i32, _vp, _sz, C.POINTER(TuneReport), _vp], C.c_int),
    "sg_dg_line_shape": ([_vp, _i32, _i32, _i32, _i32, _i32], C.c_int),
}
EXPORTED = sorted(_sigs)
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class SgdgError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.sgdg_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st, where):
    if st != 0:
        raise SgdgError(st, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream)
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_desc(inst):
    """sgdg_desc from an inputs.Instance."""
    d = Desc()
    d.d, d.n, d.k, d.nspecies = inst.d, inst.N, inst.k, inst.species
    d.sigma = 20.0
    for s, v in enumerate(inst.D):
        d.D[s] = v
    rx = np.zeros((2, 4, 4))
    rx[: inst.species] = inst.rx
    for i, v in enumerate(rx.ravel()):
        d.rx[i] = float(v)
    d.kdiag = None
    d.bc = int(getattr(inst, "bc", 0))
    return d


def factor(desc):
    f = Factor1D()
    if desc[0] == "cos":
        f.kind, f.a, f.b = 0, float(desc[1]), float(desc[2])
    elif desc[0] == "box":
        f.kind, f.a, f.b = 1, float(desc[1]), float(desc[2])
    else:
        raise ValueError(desc)
    return f


class Plan:
    """A built plan (owns the device tables; freed by close() or on collection)."""

    def __init__(self, instances, prec="fp64"):
        self.instances = list(instances)
        n = len(self.instances)
        descs = (Desc * n)()
        self._kd = []
        for i, inst in enumerate(self.instances):
            descs[i] = make_desc(inst)
            if inst.kdiag is not None:
                a0, a1, f = inst.kdiag
                kd = (Kdiag * inst.d)(*[Kdiag(a0, a1, f, 0.0) for _ in range(inst.d)])
                self._kd.append(kd)
                descs[i].kdiag = C.cast(kd, C.POINTER(Kdiag))
        self.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        h = C.c_void_p()
        _check(_lib.sg_dg_build(descs, n, self.prec, C.byref(h)), "sg_dg_build")
        self._h = h
        tot = _i64()
        _check(_lib.sg_dg_total(self._h, C.byref(tot)), "sg_dg_total")
        self.total = tot.value
        self.d = self.instances[0].d

    def close(self):
        if getattr(self, "_h", None):
            _lib.sg_dg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- host queries -------------------------------------------------
    def info(self, inst=0):
        nd, off, npt = _i64(), _i64(), _i64()
        _check(_lib.sg_dg_info(self._h, inst, C.byref(nd), C.byref(off), C.byref(npt)), "sg_dg_info")
        return nd.value, off.value, npt.value

    def workspace_size(self, M, nrhs=1):
        a, b = _sz(), _sz()
        _check(_lib.sg_dg_workspace_size(self._h, M, nrhs, C.byref(a), C.byref(b)), "sg_dg_workspace_size")
        return a.value, b.value

    def layout(self, inst=0):
        nd = self.info(inst)[0]
        lev = np.zeros((nd, self.d), np.int32)
        cell = np.zeros((nd, self.d), np.int32)
        p = np.zeros((nd, self.d), np.int32)
        _check(_lib.sg_dg_layout(self._h, inst, lev.ctypes.data, cell.ctypes.data, p.ctypes.data), "sg_dg_layout")
        return lev, cell, p

    def project(self, inst, amp, factors):
        nd = self.info(inst)[0]
        out = np.zeros(nd, np.float64)
        fs = (Factor1D * self.d)(*[factor(f) for f in factors])
        _check(_lib.sg_dg_project(self._h, inst, float(amp), fs, out.ctypes.data), "sg_dg_project")
        return out

    def norm_inf(self, inst=0, species=0):
        v = _f64()
        _check(_lib.sg_dg_norm_inf(self._h, inst, species, C.byref(v)), "sg_dg_norm_inf")
        return v.value

    # ---- device calls ---------------------------------------------------
    def apply(self, x, y, nrhs=1, stream=None):
        _check(_lib.sg_dg_apply(self._h, nrhs, _ptr(x), _ptr(y), _stream(stream)), "sg_dg_apply")

    def sweep_form(self, form):
        """0 automatic, 1 chunked gather, 2 fibre form (FP64 only), 3 fibre form with every fibre split (testing)."""
        _check(_lib.sg_dg_sweep_form(self._h, form), "sg_dg_sweep_form")

    def krylov_expv(self, h, M, v, w, workspace, stats=None, nrhs=1, stream=None):
        _check(_lib.krylov_expv(self._h, nrhs, float(h), M, _ptr(v), _ptr(w), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _ptr(stats), _stream(stream)),
               "krylov_expv")

    def reaction(self, U, F, workspace, nrhs=1, stream=None, source=None):
        _check(_lib.sgdg_reaction(self._h, nrhs, _ptr(U), _ptr(F), _ptr(source), _ptr(workspace),
                                  workspace.numel() * workspace.element_size(), _stream(stream)), "sgdg_reaction")

    def reaction_timed(self, U, F, workspace, nrhs=1, stream=None, cap=64):
        """One reaction pass with per-launch HIP-event timing; returns [(kind, ms), ...]."""
        ms = (C.c_float * cap)()
        kind = (C.c_int32 * cap)()
        n = _i32(cap)
        _check(_lib.sgdg_reaction_timed(self._h, nrhs, _ptr(U), _ptr(F), _ptr(workspace),
                                        workspace.numel() * workspace.element_size(), ms, kind, C.byref(n),
                                        _stream(stream)), "sgdg_reaction_timed")
        return [(int(kind[i]), float(ms[i])) for i in range(n.value)]

    def iif2_step(self, dt, M, U, Fcache, workspace, newton_tol=1e-14, newton_max=50, stats=None, nrhs=1,
                  stream=None, source=None):
        _check(_lib.iif2_step(self._h, nrhs, float(dt), M, _ptr(U), _ptr(Fcache), _ptr(source), float(newton_tol),
                              newton_max, _ptr(workspace), workspace.numel() * workspace.element_size(), _ptr(stats),
                              _stream(stream)), "iif2_step")

    def iif2_step_noalloc(self, dt, M, U, Fcache, newton_tol=1e-14, newton_max=50, stats=None, nrhs=1, stream=None,
                          source=None):
        _check(_lib.iif2_step_noalloc(self._h, nrhs, float(dt), M, _ptr(U), _ptr(Fcache), _ptr(source),
                                      float(newton_tol), newton_max, _ptr(stats), _stream(stream)), "iif2_step_noalloc")

    def iif3_step(self, dt, M, U, Fcur, Fprev, workspace, newton_tol=1e-14, newton_max=50, stats=None, nrhs=1,
                  stream=None, source=None):
        _check(_lib.iif3_step(self._h, nrhs, float(dt), M, _ptr(U), _ptr(Fcur), _ptr(Fprev), _ptr(source),
                              float(newton_tol), newton_max, _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _ptr(stats), _stream(stream)), "iif3_step")

    def iif2_step_local(self, dt, M, U, Fcache, workspace, stats=None, nrhs=1, stream=None, source=None):
        _check(_lib.iif2_step_local(self._h, nrhs, float(dt), M, _ptr(U), _ptr(Fcache), _ptr(source),
                                    _ptr(workspace), workspace.numel() * workspace.element_size(), _ptr(stats),
                                    _stream(stream)), "iif2_step_local")

    def rk_step(self, dt, order, U, workspace, nrhs=1, stream=None):
        _check(_lib.rk_step(self._h, nrhs, float(dt), order, _ptr(U), _ptr(workspace),
                            workspace.numel() * workspace.element_size(), _stream(stream)), "rk_step")

    def tune(self, workspace, nrhs=1, stream=None):
        """Autotune the launch shapes of the last-axis reaction kernels (sg_dg_tune); returns the report."""
        r = TuneReport()
        _check(_lib.sg_dg_tune(self._h, nrhs, _ptr(workspace), workspace.numel() * workspace.element_size(),
                               C.byref(r), _stream(stream)), "sg_dg_tune")
        return _tune_dict(r)

    def line_shape(self, cls, ninputs, rounds, wg_per_cu, waves=0):
        _check(_lib.sg_dg_line_shape(self._h, cls, ninputs, rounds, wg_per_cu, waves), "sg_dg_line_shape")


def _tune_dict(r):
    out = []
    for i in range(r.nclass):
        out.append({"class": r.cls[i], "k": r.k[i], "N": r.n[i], "species": r.nspecies[i],
                    "rounds": [r.rounds[i][0], r.rounds[i][1]], "wg_per_cu": [r.wgcu[i][0], r.wgcu[i][1]],
                    "waves": [r.waves[i][0], r.waves[i][1]],
                    "ms_default": [r.ms_default[i][0], r.ms_default[i][1]],
                    "ms_best": [r.ms_best[i][0], r.ms_best[i][1]],
                    "from_cache": [r.from_cache[i][0], r.from_cache[i][1]]})
    return out


def stats_array(stats_tensor):
    """Host view of a device stats buffer (uint8 tensor) as a structured numpy array."""
    return stats_tensor.cpu().numpy().view(STATS_DTYPE)
