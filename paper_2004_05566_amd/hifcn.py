"""ctypes binding of libhifcn (include/hifcn.h): argument marshalling only.

Every computation runs in the library's HIP kernels.  Tensors must be CUDA (HIP) FP64 and
C-contiguous; calls are ordered on torch's current stream.  Importing this module raises if
the library has not been built, so no caller can fall back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: its HIP runtime is then the one the library binds to (both carry the same
# soname), so device pointers and streams from torch are valid in the library's calls.  With the
# library loaded first, its runtime came up without the device in a later torch process.
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhifcn.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with "
                      "`python -m paper_2004_05566_amd.build` (hipcc, gfx950)")
_lib = ctypes.CDLL(_LIB_PATH)

STORE = {"f64": 0, "f32": 1, "bf16": 2}
HIF_OK, HIF_ERR_ARG, HIF_ERR_OOM, HIF_ERR_NOT_SPD, HIF_ERR_NO_CONV, HIF_ERR_HIP = range(6)


class HifError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[status {status}] {msg}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("leaf", ctypes.c_int32)]


class _Reaction(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k1", ctypes.c_double), ("k2", ctypes.c_double)]


class _CgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("warm_start", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("root", ctypes.c_int32), ("entries", ctypes.c_int64),
                ("N", ctypes.c_int64), ("store", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("build_mfma_flops", ctypes.c_int64),
                ("build_mfma_ms", ctypes.c_double), ("apply_bytes", ctypes.c_int64),
                ("top_level", ctypes.c_int32), ("top_fold", ctypes.c_int32)]


class _FactorOpts(ctypes.Structure):
    _fields_ = [("dense_top", ctypes.c_int64), ("flags", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 2)]


FACTOR_SKEL_EDGES = 1


class _StageProf(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("stage", ctypes.c_int32),
                ("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_int64),
                ("kernel", ctypes.c_char * 32)]


STAGES = {"cell_fwd": 0, "group_fwd": 1, "root": 2, "group_bwd": 3, "cell_bwd": 4}

_vp = ctypes.c_void_p
_lib.hif_factor.argtypes = [_vp, ctypes.c_double, ctypes.POINTER(_Grid), ctypes.c_double,
                            ctypes.c_int, _vp, ctypes.POINTER(_vp)]
_lib.hif_factor_ex.argtypes = [_vp, ctypes.c_double, ctypes.POINTER(_Grid), ctypes.c_double,
                               ctypes.c_int, ctypes.POINTER(_FactorOpts), _vp, ctypes.POINTER(_vp)]
_lib.hif_import.argtypes = [_vp, ctypes.c_double, ctypes.POINTER(_Grid), _vp, ctypes.c_size_t,
                            ctypes.c_int, _vp, ctypes.POINTER(_vp)]
_lib.hif_set_coefficient.argtypes = [_vp, _vp, _vp]
_lib.hif_refactor.argtypes = [_vp, _vp, _vp]
_lib.hif_apply.argtypes = [_vp, _vp, _vp, _vp]
_lib.hif_spmv.argtypes = [_vp, _vp, _vp, _vp]
_lib.cn_step.argtypes = [_vp, ctypes.POINTER(_Reaction), ctypes.POINTER(_CgOpts), _vp,
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), _vp]
_lib.cn_solve.argtypes = [_vp, ctypes.POINTER(_Reaction), ctypes.POINTER(_CgOpts), _vp,
                          ctypes.c_int32, _vp, _vp, _vp]
_lib.cn_solve_direct.argtypes = [_vp, ctypes.POINTER(_Reaction), _vp, ctypes.c_int32, _vp]
_lib.cn_batch_step.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp]
_lib.hif_inverse_error.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  _vp]
_lib.hif_inverse_error_noalloc.argtypes = [_vp, _vp, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double), _vp]
_lib.hif_factor_bytes.argtypes = [_vp]
_lib.hif_factor_bytes.restype = ctypes.c_size_t
_lib.hif_get_info.argtypes = [_vp, ctypes.POINTER(_Info)]
_lib.hif_profile_stage.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
_lib.hif_profile_read.argtypes = [_vp, ctypes.POINTER(_StageProf)]
_lib.hif_destroy.argtypes = [_vp]
_lib.hif_destroy.restype = None
_lib.hif_last_error.restype = ctypes.c_char_p
for _f in ("hif_factor", "hif_factor_ex", "hif_import", "hif_apply", "hif_spmv", "cn_step", "cn_solve",
           "cn_solve_direct", "cn_batch_step", "hif_get_info", "hif_profile_stage",
           "hif_profile_read", "hif_set_coefficient", "hif_refactor", "hif_inverse_error",
           "hif_inverse_error_noalloc"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTS = ("hif_factor", "hif_factor_ex", "hif_import", "hif_apply", "hif_spmv", "cn_step",
           "cn_solve", "cn_solve_direct", "cn_batch_step", "hif_factor_bytes", "hif_get_info",
           "hif_profile_stage", "hif_profile_read", "hif_destroy", "hif_last_error",
           "hif_set_coefficient", "hif_refactor", "hif_inverse_error",
           "hif_inverse_error_noalloc")


def _check(status: int):
    if status != HIF_OK:
        raise HifError(status, _lib.hif_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, name, numel=None):
    """The device address of a contiguous FP64 tensor.  The library takes raw pointers, so the
    length is checked here (ValueError before any launch) whenever the caller knows it."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 device tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} values, not {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _cells_numel(n: int, dim: int) -> int:
    return (n + 1) ** dim


def _grid(n: int, dim: int, leaf: int) -> _Grid:
    g = _Grid()
    g.dim = dim
    g.n[0] = g.n[1] = n
    g.n[2] = n if dim == 3 else 0
    g.leaf = leaf
    return g


class Handle:
    """A built (or imported) PHIF factor of A = I - dt/2 M plus its PCG workspace."""

    def __init__(self, ptr: ctypes.c_void_p, n: int, dim: int):
        self._h = ptr
        self.n, self.dim = n, dim
        self.N = n ** dim

    def _p(self):
        if not self._h:
            raise HifError(HIF_ERR_ARG, "handle is closed")
        return self._h

    def apply(self, x, out=None, stream=None):
        """out = F^-1 x."""
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(_lib.hif_apply(self._p(), _dev_f64(x, "x", self.N), _dev_f64(out, "out", self.N),
                              _stream(stream)))
        return out

    def spmv(self, x, out=None, stream=None):
        """out = (I - dt/2 M) x."""
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(_lib.hif_spmv(self._p(), _dev_f64(x, "x", self.N), _dev_f64(out, "out", self.N),
                             _stream(stream)))
        return out

    def cn_solve(self, u, nsteps: int, rtol: float = 1e-8, maxit: int = 500,
                 reaction=(0, 0.0, 1.0), stream=None, warm_start: bool = False):
        """Advance u (in place) by nsteps Crank-Nicolson steps; returns (iters, relres).
        warm_start: PCG starts from x0 = u^k instead of 0."""
        r = _Reaction(int(reaction[0]), float(reaction[1]), float(reaction[2]))
        o = _CgOpts(float(rtol), int(maxit), 1 if warm_start else 0)
        its = np.zeros(max(1, nsteps), np.int32)
        rel = np.zeros(max(1, nsteps), np.float64)
        st = _lib.cn_solve(self._p(), ctypes.byref(r), ctypes.byref(o), _dev_f64(u, "u", self.N),
                           int(nsteps), its.ctypes.data_as(_vp), rel.ctypes.data_as(_vp),
                           _stream(stream))
        if st == HIF_ERR_NO_CONV:
            raise HifError(st, _lib.hif_last_error().decode())
        _check(st)
        return its[:nsteps].copy(), rel[:nsteps].copy()

    def set_coefficient(self, a_cells, stream=None):
        """Later products and solves use the operator of a_cells ((n+1)^dim FP64 on the device);
        the factor is kept."""
        _check(_lib.hif_set_coefficient(self._p(), self._cells(a_cells), _stream(stream)))

    def refactor(self, a_cells, stream=None):
        """Rebuild the factor (and the operator) from a_cells with this handle's settings."""
        _check(_lib.hif_refactor(self._p(), self._cells(a_cells), _stream(stream)))

    def _cells(self, a_cells):
        return _dev_f64(a_cells, "a_cells", _cells_numel(self.n, self.dim))

    def cn_solve_direct(self, u, nsteps: int, reaction=(0, 0.0, 1.0), stream=None):
        """Advance u (in place) by nsteps Crank-Nicolson steps u <- F^-1 g, without CG."""
        r = _Reaction(int(reaction[0]), float(reaction[1]), float(reaction[2]))
        _check(_lib.cn_solve_direct(self._p(), ctypes.byref(r), _dev_f64(u, "u", self.N),
                                    int(nsteps),
                                    _stream(stream)))

    def cn_step(self, u, rtol: float = 1e-8, maxit: int = 500, reaction=(0, 0.0, 1.0),
                stream=None, warm_start: bool = False):
        r = _Reaction(int(reaction[0]), float(reaction[1]), float(reaction[2]))
        o = _CgOpts(float(rtol), int(maxit), 1 if warm_start else 0)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        _check(_lib.cn_step(self._p(), ctypes.byref(r), ctypes.byref(o), _dev_f64(u, "u", self.N),
                            ctypes.byref(it), ctypes.byref(rel), _stream(stream)))
        return it.value, rel.value

    def profile_stage(self, level: int, stage: str, enable: bool = True):
        """Time (with HIP events) every launch of one apply stage from now on."""
        _check(_lib.hif_profile_stage(self._p(), int(level), STAGES[stage], int(bool(enable))))

    def profile_read(self) -> dict:
        p = _StageProf()
        _check(_lib.hif_profile_read(self._p(), ctypes.byref(p)))
        return {"level": p.level, "stage": p.stage, "launches": p.launches, "ms": p.ms,
                "bytes": p.bytes, "kernel": p.kernel.decode()}

    def inverse_error(self, x0, iters: int = 30, stream=None) -> float:
        """hif_inverse_error: the power-iteration estimate of ||I - A F^-1||_2 from x0."""
        est = ctypes.c_double()
        _check(_lib.hif_inverse_error(self._p(), _dev_f64(x0, "x0", self.N), int(iters),
                                      ctypes.byref(est), _stream(stream)))
        return est.value

    def inverse_error_noalloc(self, x0, iters: int = 30, stream=None) -> float:
        """hif_inverse_error_noalloc: the same estimate on the library's fixed scratch."""
        est = ctypes.c_double()
        _check(_lib.hif_inverse_error_noalloc(self._p(), _dev_f64(x0, "x0", self.N), int(iters),
                                              ctypes.byref(est), _stream(stream)))
        return est.value

    def factor_bytes(self) -> int:
        return int(_lib.hif_factor_bytes(self._p()))

    def info(self) -> dict:
        i = _Info()
        _check(_lib.hif_get_info(self._p(), ctypes.byref(i)))
        return {"levels": i.levels, "root": i.root, "entries": i.entries, "N": i.N,
                "store": i.store, "dim": i.dim, "device_bytes": i.device_bytes,
                "build_mfma_flops": i.build_mfma_flops, "build_mfma_ms": i.build_mfma_ms,
                "apply_bytes": i.apply_bytes, "top_level": i.top_level,
                "top_fold": i.top_fold}

    def close(self):
        if self._h:
            _lib.hif_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cn_batch_step(handles, states, reactions, rtols, maxits, streams):
    """cn_batch_step: one Crank-Nicolson step for each (handle, state) pair, in lockstep, each on
    its own stream.  Returns (iters, relres, status) arrays; a solve that did not converge has
    status HIF_ERR_NO_CONV (the others are still advanced); any other failure raises."""
    count = len(handles)
    if not (len(states) == len(reactions) == len(rtols) == len(maxits) == len(streams) == count):
        raise ValueError("cn_batch_step: every per-solve list must have one entry per handle")
    hs = (_vp * max(1, count))(*[h._p() for h in handles])
    us = (_vp * max(1, count))(*[_dev_f64(u, "u", h.N) for h, u in zip(handles, states)])
    rs = (_Reaction * max(1, count))(*[_Reaction(int(r[0]), float(r[1]), float(r[2]))
                                      for r in reactions])
    os_ = (_CgOpts * max(1, count))(*[_CgOpts(float(t), int(m), 0)
                                      for t, m in zip(rtols, maxits)])
    ss = (_vp * max(1, count))(*[s.cuda_stream for s in streams])
    its = np.zeros(max(1, count), np.int32)
    rel = np.zeros(max(1, count), np.float64)
    sts = np.zeros(max(1, count), np.int32)
    st = _lib.cn_batch_step(hs, rs, os_, us, count, its.ctypes.data_as(_vp),
                            rel.ctypes.data_as(_vp), sts.ctypes.data_as(_vp), ss)
    if st != HIF_ERR_NO_CONV:
        _check(st)
    return its[:count].copy(), rel[:count].copy(), sts[:count].copy()


def factor(a_cells, dt: float, n: int, dim: int, eps: float, store: str = "f32",
           leaf: int = 8, stream=None, dense_top=None, skel_edges: bool = False) -> Handle:
    """hif_factor (hif_factor_ex when an option is given): build the PHIF factor on the GPU.

    dense_top: entries allowed for the dense top of the apply (0: none; None: default).
    skel_edges: 3D, skeletonize the edges of every level as well as its faces."""
    h = ctypes.c_void_p()
    g = _grid(n, dim, leaf)
    if dense_top is None and not skel_edges:
        _check(_lib.hif_factor(_dev_f64(a_cells, "a_cells", _cells_numel(n, dim)), float(dt),
                               ctypes.byref(g),
                               float(eps), STORE[store], _stream(stream), ctypes.byref(h)))
    else:
        o = _FactorOpts()
        o.dense_top = -1 if dense_top is None else int(dense_top)
        o.flags = FACTOR_SKEL_EDGES if skel_edges else 0
        _check(_lib.hif_factor_ex(_dev_f64(a_cells, "a_cells", _cells_numel(n, dim)), float(dt),
                                  ctypes.byref(g),
                                  float(eps), STORE[store], ctypes.byref(o), _stream(stream),
                                  ctypes.byref(h)))
    return Handle(h, n, dim)


def import_factor(a_cells, dt: float, n: int, dim: int, blob: bytes, store: str = "f64",
                  leaf: int = 8, stream=None) -> Handle:
    """hif_import: load a factor from an HIFB blob (test fixture)."""
    h = ctypes.c_void_p()
    g = _grid(n, dim, leaf)
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(_lib.hif_import(_dev_f64(a_cells, "a_cells", _cells_numel(n, dim)), float(dt),
                           ctypes.byref(g), buf,
                           len(blob), STORE[store], _stream(stream), ctypes.byref(h)))
    return Handle(h, n, dim)


def library_path() -> str:
    return _LIB_PATH


def raw_library():
    return _lib
