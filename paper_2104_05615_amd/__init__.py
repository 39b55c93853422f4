"""Python binding of the MI355X MSPCG library (``libmspcg.so``).

Argument marshalling only: every operator and solver step runs in the
library's HIP kernels.  The module-level functions carry the C names of
``include/mspcg.h``; ``MSPCG`` wraps a handle.  PyTorch is used only for
device memory and streams; it is imported before the library is loaded so
that both share one HIP runtime.

The library must have been built (``__graft_entry__.build()``); importing
this package without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

try:  # torch first: the library binds to the HIP runtime torch loaded
    import torch  # noqa: F401
    _HAVE_TORCH = True
except Exception:  # pragma: no cover - torch is part of the image
    _HAVE_TORCH = False

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmspcg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
MSPCG_OK = 0
MSPCG_NOT_CONVERGED = 1
MSPCG_ERR_INVALID_ARG = -1
MSPCG_ERR_BAD_TILING = -2
MSPCG_ERR_NO_GAUGE = -3
MSPCG_ERR_NO_PARAMS = -4
MSPCG_ERR_OOM = -5
MSPCG_ERR_HIP = -6
MSPCG_ERR_BREAKDOWN = -7

MSPCG_FP64, MSPCG_FP32, MSPCG_FP16, MSPCG_BF16 = 0, 1, 2, 3
PREC = {"fp64": MSPCG_FP64, "fp32": MSPCG_FP32, "fp16": MSPCG_FP16, "bf16": MSPCG_BF16}

OPS = {
    "dslash_eo": 0, "dslash_oe": 1, "dslash_dag_eo": 2, "dslash_dag_oe": 3,
    "m5": 4, "m5inv": 5, "mphi": 6, "D": 7, "Ddag": 8, "A": 9, "A_sub": 10, "precond": 11,
}

KERNEL_OUTER_HOP, KERNEL_INNER_HOP, KERNEL_PRECOND, KERNEL_OUTER_HOP64 = 0, 1, 2, 3


class mspcg_solver_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("inner_prec", ctypes.c_int), ("outer_prec", ctypes.c_int),
                ("reliable_delta", ctypes.c_double), ("beta_rule", ctypes.c_int32),
                ("use_precond", ctypes.c_int32)]


class mspcg_stats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("inner_iters_total", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("true_rel_resid", ctypes.c_double),
                ("iter_rel_resid", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_precond", ctypes.c_double)]


_h = ctypes.c_void_p
_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_d = ctypes.c_double
_SIGS = {
    "mspcg_create": [ctypes.POINTER(_h), ctypes.POINTER(_i32), _i32],
    "mspcg_destroy": [_h],
    "mspcg_load_gauge": [_h, _p],
    "mspcg_set_mobius": [_h, _i32, _d, _d, _d, _d],
    "mspcg_set_subdomains": [_h, ctypes.POINTER(_i32)],
    "mspcg_set_solver": [_h, ctypes.POINTER(mspcg_solver_params)],
    "mspcg_solve": [_h, _p, _p, _p, ctypes.POINTER(mspcg_stats)],
    "mspcg_solve_device": [_h, _p, _p, _p, _p, ctypes.POINTER(mspcg_stats)],
    "mspcg_apply": [_h, _i32, ctypes.c_int, _p, _p],
    "mspcg_apply_device": [_h, _i32, ctypes.c_int, _p, _p, _p],
    "mspcg_set_profiling": [_h, _i32],
    "mspcg_get_kernel_time": [_h, _i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_d)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
    globals()[_name] = _f
_lib.mspcg_last_error.restype = ctypes.c_char_p
_lib.mspcg_last_error.argtypes = []
mspcg_last_error = _lib.mspcg_last_error

EXPORTED = sorted(list(_SIGS) + ["mspcg_last_error"])


class MSPCGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _check(st, allow_not_converged=False):
    if st == MSPCG_OK or (allow_not_converged and st == MSPCG_NOT_CONVERGED):
        return st
    raise MSPCGError(st, mspcg_last_error().decode())


def _host_f64(a, n):
    a = np.ascontiguousarray(a)
    if a.dtype == np.complex128:
        a = a.view(np.float64)
    if a.dtype != np.float64 or a.size != n:
        raise ValueError(f"expected {n} float64 values (complex interleaved), got {a.dtype} x {a.size}")
    return a


@dataclass
class Stats:
    status: int
    outer_iters: int
    inner_iters_total: int
    reliable_updates: int
    true_rel_resid: float
    iter_rel_resid: float
    ms_total: float
    ms_precond: float


def _stats(st, s):
    return Stats(st, s.outer_iters, s.inner_iters_total, s.reliable_updates, s.true_rel_resid,
                 s.iter_rel_resid, s.ms_total, s.ms_precond)


class MSPCG:
    """One library handle (``mspcg_t``)."""

    def __init__(self, dims, device: int = 0):
        self.dims = tuple(int(d) for d in dims)
        X, Y, Z, T = self.dims
        self.vh = X * Y * Z * T // 2
        self.Ls = None
        h = _h()
        _check(mspcg_create(ctypes.byref(h), (_i32 * 4)(*self.dims), int(device)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            mspcg_destroy(self._h)
            self._h = _h()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_gauge(self, U):
        X, Y, Z, T = self.dims
        u = _host_f64(U, X * Y * Z * T * 4 * 9 * 2)
        _check(mspcg_load_gauge(self._h, u.ctypes.data))

    def set_mobius(self, Ls, b, c, M5, mf):
        _check(mspcg_set_mobius(self._h, int(Ls), float(b), float(c), float(M5), float(mf)))
        self.Ls = int(Ls)

    def set_subdomains(self, sub):
        _check(mspcg_set_subdomains(self._h, (_i32 * 4)(*[int(s) for s in sub])))

    def set_solver(self, tol=1e-10, maxiter=10000, inner_iters=6, inner_prec="fp16", outer_prec="fp32",
                   reliable_delta=0.1, beta_rule="PR", use_precond=True):
        p = mspcg_solver_params(float(tol), int(maxiter), int(inner_iters), PREC[inner_prec], PREC[outer_prec],
                                float(reliable_delta), 0 if beta_rule == "PR" else 1, 1 if use_precond else 0)
        _check(mspcg_set_solver(self._h, ctypes.byref(p)))

    def _n(self):
        return self.Ls * self.vh * 24

    def solve(self, b, x0=None):
        bb = _host_f64(b, self._n())
        x = np.empty(self._n(), dtype=np.float64)
        x0p = _host_f64(x0, self._n()).ctypes.data if x0 is not None else None
        s = mspcg_stats()
        st = _check(mspcg_solve(self._h, bb.ctypes.data, x.ctypes.data, x0p, ctypes.byref(s)),
                    allow_not_converged=True)
        return x.view(np.complex128).reshape(self.Ls, self.vh, 4, 3), _stats(st, s)

    def solve_device(self, b_ptr, x_ptr, x0_ptr=None, stream=None):
        """Device FP64 buffers (e.g. torch tensor data_ptr()); stream is a HIP stream handle."""
        s = mspcg_stats()
        st = _check(mspcg_solve_device(self._h, b_ptr, x_ptr, x0_ptr, stream, ctypes.byref(s)),
                    allow_not_converged=True)
        return _stats(st, s)

    def apply(self, op, prec, psi):
        a = _host_f64(psi, self._n())
        out = np.empty(self._n(), dtype=np.float64)
        _check(mspcg_apply(self._h, OPS[op] if isinstance(op, str) else int(op),
                           PREC[prec] if isinstance(prec, str) else int(prec), a.ctypes.data, out.ctypes.data))
        return out.view(np.complex128).reshape(self.Ls, self.vh, 4, 3)

    def apply_device(self, op, prec, in_ptr, out_ptr, stream=None):
        _check(mspcg_apply_device(self._h, OPS[op] if isinstance(op, str) else int(op),
                                  PREC[prec] if isinstance(prec, str) else int(prec), in_ptr, out_ptr, stream))

    def set_profiling(self, on=True):
        _check(mspcg_set_profiling(self._h, 1 if on else 0))

    def kernel_time(self, kind):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(mspcg_get_kernel_time(self._h, int(kind), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value
