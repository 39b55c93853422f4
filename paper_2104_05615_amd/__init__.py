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
MSPCG_BUSY = 2
MSPCG_ERR_INVALID_ARG = -1
MSPCG_ERR_BAD_TILING = -2
MSPCG_ERR_NO_GAUGE = -3
MSPCG_ERR_NO_PARAMS = -4
MSPCG_ERR_OOM = -5
MSPCG_ERR_HIP = -6
MSPCG_ERR_BREAKDOWN = -7

MSPCG_FP64, MSPCG_FP32, MSPCG_FP16, MSPCG_BF16, MSPCG_INT8 = 0, 1, 2, 3, 4
PREC = {"fp64": MSPCG_FP64, "fp32": MSPCG_FP32, "fp16": MSPCG_FP16, "bf16": MSPCG_BF16, "int8": MSPCG_INT8}

OPS = {
    "dslash_eo": 0, "dslash_oe": 1, "dslash_dag_eo": 2, "dslash_dag_oe": 3,
    "m5": 4, "m5inv": 5, "mphi": 6, "D": 7, "Ddag": 8, "A": 9, "A_sub": 10, "precond": 11,
    "store": 12,
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
                ("ms_precond", ctypes.c_double), ("status", ctypes.c_int32)]


class mspcg_request(ctypes.Structure):
    _fields_ = [("field", ctypes.c_int32), ("Ls", ctypes.c_int32), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("M5", ctypes.c_double), ("mf", ctypes.c_double), ("sub", ctypes.c_int32 * 4),
                ("solver", mspcg_solver_params), ("nrhs", ctypes.c_int32), ("src", ctypes.c_void_p),
                ("x", ctypes.c_void_p)]


class mspcg_server_stats(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_int64), ("bytes_in_use", ctypes.c_int64), ("bytes_peak", ctypes.c_int64),
                ("inflight", ctypes.c_int32), ("waiting", ctypes.c_int32), ("peak_inflight", ctypes.c_int32),
                ("contexts", ctypes.c_int32), ("completed", ctypes.c_int64), ("evictions", ctypes.c_int64)]


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
    "mspcg_solve_batch_device": [_h, _i32, _p, _p, _p, _p, ctypes.POINTER(mspcg_stats)],
    "mspcg_solve_full_device": [_h, _p, _p, _p, ctypes.POINTER(mspcg_stats), ctypes.POINTER(_d)],
    "mspcg_autotune": [_h, _i32],
    "mspcg_share_gauge": [_h, _h],
    "mspcg_set_reduced": [_h, _i32, _d, _d, _d, _p],
    "mspcg_get_reduced": [_h, ctypes.POINTER(_i32), _p],
    "mspcg_reduced_loss": [_h, _i32, _p, ctypes.POINTER(_d), _p],
    "mspcg_train_reduced": [_h, _i32, _p, _i32, _d, _p],
    "mspcg_set_graphs": [_h, _i32],
    "mspcg_set_log": [_h, _i32],
    "mspcg_set_mfma": [_i32],
    "mspcg_server_set_graphs": [_h, _i32],
    "mspcg_server_set_mode": [_h, _i32, _i32],
    "mspcg_footprint": [_h, _i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "mspcg_server_create": [ctypes.POINTER(_h), _i32, ctypes.c_int64, _i32],
    "mspcg_server_destroy": [_h],
    "mspcg_server_add_field": [_h, ctypes.POINTER(_i32), _p, ctypes.POINTER(_i32)],
    "mspcg_server_submit": [_h, ctypes.POINTER(mspcg_request), ctypes.POINTER(ctypes.c_int64)],
    "mspcg_server_poll": [_h, ctypes.c_int64, ctypes.POINTER(_i32)],
    "mspcg_server_wait": [_h, ctypes.c_int64, ctypes.POINTER(mspcg_stats), ctypes.POINTER(_d)],
    "mspcg_server_info": [_h, ctypes.POINTER(mspcg_server_stats)],
    "mspcg_get_schedule": [_h, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_d)],
    "mspcg_set_schedule": [_h, _i32, _i32, _i32, _i32, _i32],
    "mspcg_get_tchunk": [_h, _i32, _i32, ctypes.POINTER(_i32)],
    "mspcg_apply": [_h, _i32, ctypes.c_int, _p, _p],
    "mspcg_apply_device": [_h, _i32, ctypes.c_int, _p, _p, _p],
    "mspcg_apply_device_noalloc": [_h, _i32, ctypes.c_int, _p, _p, _p],
    "mspcg_get_history": [_h, _p, _p, _i32, ctypes.POINTER(_i32)],
    "mspcg_cb_open": [_h, _i32, _p],
    "mspcg_cb_submit": [_h, _p, _p, ctypes.POINTER(_i32)],
    "mspcg_cb_step": [_h, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "mspcg_cb_poll": [_h, _i32, ctypes.POINTER(_i32), ctypes.POINTER(mspcg_stats)],
    "mspcg_cb_close": [_h],
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


def _solver_params(tol=1e-10, maxiter=10000, inner_iters=6, inner_prec="fp16", outer_prec="fp32",
                   reliable_delta=0.1, beta_rule="PR", use_precond=True):
    return mspcg_solver_params(float(tol), int(maxiter), int(inner_iters), PREC[inner_prec], PREC[outer_prec],
                               float(reliable_delta), 0 if beta_rule == "PR" else 1, 1 if use_precond else 0)


def _stats(st, s):
    return Stats(st, s.outer_iters, s.inner_iters_total, s.reliable_updates, s.true_rel_resid,
                 s.iter_rel_resid, s.ms_total, s.ms_precond)


KIND_OUTER, KIND_FP64, KIND_INNER = 0, 1, 2


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
        self.b, self.c = float(b), float(c)

    def set_subdomains(self, sub):
        _check(mspcg_set_subdomains(self._h, (_i32 * 4)(*[int(s) for s in sub])))

    def set_solver(self, tol=1e-10, maxiter=10000, inner_iters=6, inner_prec="fp16", outer_prec="fp32",
                   reliable_delta=0.1, beta_rule="PR", use_precond=True):
        p = _solver_params(tol, maxiter, inner_iters, inner_prec, outer_prec, reliable_delta, beta_rule, use_precond)
        _check(mspcg_set_solver(self._h, ctypes.byref(p)))

    def set_graphs(self, on=True):
        _check(mspcg_set_graphs(self._h, 1 if on else 0))

    def set_log(self, every=0):
        _check(mspcg_set_log(self._h, int(every)))

    def share_gauge(self, other):
        _check(mspcg_share_gauge(self._h, other._h))

    # ---- reduced-Ls preconditioner (Sec. 3.3)
    def set_reduced(self, Lhat, b_hat=None, c_hat=None, mu=0.0, T=None):
        """Use z = (T^dag Mhat^-1 T + mu) r as the preconditioner; T complex of shape
        (Lhat, 4, Ls, 4).  b_hat / c_hat default to this handle's b, c.  Lhat = 0: off."""
        if int(Lhat) == 0:
            _check(mspcg_set_reduced(self._h, 0, 0.0, 0.0, 0.0, None))
            return
        T = np.ascontiguousarray(np.asarray(T, dtype=np.complex128).reshape(int(Lhat), 4, self.Ls, 4))
        self._T_keep = T
        _check(mspcg_set_reduced(self._h, int(Lhat), float(self.b if b_hat is None else b_hat),
                                 float(self.c if c_hat is None else c_hat), float(mu),
                                 T.ctypes.data_as(ctypes.c_void_p)))

    def reduced(self):
        """(Lhat, T) of the current reduced-Ls preconditioner ((0, None) when off)."""
        L = _i32()
        _check(mspcg_get_reduced(self._h, ctypes.byref(L), None))
        if L.value == 0:
            return 0, None
        T = np.empty((L.value, 4, self.Ls, 4), dtype=np.complex128)
        _check(mspcg_get_reduced(self._h, ctypes.byref(L), T.ctypes.data_as(ctypes.c_void_p)))
        return L.value, T

    def reduced_loss(self, nvec, v_ptr, gradient=False):
        """chi^2 over nvec device FP64 fields at v_ptr (and its gradient, complex (Lhat, 4, Ls, 4))."""
        c = _d()
        L = self.reduced()[0]
        g = np.empty((L, 4, self.Ls, 4), dtype=np.complex128) if gradient else None
        _check(mspcg_reduced_loss(self._h, int(nvec), ctypes.c_void_p(v_ptr), ctypes.byref(c),
                                  g.ctypes.data_as(ctypes.c_void_p) if gradient else None))
        return (c.value, g) if gradient else c.value

    def train_reduced(self, nvec, v_ptr, iters, momentum=0.5):
        """Train T in place; returns the chi^2 history (iters + 1 values)."""
        hist = np.zeros(int(iters) + 1)
        _check(mspcg_train_reduced(self._h, int(nvec), ctypes.c_void_p(v_ptr), int(iters), float(momentum),
                                   hist.ctypes.data_as(ctypes.c_void_p)))
        return hist

    def footprint(self, nrhs=1):
        """(bytes a batched solve of nrhs allocates, bytes held now)."""
        e, a = ctypes.c_int64(), ctypes.c_int64()
        _check(mspcg_footprint(self._h, int(nrhs), ctypes.byref(e), ctypes.byref(a)))
        return e.value, a.value

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

    def solve_full_device(self, phi_ptr, psi_ptr, stream=None):
        """Full 5D system on both parities (device FP64, even half then odd
        half); returns (Stats of the even solve, ||phi - M psi|| / ||phi||)."""
        s = mspcg_stats()
        r = _d()
        st = _check(mspcg_solve_full_device(self._h, phi_ptr, psi_ptr, stream, ctypes.byref(s), ctypes.byref(r)),
                    allow_not_converged=True)
        return _stats(st, s), r.value

    def solve_full(self, phi_e, phi_o):
        """Host convenience around solve_full_device: returns psi_e, psi_o, stats, full residual."""
        import torch
        n = self._n()
        buf = np.concatenate([_host_f64(phi_e, n), _host_f64(phi_o, n)])
        dphi = torch.from_numpy(buf).cuda()
        dpsi = torch.empty_like(dphi)
        torch.cuda.synchronize()
        st, res = self.solve_full_device(dphi.data_ptr(), dpsi.data_ptr())
        out = dpsi.cpu().numpy().view(np.complex128).reshape(2, self.Ls, self.vh, 4, 3)
        return out[0], out[1], st, res

    def solve_batch_device(self, nrhs, b_ptr, x_ptr, x0_ptr=None, stream=None):
        """nrhs device FP64 fields one after another; returns (status, [Stats per RHS])."""
        arr = (mspcg_stats * int(nrhs))()
        st = mspcg_solve_batch_device(self._h, int(nrhs), b_ptr, x_ptr, x0_ptr, stream, arr)
        if st not in (MSPCG_OK, MSPCG_NOT_CONVERGED, MSPCG_ERR_BREAKDOWN):
            _check(st)
        return st, [_stats(a.status, a) for a in arr]

    def autotune(self, nrhs=1):
        _check(mspcg_autotune(self._h, int(nrhs)))

    def schedule(self, kind, nrhs=1):
        """(RHS order, XCD mapping, tuned microseconds) of a hop kind (KIND_*)."""
        o, x, us = _i32(), _i32(), _d()
        _check(mspcg_get_schedule(self._h, int(kind), int(nrhs), ctypes.byref(o), ctypes.byref(x), ctypes.byref(us)))
        return o.value, x.value, us.value

    def set_schedule(self, kind, nrhs=1, order=0, xcd=1, tchunk=0):
        _check(mspcg_set_schedule(self._h, int(kind), int(nrhs), int(order), int(xcd), int(tchunk)))

    def tchunk(self, kind, nrhs=1):
        """Block order of the full-lattice hops of a kind: 0 lexicographic, k > 0 chunked t sweep."""
        t = _i32()
        _check(mspcg_get_tchunk(self._h, int(kind), int(nrhs), ctypes.byref(t)))
        return t.value

    def apply(self, op, prec, psi):
        a = _host_f64(psi, self._n())
        out = np.empty(self._n(), dtype=np.float64)
        _check(mspcg_apply(self._h, OPS[op] if isinstance(op, str) else int(op),
                           PREC[prec] if isinstance(prec, str) else int(prec), a.ctypes.data, out.ctypes.data))
        return out.view(np.complex128).reshape(self.Ls, self.vh, 4, 3)

    def apply_device(self, op, prec, in_ptr, out_ptr, stream=None):
        _check(mspcg_apply_device(self._h, OPS[op] if isinstance(op, str) else int(op),
                                  PREC[prec] if isinstance(prec, str) else int(prec), in_ptr, out_ptr, stream))

    def apply_device_noalloc(self, op, prec, in_ptr, out_ptr, stream=None):
        _check(mspcg_apply_device_noalloc(self._h, OPS[op] if isinstance(op, str) else int(op),
                                          PREC[prec] if isinstance(prec, str) else int(prec), in_ptr, out_ptr, stream))

    def history(self, pap=False):
        """|r_k| / |b| of the last single-RHS solve, k = 0 .. outer iterations;
        with pap also <p_k, A p_k> / |b|^2 of every outer iteration."""
        n = _i32()
        _check(mspcg_get_history(self._h, None, None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1))
        pp = np.zeros(max(n.value, 1))
        _check(mspcg_get_history(self._h, out.ctypes.data, pp.ctypes.data, n.value, ctypes.byref(n)))
        return (out[:n.value], pp[:max(n.value - 1, 0)]) if pap else out[:n.value]

    # continuous batching (mspcg_cb_*): slots that sources enter and leave
    def cb_open(self, slots, stream=None):
        _check(mspcg_cb_open(self._h, int(slots), stream))

    def cb_submit(self, b_ptr, x_ptr):
        """The slot the source took, or None when every slot is taken."""
        s = _i32()
        st = mspcg_cb_submit(self._h, b_ptr, x_ptr, ctypes.byref(s))
        if st == MSPCG_BUSY:
            return None
        _check(st)
        return s.value

    def cb_step(self):
        """(running, pending) after one step."""
        r, p = _i32(), _i32()
        _check(mspcg_cb_step(self._h, ctypes.byref(r), ctypes.byref(p)))
        return r.value, p.value

    def cb_poll(self, slot):
        """Stats of the slot once it has finished (the slot is then free), else None."""
        d = _i32()
        a = mspcg_stats()
        _check(mspcg_cb_poll(self._h, int(slot), ctypes.byref(d), ctypes.byref(a)))
        return _stats(a.status, a) if d.value else None

    def cb_close(self):
        _check(mspcg_cb_close(self._h))

    def set_profiling(self, on=True, stride=1):
        """HIP-event timing of the hop stages; stride N > 1 times one launch in N of each stage."""
        _check(mspcg_set_profiling(self._h, (max(1, int(stride)) if on else 0)))

    def kernel_time(self, kind):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(mspcg_get_kernel_time(self._h, int(kind), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


class Server:
    """A request loop (``mspcg_server_t``) on one device."""

    def __init__(self, device=0, hbm_budget=64 << 30, max_inflight=4):
        h = _h()
        _check(mspcg_server_create(ctypes.byref(h), int(device), int(hbm_budget), int(max_inflight)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            mspcg_server_destroy(self._h)
            self._h = _h()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_field(self, dims, U):
        X, Y, Z, T = (int(d) for d in dims)
        u = _host_f64(U, X * Y * Z * T * 4 * 9 * 2)
        f = _i32()
        _check(mspcg_server_add_field(self._h, (_i32 * 4)(X, Y, Z, T), u.ctypes.data, ctypes.byref(f)))
        return f.value

    def submit(self, field, Ls, b, c, M5, mf, sub, nrhs, src_ptr, x_ptr, **solver):
        """src_ptr / x_ptr: device FP64 buffers of nrhs fields, src ready before the call."""
        r = mspcg_request(int(field), int(Ls), float(b), float(c), float(M5), float(mf),
                          (_i32 * 4)(*[int(v) for v in (sub or (0, 0, 0, 0))]), _solver_params(**solver),
                          int(nrhs), src_ptr, x_ptr)
        t = ctypes.c_int64()
        _check(mspcg_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._nrhs = getattr(self, "_nrhs", {})
        self._nrhs[t.value] = int(nrhs)
        return t.value

    def poll(self, ticket):
        d = _i32()
        _check(mspcg_server_poll(self._h, int(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket):
        """(status, [Stats per RHS], latency in ms); errors other than the
        solve outcomes (OK, NOT_CONVERGED, BREAKDOWN, OOM) raise."""
        n = self._nrhs.pop(int(ticket), 1)
        arr = (mspcg_stats * n)()
        lat = _d()
        st = mspcg_server_wait(self._h, int(ticket), arr, ctypes.byref(lat))
        if st not in (MSPCG_OK, MSPCG_NOT_CONVERGED, MSPCG_ERR_BREAKDOWN, MSPCG_ERR_OOM):
            _check(st)
        return st, [_stats(a.status, a) for a in arr], lat.value

    def set_graphs(self, on=True):
        _check(mspcg_server_set_graphs(self._h, 1 if on else 0))

    def set_mode(self, mode="batching", slots=8):
        """'batching' (continuous batching, default) or 'contexts' (one batched solve per request)."""
        _check(mspcg_server_set_mode(self._h, 1 if mode == "batching" else 0, int(slots)))

    def info(self):
        i = mspcg_server_stats()
        _check(mspcg_server_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in mspcg_server_stats._fields_}
