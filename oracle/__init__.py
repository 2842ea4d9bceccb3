"""CPU FP64 reference oracle for PDMCF.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP solver never imports, links or
calls it, and it never imports the HIP solver.

The arithmetic lives in ``pdmcf_oracle.c`` (plain C, FP64); this module is the
ctypes binding and the build step.  Array conventions follow the C side:
F is flat ``n*m`` with ``F[l*n+i]``, Y/T/W are flat ``n*n`` with ``X[j*n+i]``.
The ``as_math_*`` helpers give the (row=i) matrix views used in tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdmcf_oracle.c")
_LIB = os.path.join(_HERE, "libpdmcf_oracle.so")

METRICS = ["k", "omega", "alpha", "beta", "dF", "dY", "r", "r_paper", "rel_primal", "rel_dual",
           "rel_gap", "rel_kkt", "primal_obj", "dual_obj", "infeasible_frac", "checked", "a", "b", "e"]

STATE_NAMES = {1: "converged", 2: "max_iter", 3: "diverged"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_lib = None

_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_create.restype = _vp
        L.orc_create.argtypes = [_i32, _i32, _ip, _ip, _dp, _i32, _d, _dp, _d, _d, _d, _d, _i32, _i32, _i64]
        L.orc_destroy.argtypes = [_vp]
        L.orc_reset.argtypes = [_vp]
        L.orc_step.argtypes = [_vp, _i32]
        L.orc_solve.restype = _i32
        L.orc_solve.argtypes = [_vp, _d, _i32, _i64, _i32]
        L.orc_get_metrics.argtypes = [_vp, _dp]
        L.orc_metric_count.restype = _i32
        L.orc_get_eta.restype = _d
        L.orc_get_eta.argtypes = [_vp]
        L.orc_get_state.argtypes = [_vp, _dp, _dp, _dp]
        L.orc_set_state.argtypes = [_vp, _dp, _dp, _dp]
        L.orc_get_last.argtypes = [_vp, _dp, _dp, _dp]
        L.orc_poison.argtypes = [_vp, _i32, _i64]
        L.orc_eval_residual.argtypes = [_vp, _dp, _dp, _dp, _dp]
        L.orc_prox_log.restype = _d
        L.orc_prox_log.argtypes = [_d, _d, _d]
        L.orc_prox_power.restype = _d
        L.orc_prox_power.argtypes = [_d, _d, _d, _d]
        L.orc_prox_alpha.restype = _d
        L.orc_prox_alpha.argtypes = [_d, _d, _d, _d]
        L.orc_project.restype = _d
        L.orc_project.argtypes = [_i32, _dp, _d, _dp]
        L.orc_eta.restype = _d
        L.orc_eta.argtypes = [_i32, _i32, _ip, _ip]
        L.orc_edge_column.restype = _d
        L.orc_edge_column.argtypes = [_i32, _dp, _dp, _dp, _d, _d, _d, _dp, _dp, _dp]
        L.orc_node_column.argtypes = [_i32, _i32, _i32, _dp, _i32, _dp, _dp, _dp, _d, _d, _i32, _d,
                                      _dp, _dp, _dp]
        L.orc_num_threads_available.restype = _i32
        assert L.orc_metric_count() == len(METRICS)
        _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32a(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ primitives
def prox_log(y: float, beta: float, w: float) -> float:
    return lib().orc_prox_log(float(y), float(beta), float(w))


def prox_power(y: float, beta: float, w: float, gamma: float) -> float:
    return lib().orc_prox_power(float(y), float(beta), float(w), float(gamma))


def prox_alpha(y: float, beta: float, w: float, alpha: float) -> float:
    return lib().orc_prox_alpha(float(y), float(beta), float(w), float(alpha))


def project(q, c: float):
    """Euclidean projection of q onto {x >= 0, sum x <= c}; returns (x, mu)."""
    q = _f64(q)
    out = np.empty_like(q)
    mu = lib().orc_project(q.shape[0], _p(q), float(c), _p(out))
    return out, mu


def eta(n: int, tail, head) -> float:
    t, h = _i32a(tail), _i32a(head)
    return lib().orc_eta(n, t.shape[0], _p(t, _ip), _p(h, _ip))


def edge_column(f, yh, yt, alpha, c, rho):
    """One edge column of the PDHG step: returns (fhat, fbar, fnew, mu)."""
    f, yh, yt = _f64(f), _f64(yh), _f64(yt)
    n = f.shape[0]
    fhat, fbar, fnew = np.empty(n), np.empty(n), np.empty(n)
    mu = lib().orc_edge_column(n, _p(f), _p(yh), _p(yt), float(alpha), float(c), float(rho),
                               _p(fhat), _p(fbar), _p(fnew))
    return fhat, fbar, fnew, mu


def node_column(j, fbar_in, fbar_out, y, w, beta, rho, utility, gamma):
    """One node column of the PDHG step from the Fbar columns of the edges
    entering (fbar_in, shape (nin, n)) and leaving (fbar_out) node j.
    Returns (v, yhat, ynew)."""
    y, w = _f64(y), _f64(w)
    n = y.shape[0]
    fi = _f64(np.asarray(fbar_in).reshape(-1, n))
    fo = _f64(np.asarray(fbar_out).reshape(-1, n))
    v, yhat, ynew = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_node_column(n, int(j), fi.shape[0], _p(fi), fo.shape[0], _p(fo), _p(y), _p(w), float(beta),
                          float(rho), int(utility), float(gamma), _p(v), _p(yhat), _p(ynew))
    return v, yhat, ynew


def num_threads_available() -> int:
    return lib().orc_num_threads_available()


# ---------------------------------------------------------------------- solver
class OracleSolver:
    """FP64 PDMCF (Algorithm 2.1) on one instance."""

    def __init__(self, inst, rho=1.9, theta=0.5, tau=1e-5, omega0=1.0, k_adapt=100, threads=1, adapt_until=-1):
        self.n, self.m = int(inst.n), int(inst.m)
        self._tail, self._head = _i32a(inst.tail), _i32a(inst.head)
        self._cap, self._w = _f64(inst.cap), _f64(inst.w)
        self.utility, self.gamma = int(inst.utility), float(inst.gamma)
        self.threads = int(threads)
        h = lib().orc_create(self.n, self.m, _p(self._tail, _ip), _p(self._head, _ip), _p(self._cap),
                             self.utility, self.gamma, _p(self._w), float(rho), float(theta), float(tau),
                             float(omega0), int(k_adapt), self.threads, int(adapt_until))
        if not h:
            raise MemoryError("oracle allocation failed")
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def eta(self) -> float:
        return lib().orc_get_eta(self._h)

    def reset(self):
        lib().orc_reset(self._h)

    def step(self, check: bool = True) -> dict:
        lib().orc_step(self._h, 1 if check else 0)
        return self.metrics()

    def run(self, iters: int, check: bool = True):
        for _ in range(int(iters)):
            lib().orc_step(self._h, 1 if check else 0)
        return self.metrics()

    def solve(self, tol: float, stop_rule: int = 0, max_iter: int = 100000, check_every: int = 1) -> str:
        st = lib().orc_solve(self._h, float(tol), int(stop_rule), int(max_iter), int(check_every))
        return STATE_NAMES[st]

    def metrics(self) -> dict:
        out = np.empty(len(METRICS))
        lib().orc_get_metrics(self._h, _p(out))
        return dict(zip(METRICS, out.tolist()))

    def get_state(self):
        F = np.empty(self.n * self.m)
        Y = np.empty(self.n * self.n)
        sc = np.empty(4)
        lib().orc_get_state(self._h, _p(F), _p(Y), _p(sc))
        return F, Y, {"k": int(sc[0]), "omega": sc[1], "alpha": sc[2], "beta": sc[3]}

    def set_state(self, F, Y, k: int, omega: float):
        F, Y = _f64(F), _f64(Y)
        sc = np.array([float(k), float(omega), 0.0, 0.0])
        lib().orc_set_state(self._h, _p(F), _p(Y), _p(sc))

    def get_last(self):
        """(Fhat, That, Q) of the last step; Fhat/That are the solution when it was checked."""
        Fh = np.empty(self.n * self.m)
        Th = np.empty(self.n * self.n)
        Q = np.empty(self.n * self.m)
        lib().orc_get_last(self._h, _p(Fh), _p(Th), _p(Q))
        return Fh, Th, Q

    def eval_residual(self, Q, Fhat, Y) -> dict:
        out = np.empty(len(METRICS))
        Q, Fhat, Y = _f64(Q), _f64(Fhat), _f64(Y)
        lib().orc_eval_residual(self._h, _p(Q), _p(Fhat), _p(Y), _p(out))
        return dict(zip(METRICS, out.tolist()))

    def poison(self, which: str, idx: int):
        lib().orc_poison(self._h, 0 if which == "F" else 1, int(idx))


def as_math_F(F, n, m):
    """flat F[l*n+i] -> (n, m) matrix with entry (i, l)."""
    return np.asarray(F).reshape(m, n).T


def as_math_sq(X, n):
    """flat X[j*n+i] -> (n, n) matrix with entry (i, j)."""
    return np.asarray(X).reshape(n, n).T
