"""ctypes binding of libmcf (include/mcf.h).  Argument marshalling only: every
step of the solve runs in the library's HIP kernels.

The module-level functions carry the C names (``mcf_create``, ``mcf_solve``,
``mcf_status`` ...).  ``Solver`` wraps one handle for convenience.  PyTorch, when
present, is imported first so that the library binds to the same HIP runtime
as torch (streams and device pointers can then be shared with it).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # one HIP runtime per process: let torch's copy load first when it is installed
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional for the binding
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcf.so")

MCF_UTIL_LOG, MCF_UTIL_POWER, MCF_UTIL_ALPHA = 0, 1, 2
MCF_FP64, MCF_FP32 = 0, 1
MCF_STOP_REL_KKT, MCF_STOP_PAPER = 0, 1
MCF_OK, MCF_E_ARG, MCF_E_GRAPH, MCF_E_NOMEM, MCF_E_DEVICE, MCF_E_STATE = 0, -1, -2, -3, -4, -5
MCF_RUNNING, MCF_CONVERGED, MCF_MAX_ITER, MCF_DIVERGED = 0, 1, 2, 3
MCF_KERNELS_AUTO, MCF_KERNELS_TWO_PHASE, MCF_KERNELS_FUSED = 0, 1, 2
STATE_NAMES = {0: "running", 1: "converged", 2: "max_iter", 3: "diverged"}

EXPORTED = [
    "mcf_options_default", "mcf_workspace_bytes", "mcf_create", "mcf_solve", "mcf_solve_async", "mcf_run",
    "mcf_reset",
    "mcf_status", "mcf_get_solution", "mcf_get_state", "mcf_set_state", "mcf_destroy", "mcf_strerror",
    "mcf_solve_static", "mcf_debug_poison", "mcf_enable_kernel_timing", "mcf_kernel_time", "mcf_layout", "mcf_edge_shapes",
    "mcf_pool_options_default", "mcf_pool_create", "mcf_pool_shape", "mcf_pool_instance_options", "mcf_pool_admit", "mcf_pool_step", "mcf_pool_sync", "mcf_pool_poll", "mcf_pool_retire",
    "mcf_pool_info", "mcf_pool_destroy",
]
MCF_POOL_MAX_SLOTS = 256
FUSED_MAX_N = 512          # largest n of the single-launch iteration, the only one the pool runs


class mcf_options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("check_every", ctypes.c_int32), ("k_adapt", ctypes.c_int32),
                ("rho", ctypes.c_double), ("theta", ctypes.c_double), ("tau", ctypes.c_double),
                ("omega0", ctypes.c_double), ("device", ctypes.c_int32), ("kernel_mode", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("adapt_until", ctypes.c_int64), ("edge_waves", ctypes.c_int32), ("edge_vectors", ctypes.c_int32),
                ("node_block", ctypes.c_int32), ("graphs", ctypes.c_int32), ("node_form", ctypes.c_int32)]


class mcf_pool_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t),
                ("max_slots", ctypes.c_int32), ("check_every", ctypes.c_int32), ("n_max", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("graphs", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class mcf_result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("checked", ctypes.c_int32), ("iters", ctypes.c_int64)] + [
        (k, ctypes.c_double) for k in ("r", "r_paper", "rel_primal", "rel_dual", "rel_gap", "rel_kkt",
                                       "primal_obj", "dual_obj", "infeasible_frac", "omega", "alpha", "beta",
                                       "delta_f", "delta_y", "seconds")]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["state_name"] = STATE_NAMES.get(self.state, "?")
        return d


class mcf_scalars(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("omega", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("r", ctypes.c_double)]


class MCFError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {mcf_strerror(code)} ({code})")
        self.code = code


_lib = None
_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)


def lib():
    """Loads libmcf.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2501_17996_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        L.mcf_options_default.argtypes = [ctypes.POINTER(mcf_options)]
        L.mcf_options_default.restype = None
        L.mcf_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.mcf_workspace_bytes.restype = ctypes.c_size_t
        L.mcf_create.argtypes = [ctypes.c_int32, ctypes.c_int32, _ip, _ip, _dp, ctypes.c_int32, ctypes.c_double,
                                 _dp, ctypes.POINTER(mcf_options), ctypes.POINTER(_vp)]
        for name in ("mcf_solve", "mcf_solve_async", "mcf_reset"):
            getattr(L, name).argtypes = [_vp]
        L.mcf_run.argtypes = [_vp, ctypes.c_int64]
        L.mcf_status.argtypes = [_vp, ctypes.POINTER(mcf_result)]
        L.mcf_get_solution.argtypes = [_vp, _dp, _dp, _dp]
        L.mcf_get_state.argtypes = [_vp, _dp, _dp, ctypes.POINTER(mcf_scalars)]
        L.mcf_set_state.argtypes = [_vp, _dp, _dp, ctypes.POINTER(mcf_scalars)]
        L.mcf_destroy.argtypes = [_vp]
        L.mcf_destroy.restype = None
        L.mcf_strerror.argtypes = [ctypes.c_int]
        L.mcf_strerror.restype = ctypes.c_char_p
        L.mcf_solve_static.argtypes = [ctypes.c_int32, ctypes.c_int32, _ip, _ip, _dp, ctypes.c_int32,
                                       ctypes.c_double, _dp, ctypes.POINTER(mcf_options), _dp, _dp, _dp,
                                       ctypes.POINTER(mcf_result)]
        L.mcf_debug_poison.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64]
        L.mcf_enable_kernel_timing.argtypes = [_vp, ctypes.c_int32]
        L.mcf_kernel_time.argtypes = [_vp, _dp, ctypes.POINTER(ctypes.c_int64)]
        L.mcf_layout.argtypes = [_vp, _ip, _ip, _ip, _ip]
        L.mcf_edge_shapes.argtypes = [ctypes.c_int32, _ip, _ip, ctypes.c_int32]
        L.mcf_edge_shapes.restype = ctypes.c_int32
        L.mcf_pool_options_default.argtypes = [ctypes.POINTER(mcf_pool_options)]
        L.mcf_pool_options_default.restype = None
        L.mcf_pool_create.argtypes = [ctypes.POINTER(mcf_pool_options), ctypes.POINTER(_vp)]
        L.mcf_pool_shape.argtypes = [_vp, _ip, _ip, _ip]
        L.mcf_pool_instance_options.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(mcf_options)]
        L.mcf_pool_admit.argtypes = [_vp, _vp, _ip]
        L.mcf_pool_step.argtypes = [_vp, ctypes.c_int32]
        L.mcf_pool_sync.argtypes = [_vp]
        L.mcf_pool_poll.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(mcf_result)]
        L.mcf_pool_retire.argtypes = [_vp, ctypes.c_int32]
        L.mcf_pool_info.argtypes = [_vp, _ip, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int64)]
        L.mcf_pool_destroy.argtypes = [_vp]
        L.mcf_pool_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != MCF_OK:
        raise MCFError(rc, what)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


# ------------------------------------------------------- C-named entry points
def mcf_options_default() -> mcf_options:
    o = mcf_options()
    lib().mcf_options_default(ctypes.byref(o))
    return o


def mcf_workspace_bytes(n: int, m: int, precision: int) -> int:
    return int(lib().mcf_workspace_bytes(int(n), int(m), int(precision)))


def mcf_strerror(code: int) -> str:
    return lib().mcf_strerror(int(code)).decode()


def mcf_create(n, tail, head, cap, utility, gamma, w, opt: mcf_options | None = None):
    """Returns a handle (c_void_p).  Raises MCFError on a non-zero code."""
    tail = np.ascontiguousarray(tail, dtype=np.int32)
    head = np.ascontiguousarray(head, dtype=np.int32)
    cap, w = _f64(cap), _f64(w)
    h = _vp()
    rc = lib().mcf_create(int(n), int(tail.shape[0]), _ptr(tail, _ip), _ptr(head, _ip), _ptr(cap), int(utility),
                          float(gamma), _ptr(w), ctypes.byref(opt) if opt is not None else None, ctypes.byref(h))
    _check(rc, "mcf_create")
    return h


def mcf_solve(h):
    _check(lib().mcf_solve(h), "mcf_solve")


def mcf_solve_async(h):
    _check(lib().mcf_solve_async(h), "mcf_solve_async")


def mcf_run(h, iters: int):
    _check(lib().mcf_run(h, int(iters)), "mcf_run")


def mcf_reset(h):
    _check(lib().mcf_reset(h), "mcf_reset")


def mcf_status(h) -> dict:
    r = mcf_result()
    _check(lib().mcf_status(h, ctypes.byref(r)), "mcf_status")
    return r.as_dict()


def mcf_get_solution(h, n: int, m: int):
    F, T, Y = np.empty(n * m), np.empty(n * n), np.empty(n * n)
    _check(lib().mcf_get_solution(h, _ptr(F), _ptr(T), _ptr(Y)), "mcf_get_solution")
    return F, T, Y


def mcf_get_state(h, n: int, m: int):
    F, Y = np.empty(n * m), np.empty(n * n)
    sc = mcf_scalars()
    _check(lib().mcf_get_state(h, _ptr(F), _ptr(Y), ctypes.byref(sc)), "mcf_get_state")
    return F, Y, {"k": int(sc.k), "omega": float(sc.omega), "alpha": float(sc.alpha), "beta": float(sc.beta),
                  "r": float(sc.r)}


def mcf_set_state(h, F, Y=None, k: int | None = None, omega: float | None = None):
    F = _f64(F)
    Yk = _f64(Y) if Y is not None else None
    sc = mcf_scalars(int(k), float(omega), 0.0, 0.0, 0.0) if k is not None else None
    _check(lib().mcf_set_state(h, _ptr(F), _ptr(Yk) if Yk is not None else None,
                               ctypes.byref(sc) if sc is not None else None), "mcf_set_state")


MCF_STATIC_BYTES = 64 << 20


def mcf_solve_static(n, tail, head, cap, utility, gamma, w, opt: mcf_options | None = None):
    """The solve that allocates nothing (static device workspace).  Returns (F, T, Y, result)."""
    tail = np.ascontiguousarray(tail, dtype=np.int32)
    head = np.ascontiguousarray(head, dtype=np.int32)
    cap, w = _f64(cap), _f64(w)
    m = int(tail.shape[0])
    F, T, Y = np.empty(n * m), np.empty(n * n), np.empty(n * n)
    r = mcf_result()
    rc = lib().mcf_solve_static(int(n), m, _ptr(tail, _ip), _ptr(head, _ip), _ptr(cap), int(utility), float(gamma),
                                _ptr(w), ctypes.byref(opt) if opt is not None else None, _ptr(F), _ptr(T), _ptr(Y),
                                ctypes.byref(r))
    _check(rc, "mcf_solve_static")
    return F, T, Y, r.as_dict()


def mcf_destroy(h):
    if h:
        lib().mcf_destroy(h)


def mcf_debug_poison(h, which: str, index: int):
    _check(lib().mcf_debug_poison(h, 0 if which == "F" else 1, int(index)), "mcf_debug_poison")


def mcf_enable_kernel_timing(h, enable: bool):
    _check(lib().mcf_enable_kernel_timing(h, 1 if enable else 0), "mcf_enable_kernel_timing")


def mcf_kernel_time(h):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib().mcf_kernel_time(h, ctypes.byref(ms), ctypes.byref(cnt)), "mcf_kernel_time")
    return float(ms.value), int(cnt.value)


def mcf_layout(h):
    ld, b, e, km = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mcf_layout(h, ctypes.byref(ld), ctypes.byref(b), ctypes.byref(e), ctypes.byref(km)), "mcf_layout")
    return {"ld": ld.value, "edge_block": b.value, "edge_ept": e.value,
            "kernel_mode": {1: "two_phase", 2: "fused"}.get(km.value, "?")}


def mcf_edge_shapes(precision: int):
    """The compiled two-phase edge shapes as (edge_waves, edge_vectors) pairs."""
    cnt = lib().mcf_edge_shapes(int(precision), None, None, 0)
    wv = (ctypes.c_int32 * max(cnt, 1))()
    vc = (ctypes.c_int32 * max(cnt, 1))()
    lib().mcf_edge_shapes(int(precision), wv, vc, cnt)
    return [(int(wv[x]), int(vc[x])) for x in range(cnt)]


# --------------------------------------------------------------- convenience
class Solver:
    """One solver handle for an ``instances.Instance``."""

    def __init__(self, inst, precision: int = MCF_FP64, tol: float = 1e-4, max_iter: int = 100000,
                 check_every: int = 1, stop_rule: int = MCF_STOP_REL_KKT, stream=None, **kw):
        o = mcf_options_default()
        o.precision, o.tol, o.max_iter = int(precision), float(tol), int(max_iter)
        o.check_every, o.stop_rule = int(check_every), int(stop_rule)
        for k, v in kw.items():
            setattr(o, k, v)
        if stream is not None:
            o.stream = int(stream)
        self.n, self.m = int(inst.n), int(inst.m)
        self.workspace = kw.get("workspace")
        self.opt = o
        self.h = mcf_create(inst.n, inst.tail, inst.head, inst.cap, inst.utility, inst.gamma, inst.w, o)

    def close(self):
        if getattr(self, "h", None):
            mcf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self) -> dict:
        mcf_solve(self.h)
        return self.status()

    def solve_async(self):
        """Starts the solve and returns; poll status() until its state is not "running"."""
        mcf_solve_async(self.h)

    def wait(self, poll_s: float = 1e-3) -> dict:
        """Polls status() until an asynchronous solve has ended; returns its record."""
        import time
        while True:
            st = self.status()
            if st["state_name"] != "running":
                return st
            time.sleep(poll_s)

    def run(self, iters: int) -> dict:
        mcf_run(self.h, iters)
        return self.status()

    def reset(self):
        mcf_reset(self.h)

    def status(self) -> dict:
        return mcf_status(self.h)

    def solution(self):
        return mcf_get_solution(self.h, self.n, self.m)

    def get_state(self):
        return mcf_get_state(self.h, self.n, self.m)

    def set_state(self, F, Y=None, k=None, omega=None):
        mcf_set_state(self.h, F, Y, k, omega)

    def poison(self, which: str, index: int):
        mcf_debug_poison(self.h, which, index)

    def layout(self) -> dict:
        return mcf_layout(self.h)


# ------------------------------------------------------------------- batching pool
def mcf_pool_options_default() -> mcf_pool_options:
    o = mcf_pool_options()
    lib().mcf_pool_options_default(ctypes.byref(o))
    return o


def mcf_pool_create(precision: int, hbm_budget: int = 0, max_slots: int = 64, check_every: int = 20,
                    stream=None, device: int = 0, n_max: int = 0, waves: int = 0, graphs: int = 1):
    o = mcf_pool_options_default()
    o.device, o.precision, o.hbm_budget = int(device), int(precision), int(hbm_budget)
    o.max_slots, o.check_every, o.n_max = int(max_slots), int(check_every), int(n_max)
    o.waves, o.graphs = int(waves), int(graphs)
    o.stream = stream
    h = _vp()
    _check(lib().mcf_pool_create(ctypes.byref(o), ctypes.byref(h)), "mcf_pool_create")
    return h


def mcf_pool_shape(p) -> dict:
    w, g, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mcf_pool_shape(p, ctypes.byref(w), ctypes.byref(g), ctypes.byref(e)), "mcf_pool_shape")
    return {"waves": w.value, "grid": g.value, "max_ept": e.value}


POOL_INSTANCE_FIELDS = ("precision", "kernel_mode", "edge_waves", "edge_vectors", "node_block")


def mcf_pool_instance_options(p, n: int) -> dict:
    """The precision, organisation and launch shape an instance of n nodes should be created
    with to run in this pool (keyword arguments of Solver)."""
    o = mcf_options_default()
    _check(lib().mcf_pool_instance_options(p, int(n), ctypes.byref(o)), "mcf_pool_instance_options")
    return {k: int(getattr(o, k)) for k in POOL_INSTANCE_FIELDS}


def mcf_pool_admit(p, s) -> int:
    slot = ctypes.c_int32()
    _check(lib().mcf_pool_admit(p, s, ctypes.byref(slot)), "mcf_pool_admit")
    return slot.value


def mcf_pool_step(p, iters: int):
    _check(lib().mcf_pool_step(p, int(iters)), "mcf_pool_step")


def mcf_pool_sync(p):
    _check(lib().mcf_pool_sync(p), "mcf_pool_sync")


def mcf_pool_poll(p, slot: int) -> dict:
    r = mcf_result()
    _check(lib().mcf_pool_poll(p, int(slot), ctypes.byref(r)), "mcf_pool_poll")
    return r.as_dict()


def mcf_pool_retire(p, slot: int):
    _check(lib().mcf_pool_retire(p, int(slot)), "mcf_pool_retire")


def mcf_pool_info(p) -> dict:
    a, u, g = ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_int64()
    _check(lib().mcf_pool_info(p, ctypes.byref(a), ctypes.byref(u), ctypes.byref(g)), "mcf_pool_info")
    return {"active": a.value, "used_bytes": u.value, "iterations": g.value}


def mcf_pool_destroy(p):
    if p:
        lib().mcf_pool_destroy(p)


class Pool:
    """A batching pool: many instances advanced by one launch per iteration."""

    def __init__(self, precision: int = MCF_FP32, hbm_budget: int = 0, max_slots: int = 64, check_every: int = 20,
                 stream=None, n_max: int = 0, waves: int = 0, graphs: int = 1):
        self.check_every = int(check_every)
        self.h = mcf_pool_create(precision, hbm_budget, max_slots, check_every,
                                 ctypes.c_void_p(int(stream)) if stream is not None else None, n_max=n_max,
                                 waves=waves, graphs=graphs)

    def shape(self) -> dict:
        return mcf_pool_shape(self.h)

    def instance_options(self, n: int) -> dict:
        return mcf_pool_instance_options(self.h, n)

    def admit(self, solver: "Solver") -> int:
        return mcf_pool_admit(self.h, solver.h)

    def step(self, iters: int | None = None):
        mcf_pool_step(self.h, iters or self.check_every)

    def sync(self):
        mcf_pool_sync(self.h)

    def poll(self, slot: int) -> dict:
        return mcf_pool_poll(self.h, slot)

    def retire(self, slot: int):
        mcf_pool_retire(self.h, slot)

    def info(self) -> dict:
        return mcf_pool_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            mcf_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
