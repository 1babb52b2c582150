"""Thin ctypes binding of libfgh (include/fgh.h).

Every step of the computation runs in the HIP library; this module only marshals arguments.
PyTorch provides device memory and the stream.  The functions keep the C names; ``Plan`` is a
small convenience owner of the workspace and of the tensors a plan points to.

The library must have been built (``python -m paper_1508_02045_amd.build``); importing this
module on a machine without it raises immediately: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgh.so")

FGH_OK = 0
FGH_E_INVALID = 1
FGH_E_NOT_SPD = 2
FGH_E_UNSUPPORTED = 3
FGH_E_WORKSPACE = 4
FGH_E_NO_CONVERGENCE = 5
FGH_E_DIVERGED = 6
FGH_E_DEVICE = 7
FGH_E_CANCELLED = 8

FGH_GANI, FGH_GA = 0, 1
FGH_RICHARDSON, FGH_CG, FGH_CHEBYSHEV, FGH_EYRE_MILTON = 0, 1, 2, 3
FGH_FP64, FGH_FP32_REFINED = 0, 1
FGH_A_SYM, FGH_A_ISO, FGH_A_PHASE = 0, 1, 2

SOLVERS = {"richardson": FGH_RICHARDSON, "cg": FGH_CG, "chebyshev": FGH_CHEBYSHEV,
           "eyre_milton": FGH_EYRE_MILTON}

EXPORTS = ["fgh_plan_workspace", "fgh_plan_create", "fgh_plan_destroy", "fgh_plan_grid_points",
           "fgh_plan_bounds", "fgh_apply", "fgh_apply_f32", "fgh_apply_noalloc", "fgh_ga_coefficients", "fgh_solve",
           "fgh_solve_fixed", "fgh_solve_batch", "fgh_effective", "fgh_gani_bound", "fgh_plan_set_history", "fgh_estimate_bounds",
           "fgh_plan_set_bounds", "fgh_plan_set_profiling", "fgh_plan_read_profile", "fgh_request_footprint", "fgh_server_create", "fgh_server_submit", "fgh_server_poll",
           "fgh_server_wait", "fgh_server_drain", "fgh_server_stats", "fgh_server_batch_stats", "fgh_server_destroy",
           "fgh_status_string"]
PASS_NAMES = ["first", "axis_fwd", "middle", "axis_inv", "last", "cg_update", "reduce"]


class FghError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("fp64_applies", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("c_A", ctypes.c_double), ("C_A", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int32 * 3), ("rule", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("solver", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("E", ctypes.c_double * 3), ("phase", ctypes.c_void_p),
                ("phase_table", ctypes.c_void_p), ("n_phases", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("c_A", ctypes.c_double), ("C_A", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("pad", ctypes.c_int32), ("energy", ctypes.c_double),
                ("flux", ctypes.c_double * 3), ("rel_res_true", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("solve_seconds", ctypes.c_double)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}
        out["flux"] = list(self.flux)
        return out


RETIRE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int)

_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load libfgh.so (raises if it is missing: the HIP path is the only path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libfgh.so not built at {LIB_PATH}; run python -m paper_1508_02045_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.fgh_plan_workspace.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_size_t)]
        L.fgh_plan_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _vp, _vp, _dp, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, _vp, ctypes.c_size_t, _vp]
        L.fgh_plan_destroy.argtypes = [_vp]
        L.fgh_plan_destroy.restype = None
        L.fgh_plan_grid_points.argtypes = [_vp]
        L.fgh_plan_grid_points.restype = ctypes.c_int64
        L.fgh_plan_bounds.argtypes = [_vp, _dp, _dp]
        L.fgh_apply.argtypes = [_vp, _vp, _vp]
        L.fgh_apply_f32.argtypes = [_vp, _vp, _vp]
        L.fgh_apply_noalloc.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, _vp, _vp, _dp, ctypes.c_int, _vp, _vp, _vp]
        L.fgh_ga_coefficients.argtypes = [_vp, _vp]
        L.fgh_solve.argtypes = [_vp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _vp,
                                ctypes.POINTER(Stats)]
        L.fgh_solve_fixed.argtypes = [_vp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _vp,
                                      ctypes.POINTER(Stats)]
        L.fgh_solve_batch.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                      ctypes.POINTER(_vp), ctypes.POINTER(Stats), RETIRE_FN, _vp]
        L.fgh_effective.argtypes = [_vp, _dp, ctypes.c_int, _vp, _dp, _dp]
        L.fgh_gani_bound.argtypes = [_vp, _vp, _dp, _vp, _dp]
        L.fgh_plan_set_history.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp]
        L.fgh_estimate_bounds.argtypes = [_vp, _dp, ctypes.c_int, _vp, _dp, ctypes.POINTER(ctypes.c_int), _dp, _dp]
        L.fgh_plan_set_bounds.argtypes = [_vp, ctypes.c_double, ctypes.c_double]
        L.fgh_plan_set_profiling.argtypes = [_vp, ctypes.c_int]
        L.fgh_plan_read_profile.argtypes = [_vp, _dp, ctypes.POINTER(ctypes.c_int64)]
        L.fgh_request_footprint.argtypes = [ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_size_t)]
        L.fgh_server_create.argtypes = [ctypes.POINTER(_vp), _vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int]
        L.fgh_server_submit.argtypes = [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_int64)]
        L.fgh_server_poll.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(Result)]
        L.fgh_server_wait.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(Result)]
        L.fgh_server_drain.argtypes = [_vp]
        L.fgh_server_stats.argtypes = [_vp, _dp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int)]
        L.fgh_server_batch_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]
        L.fgh_server_destroy.argtypes = [_vp]
        L.fgh_server_destroy.restype = None
        for name in ("fgh_request_footprint", "fgh_server_create", "fgh_server_submit", "fgh_server_poll",
                     "fgh_server_wait", "fgh_server_drain", "fgh_server_stats", "fgh_server_batch_stats"):
            getattr(L, name).restype = ctypes.c_int
        L.fgh_status_string.argtypes = [ctypes.c_int]
        L.fgh_status_string.restype = ctypes.c_char_p
        for name in ("fgh_plan_workspace", "fgh_plan_create", "fgh_plan_bounds", "fgh_apply", "fgh_apply_f32", "fgh_apply_noalloc",
                     "fgh_ga_coefficients", "fgh_solve", "fgh_solve_fixed", "fgh_solve_batch", "fgh_effective",
                     "fgh_gani_bound", "fgh_plan_set_history", "fgh_estimate_bounds", "fgh_plan_set_bounds",
                     "fgh_plan_set_profiling", "fgh_plan_read_profile"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().fgh_status_string(int(status)).decode()


def _n32(N):
    return (ctypes.c_int32 * len(N))(*[int(n) for n in N])


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _hostd(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


# ----------------------------------------------------------------------------- C-name wrappers
def fgh_plan_workspace(d: int, N: Sequence[int], rule: int, precision: int, a_kind: int) -> int:
    out = ctypes.c_size_t()
    st = lib().fgh_plan_workspace(d, _n32(N), rule, precision, a_kind, ctypes.byref(out))
    if st:
        raise FghError(st, "fgh_plan_workspace")
    return out.value


def fgh_plan_create(d, N, rule, precision, a_kind, A, phase, phase_table, n_phases, c_A, C_A, workspace,
                    workspace_bytes, stream) -> int:
    h = ctypes.c_void_p()
    tab_keep = None
    tab_ptr = None
    if phase_table is not None:
        tab_keep, tab_ptr = _hostd(phase_table)
    st = lib().fgh_plan_create(ctypes.byref(h), d, _n32(N), rule, precision, a_kind, _ptr(A), _ptr(phase),
                               tab_ptr, int(n_phases), float(c_A), float(C_A), _ptr(workspace),
                               int(workspace_bytes), ctypes.c_void_p(stream))
    del tab_keep
    if st:
        raise FghError(st, "fgh_plan_create")
    return h.value


def fgh_plan_destroy(plan) -> None:
    lib().fgh_plan_destroy(ctypes.c_void_p(plan))


def fgh_apply(plan, x, y) -> None:
    st = lib().fgh_apply(ctypes.c_void_p(plan), _ptr(x), _ptr(y))
    if st:
        raise FghError(st, "fgh_apply")


def fgh_apply_f32(plan, x, y) -> None:
    st = lib().fgh_apply_f32(ctypes.c_void_p(plan), _ptr(x), _ptr(y))
    if st:
        raise FghError(st, "fgh_apply_f32")


def fgh_apply_noalloc(d, N, a_kind, A, phase, phase_table, x, y, stream) -> None:
    """y = G A x without a plan or any device allocation (GaNi, FP64); see include/fgh.h."""
    tab_keep, tab_ptr, nph = None, None, 0
    if phase_table is not None:
        tab_keep, tab_ptr = _hostd(phase_table)
        nph = tab_keep.shape[0]
    st = lib().fgh_apply_noalloc(int(d), _n32(N), int(a_kind), _ptr(A), _ptr(phase), tab_ptr, int(nph), _ptr(x),
                                 _ptr(y), ctypes.c_void_p(stream))
    del tab_keep
    if st:
        raise FghError(st, "fgh_apply_noalloc")


def fgh_solve(plan, solver, E, nrhs, tol, max_iter, e, raise_on=(FGH_E_INVALID, FGH_E_UNSUPPORTED, FGH_E_DEVICE,
                                                               FGH_E_WORKSPACE, FGH_E_NOT_SPD)):
    Ek, Ep = _hostd(E)
    stats = (Stats * nrhs)()
    st = lib().fgh_solve(ctypes.c_void_p(plan), int(solver), Ep, int(nrhs), float(tol), int(max_iter), _ptr(e), stats)
    if st in raise_on:
        raise FghError(st, "fgh_solve")
    return st, [s.as_dict() for s in stats]


def fgh_solve_fixed(plan, solver, E, nrhs, iters, e):
    Ek, Ep = _hostd(E)
    stats = (Stats * nrhs)()
    st = lib().fgh_solve_fixed(ctypes.c_void_p(plan), int(solver), Ep, int(nrhs), int(iters), _ptr(e), stats)
    if st in (FGH_E_INVALID, FGH_E_UNSUPPORTED, FGH_E_DEVICE):
        raise FghError(st, "fgh_solve_fixed")
    return st, [s.as_dict() for s in stats]


def fgh_solve_batch(plans, solver, E, tol, max_iter, e, retire=None):
    """Solves of one shape together (see include/fgh.h).  plans: plan handles; E: [n][d]; tol: [n];
    e: device tensors (one per plan); retire: optional callable(k) called as member k finishes.
    Returns (status, stats list)."""
    n = len(plans)
    Ek, Ep = _hostd(np.asarray(E, dtype=np.float64).reshape(n, -1))
    Tk, Tp = _hostd(np.asarray(tol, dtype=np.float64).reshape(n))
    hp = (_vp * n)(*[ctypes.c_void_p(h) for h in plans])
    ep = (_vp * n)(*[ctypes.c_void_p(t.data_ptr()) for t in e])
    stats = (Stats * n)()
    cb = RETIRE_FN(lambda user, k: retire(k)) if retire is not None else RETIRE_FN()
    st = lib().fgh_solve_batch(hp, n, int(SOLVERS.get(solver, solver)), Ep, Tp, int(max_iter), ep, stats, cb, None)
    del Ek, Tk
    if st in (FGH_E_INVALID, FGH_E_UNSUPPORTED, FGH_E_DEVICE, FGH_E_WORKSPACE, FGH_E_NOT_SPD):
        raise FghError(st, "fgh_solve_batch")
    return st, [s.as_dict() for s in stats]


def fgh_effective(plan, E, nrhs, e, d):
    Ek, Ep = _hostd(E)
    bil = np.zeros((nrhs, nrhs))
    flux = np.zeros((nrhs, d))
    st = lib().fgh_effective(ctypes.c_void_p(plan), Ep, int(nrhs), _ptr(e), bil.ctypes.data_as(_dp),
                             flux.ctypes.data_as(_dp))
    if st:
        raise FghError(st, "fgh_effective")
    return bil, flux


def fgh_gani_bound(gani, ga, E, e):
    """Guaranteed upper bound (A_{2N-1}(E + R e), E + R e) of a GaNi solution e (eq:ev_bounds_GaNi)."""
    Ek, Ep = _hostd(E)
    out = ctypes.c_double()
    st = lib().fgh_gani_bound(ctypes.c_void_p(gani), ctypes.c_void_p(ga), Ep, _ptr(e), ctypes.byref(out))
    if st:
        raise FghError(st, "fgh_gani_bound")
    return out.value


# ----------------------------------------------------------------------------- convenience owner
class Plan:
    """Owns the workspace (a torch uint8 tensor on the device) and keeps A alive.

    A: torch float64 device tensor [ncoef, *N] (FGH_A_SYM) or [*N] (FGH_A_ISO), or None with
    phase (torch uint8 device tensor [*N]) and phase_table (numpy [n_phases, ncoef])."""

    def __init__(self, N, rule=FGH_GANI, precision=FGH_FP64, A=None, phase=None, phase_table=None, a_kind=None,
                 c_A=0.0, C_A=0.0, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.N = tuple(int(n) for n in N)
        self.d = len(self.N)
        self.rule = rule
        self.precision = precision
        if a_kind is None:
            a_kind = FGH_A_PHASE if phase is not None else (FGH_A_ISO if A.dim() == self.d else FGH_A_SYM)
        self.a_kind = a_kind
        self.A = A.contiguous() if A is not None else None
        self.phase = phase.contiguous() if phase is not None else None
        self.phase_table = None if phase_table is None else np.ascontiguousarray(phase_table, dtype=np.float64)
        nbytes = fgh_plan_workspace(self.d, self.N, rule, precision, a_kind)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_view = self.workspace[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = fgh_plan_create(self.d, self.N, rule, precision, a_kind, self.A, self.phase, self.phase_table,
                                      0 if self.phase_table is None else self.phase_table.shape[0], c_A, C_A,
                                      self._ws_view, nbytes, self.stream.cuda_stream)
        self.grid = tuple(self.N) if rule == FGH_GANI else tuple(2 * n - 1 for n in self.N)
        self.npts = int(np.prod(self.grid))

    def bounds(self):
        lo = ctypes.c_double()
        hi = ctypes.c_double()
        lib().fgh_plan_bounds(ctypes.c_void_p(self.handle), ctypes.byref(lo), ctypes.byref(hi))
        return lo.value, hi.value

    def field(self, nrhs=1, dtype=None):
        t = self.torch
        shape = (self.d,) + self.grid if nrhs == 1 else (nrhs, self.d) + self.grid
        return t.zeros(shape, dtype=dtype or t.float64, device=self.workspace.device)

    def apply(self, x, y=None):
        if y is None:
            y = self.torch.empty_like(x)
        if x.dtype == self.torch.float32:
            fgh_apply_f32(self.handle, x, y)
        else:
            fgh_apply(self.handle, x, y)
        return y

    def solve(self, solver, E, tol, max_iter=10000, e=None):
        E = np.atleast_2d(np.asarray(E, dtype=np.float64))
        nrhs = E.shape[0]
        if e is None:
            e = self.field(nrhs)
        solver = SOLVERS.get(solver, solver)
        st, stats = fgh_solve(self.handle, solver, E, nrhs, tol, max_iter, e)
        return e, st, stats

    def solve_fixed(self, solver, E, iters, e=None):
        E = np.atleast_2d(np.asarray(E, dtype=np.float64))
        nrhs = E.shape[0]
        if e is None:
            e = self.field(nrhs)
        solver = SOLVERS.get(solver, solver)
        st, stats = fgh_solve_fixed(self.handle, solver, E, nrhs, iters, e)
        return e, st, stats

    def effective(self, E, e):
        E = np.atleast_2d(np.asarray(E, dtype=np.float64))
        return fgh_effective(self.handle, E, E.shape[0], e, self.d)

    def gani_bound(self, ga_plan, E, e):
        """This GaNi plan's solution e prolonged to the double grid of `ga_plan` (a Ga plan of the
        same microstructure) and integrated exactly there: an upper bound of (A_H E, E)."""
        return fgh_gani_bound(self.handle, ga_plan.handle, np.asarray(E, dtype=np.float64), e)

    def estimate_bounds(self, E, iters, e=None):
        """Lanczos estimates of the spectrum of C on the Krylov space of load E from `iters` CG
        bodies (fewer if the space becomes invariant).  Returns a dict: "lo", "hi" (extreme Ritz
        values), "steps" (m), "diag" and "off" (the tridiagonal T_m, numpy), "e" (the CG iterate)."""
        E = np.asarray(E, dtype=np.float64)
        if e is None:
            e = self.field(1)
        tri = np.zeros(2 * int(iters), dtype=np.float64)
        steps = ctypes.c_int()
        lo = ctypes.c_double()
        hi = ctypes.c_double()
        st = lib().fgh_estimate_bounds(ctypes.c_void_p(self.handle), E.ctypes.data_as(_dp), int(iters), _ptr(e),
                                       tri.ctypes.data_as(_dp), ctypes.byref(steps), ctypes.byref(lo),
                                       ctypes.byref(hi))
        if st:
            raise FghError(st, "fgh_estimate_bounds")
        m = steps.value
        return {"lo": lo.value, "hi": hi.value, "steps": m, "diag": tri[:m].copy(),
                "off": tri[iters: iters + max(m - 1, 0)].copy(), "e": e}

    def set_bounds(self, c_A, C_A):
        """Spectral bounds for Richardson, Chebyshev and Eyre-Milton from now on."""
        st = lib().fgh_plan_set_bounds(ctypes.c_void_p(self.handle), float(c_A), float(C_A))
        if st:
            raise FghError(st, "fgh_plan_set_bounds")

    def set_history(self, capacity=0, nrhs=1, residual=True, energy=True, conformity=False, bound_plan=None):
        """Record per-iteration histories of later solves into device arrays [nrhs][capacity]:
        the residual quantity of the stopping test, the energy U_E of the iterate (or, with
        bound_plan, a Ga plan of the same N, the GaNi guaranteed bound of the iterate), and with
        conformity=True the non-conformity ||G e - e|| and its mean-value part.  capacity 0 turns
        recording off.  Returns a dict of the tensors recorded ("res", "energy", "nonconf",
        "mean"; None where not recorded)."""
        if capacity <= 0:
            st = lib().fgh_plan_set_history(ctypes.c_void_p(self.handle), None, None, None, None, None, 0, None)
            self._hist = None
            if st:
                raise FghError(st, "fgh_plan_set_history")
            return {"res": None, "energy": None, "nonconf": None, "mean": None}
        mk = lambda on: (self.torch.full((nrhs, capacity), float("nan"), dtype=self.torch.float64,
                                         device=self.workspace.device) if on else None)
        h = {"res": mk(residual), "energy": mk(energy), "nonconf": mk(conformity), "mean": mk(conformity)}
        p = lambda t: _ptr(t) if t is not None else None
        scratch = self.field(1) if conformity else None
        st = lib().fgh_plan_set_history(ctypes.c_void_p(self.handle), p(h["res"]), p(h["energy"]), p(h["nonconf"]),
                                        p(h["mean"]), p(scratch), int(capacity),
                                        ctypes.c_void_p(bound_plan.handle) if bound_plan is not None else None)
        if st:
            raise FghError(st, "fgh_plan_set_history")
        self._hist = (h, scratch, bound_plan)  # keep alive while recording
        return h

    def ga_coefficients(self):
        ncoef = (3 if self.d == 2 else 6) if self.a_kind == FGH_A_SYM else 1
        out = self.torch.empty((ncoef,) + self.grid, dtype=self.torch.float64, device=self.workspace.device)
        st = lib().fgh_ga_coefficients(ctypes.c_void_p(self.handle), _ptr(out))
        if st:
            raise FghError(st, "fgh_ga_coefficients")
        return out

    def set_profiling(self, enable=True, passes=None):
        """enable: switch per-pass timing on/off; passes: names from PASS_NAMES (default all)."""
        mask = 0
        if enable:
            names = PASS_NAMES if passes is None else passes
            for n in names:
                mask |= 1 << PASS_NAMES.index(n)
        st = lib().fgh_plan_set_profiling(ctypes.c_void_p(self.handle), mask)
        if st:
            raise FghError(st, "fgh_plan_set_profiling")

    def read_profile(self):
        k = len(PASS_NAMES)
        ms = (ctypes.c_double * k)()
        n = (ctypes.c_int64 * k)()
        st = lib().fgh_plan_read_profile(ctypes.c_void_p(self.handle), ms, n)
        if st:
            raise FghError(st, "fgh_plan_read_profile")
        return {PASS_NAMES[i]: (ms[i], n[i]) for i in range(k)}

    def close(self):
        if getattr(self, "handle", None):
            fgh_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- serving
def make_request(d, N, phase, table, E, solver, tol, rule=FGH_GANI, precision=FGH_FP32_REFINED, max_iter=20000,
                 c_A=0.0, C_A=0.0):
    """Build a Request; returns (request, keep) -- keep the arrays alive until submission."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    table = np.ascontiguousarray(table, dtype=np.float64)
    r = Request()
    r.d = d
    for a in range(3):
        r.N[a] = int(N[a]) if a < d else 1
    r.rule = int(rule)
    r.precision = int(precision)
    r.solver = int(SOLVERS.get(solver, solver))
    r.max_iter = int(max_iter)
    r.tol = float(tol)
    for a in range(3):
        r.E[a] = float(E[a]) if a < d else 0.0
    r.phase = phase.ctypes.data
    r.phase_table = table.ctypes.data
    r.n_phases = table.shape[0]
    r.c_A = float(c_A)
    r.C_A = float(C_A)
    return r, (phase, table)


def fgh_request_footprint(request) -> int:
    out = ctypes.c_size_t()
    st = lib().fgh_request_footprint(ctypes.byref(request), ctypes.byref(out))
    if st:
        raise FghError(st, "fgh_request_footprint")
    return out.value


class Server:
    """Serving loop over a device pool (torch uint8 tensor) with `max_active` worker slots."""

    def __init__(self, pool_bytes, max_active=4, device=0):
        import torch

        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=f"cuda:{device}")
        off = (-self.pool.data_ptr()) % 256
        self.handle = ctypes.c_void_p()
        st = lib().fgh_server_create(ctypes.byref(self.handle), ctypes.c_void_p(self.pool.data_ptr() + off),
                                     int(pool_bytes), int(max_active), int(device))
        if st:
            raise FghError(st, "fgh_server_create")

    def submit(self, request) -> int:
        rid = ctypes.c_int64()
        st = lib().fgh_server_submit(self.handle, ctypes.byref(request), ctypes.byref(rid))
        if st:
            raise FghError(st, "fgh_server_submit")
        return rid.value

    def poll(self, rid):
        """The result once request `rid` has finished (released: ask once), None while pending."""
        res = Result()
        st = lib().fgh_server_poll(self.handle, int(rid), ctypes.byref(res))
        if st == FGH_E_NO_CONVERGENCE:
            return None
        if st:
            raise FghError(st, "fgh_server_poll")
        return res.as_dict()

    def wait(self, rid):
        res = Result()
        st = lib().fgh_server_wait(self.handle, int(rid), ctypes.byref(res))
        if st:
            raise FghError(st, "fgh_server_wait")
        return res.as_dict()

    def drain(self):
        st = lib().fgh_server_drain(self.handle)
        if st:
            raise FghError(st, "fgh_server_drain")

    def stats(self):
        now = ctypes.c_double()
        peak = ctypes.c_size_t()
        act = ctypes.c_int()
        lib().fgh_server_stats(self.handle, ctypes.byref(now), ctypes.byref(peak), ctypes.byref(act))
        pb = ctypes.c_int()
        nb = ctypes.c_int64()
        lib().fgh_server_batch_stats(self.handle, ctypes.byref(pb), ctypes.byref(nb))
        return {"now": now.value, "peak_pool_bytes": peak.value, "peak_active": act.value, "peak_batch": pb.value,
                "batches": nb.value}

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().fgh_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
