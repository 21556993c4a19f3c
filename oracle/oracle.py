"""ctypes binding of the CPU oracle (hcn_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg use this module; the product path never does.
It imports nothing from the GPU package.  Systems are passed duck-typed
(attributes N, n, P, eq_ptr, mon_ptr, var, exp, coef as numpy arrays).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from types import SimpleNamespace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hcn_oracle.c")
LIB = os.path.join(HERE, "libhcn_oracle.so")

OK, EINVAL, ENOMEM, ESINGULAR = 0, -1, -2, -4
NOT_CONVERGED, DIVERGED, MAX_STEPS, STEP_TOO_SMALL, NAN = 1, 2, 3, 4, 5

OP = dict(add=0, sub=1, mul=2, div=3, sqrt=4, mul_d=5,
          cadd=10, csub=11, cmul=12, cmul_conj=13, cnorm2=14, cscale=15,
          two_sum=20, fast_two_sum=21, two_prod=22)

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99", "-fopenmp"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction of a*b+c into fma)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Sys(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("n", ctypes.c_int), ("P", ctypes.c_int),
                ("eq_ptr", ctypes.c_void_p), ("mon_ptr", ctypes.c_void_p),
                ("var", ctypes.c_void_p), ("exp", ctypes.c_void_p),
                ("coef", ctypes.c_void_p)]


class _NewtonParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("tol_res", ctypes.c_double),
                ("tol_dx", ctypes.c_double), ("max_eq_val", ctypes.c_double)]


class _NewtonResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("res_norm", ctypes.c_double), ("dx_norm", ctypes.c_double)]


class _TrackParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("tol_res", ctypes.c_double),
                ("tol_dx", ctypes.c_double), ("max_eq_val", ctypes.c_double),
                ("max_dt", ctypes.c_double), ("min_dt", ctypes.c_double),
                ("max_steps", ctypes.c_int), ("end_iters", ctypes.c_int),
                ("end_tol", ctypes.c_double), ("predictor_order", ctypes.c_int)]


class _PathResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_int),
                ("newton_iters", ctypes.c_int), ("end_iters", ctypes.c_int),
                ("end_status", ctypes.c_int), ("accepted", ctypes.c_int),
                ("t", ctypes.c_double), ("res_norm", ctypes.c_double),
                ("dx_norm", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        _lib.ora_elementwise.argtypes = [ci, ci, ci, vp, vp, vp]
        _lib.ora_eval.argtypes = [ctypes.POINTER(_Sys), vp, vp, vp]
        _lib.ora_eval_h.argtypes = [ctypes.POINTER(_Sys), ctypes.POINTER(_Sys), vp, ci, cd, vp, vp, vp]
        _lib.ora_mgs_solve.argtypes = [ci, ci, ci, vp, vp, vp, vp]
        _lib.ora_newton.argtypes = [ctypes.POINTER(_Sys), ctypes.POINTER(_Sys), vp, ci, cd, vp,
                                    ctypes.POINTER(_NewtonParams), ctypes.POINTER(_NewtonResult)]
        _lib.ora_newton_step.argtypes = [ctypes.POINTER(_Sys), ctypes.POINTER(_Sys), vp, ci, cd, vp, vp]
        _lib.ora_track.argtypes = [ctypes.POINTER(_Sys), ctypes.POINTER(_Sys), vp, ci, vp,
                                   ctypes.POINTER(_TrackParams), vp, ctypes.POINTER(_PathResult)]
        _lib.ora_track_trace.argtypes = [ctypes.POINTER(_Sys), ctypes.POINTER(_Sys), vp, ci, vp,
                                         ctypes.POINTER(_TrackParams), vp,
                                         ctypes.POINTER(_PathResult), vp, ci]
        _lib.ora_predict.argtypes = [ci, ci, ci, vp, vp, cd, vp]
        _lib.ora_sum.argtypes = [ci, ci, vp, vp]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class SysRef:
    """Keeps contiguous copies of a system's tables alive for ctypes."""

    def __init__(self, s):
        self.N, self.n, self.P = int(s.N), int(s.n), int(s.P)
        self.eq_ptr = np.ascontiguousarray(s.eq_ptr, dtype=np.int32)
        self.mon_ptr = np.ascontiguousarray(s.mon_ptr, dtype=np.int32)
        self.var = np.ascontiguousarray(s.var, dtype=np.int32)
        self.exp = np.ascontiguousarray(s.exp, dtype=np.int32)
        self.coef = np.ascontiguousarray(s.coef, dtype=np.float64)
        self.c = _Sys(self.N, self.n, self.P, _p(self.eq_ptr).value, _p(self.mon_ptr).value,
                      _p(self.var).value, _p(self.exp).value, _p(self.coef).value)


def _ref(s):
    if s is None:
        return None
    return s if isinstance(s, SysRef) else SysRef(s)


def _sp(r):
    return ctypes.byref(r.c) if r is not None else None


# ---------------------------------------------------------------------------

def elementwise(op: str, P: int, a: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """Elementwise DD/QD op.  Real ops take [count][P], complex ops
    [count][2][P]; mul_d takes b as [count] doubles, cscale takes b as a real
    [count][P]; the error-free transformations take doubles [count] and
    return [count][2]."""
    code = OP[op]
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b if b is not None else np.zeros_like(a), dtype=np.float64)
    if code >= 20:
        count = a.size
        out = np.zeros((count, 2))
    elif code >= 10:
        count = a.shape[0]
        out = np.zeros((count, P)) if op == "cnorm2" else np.zeros((count, 2, P))
    else:
        count = a.shape[0]
        out = np.zeros((count, P))
    rc = lib().ora_elementwise(code, P, count, _p(a), _p(b), _p(out))
    if rc:
        raise ValueError(f"ora_elementwise rc={rc}")
    return out


def accurate_sum(P: int, a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, P)
    out = np.zeros(P)
    lib().ora_sum(P, a.shape[0], _p(a), _p(out))
    return out


def eval_jac(s, x: np.ndarray):
    """f [N][2][P] and column-major J [n][N][2][P] at x [n][2][P]."""
    r = _ref(s)
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros((r.N, 2, r.P))
    J = np.zeros((r.n, r.N, 2, r.P))
    rc = lib().ora_eval(_sp(r), _p(x), _p(f), _p(J))
    if rc:
        raise ValueError(f"ora_eval rc={rc}")
    return f, J


def eval_h(F, G, gamma, k: int, t: float, x: np.ndarray):
    rf, rg = _ref(F), _ref(G)
    x = np.ascontiguousarray(x, dtype=np.float64)
    gam = np.ascontiguousarray(gamma if gamma is not None else np.zeros((2, rf.P)), dtype=np.float64)
    h = np.zeros((rf.N, 2, rf.P))
    J = np.zeros((rf.n, rf.N, 2, rf.P))
    rc = lib().ora_eval_h(_sp(rf), _sp(rg), _p(gam), int(k), float(t), _p(x), _p(h), _p(J))
    if rc:
        raise ValueError(f"ora_eval_h rc={rc}")
    return h, J


def mgs_solve(P: int, A: np.ndarray, b: np.ndarray):
    """MGS solve of A dx = b, A column-major [n][N][2][P].  Returns
    (status, dx, Q, R, b_out) with R column-major [n+1][n][2][P]."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    b = np.array(b, dtype=np.float64, order="C", copy=True)
    n, N = A.shape[0], A.shape[1]
    dx = np.zeros((n, 2, P))
    R = np.zeros((n + 1, n, 2, P))
    rc = lib().ora_mgs_solve(P, N, n, _p(A), _p(b), _p(dx), _p(R))
    return rc, dx, A, R, b


def newton(F, G, gamma, k: int, t: float, x: np.ndarray, max_iter=3, tol_res=1e-12,
           tol_dx=1e-12, max_eq_val=1.0):
    rf, rg = _ref(F), _ref(G)
    x = np.array(x, dtype=np.float64, copy=True)
    gam = np.ascontiguousarray(gamma if gamma is not None else np.zeros((2, rf.P)), dtype=np.float64)
    prm = _NewtonParams(int(max_iter), float(tol_res), float(tol_dx), float(max_eq_val))
    res = _NewtonResult()
    lib().ora_newton(_sp(rf), _sp(rg), _p(gam), int(k), float(t), _p(x),
                     ctypes.byref(prm), ctypes.byref(res))
    return x, SimpleNamespace(status=res.status, iters=res.iters,
                              res_norm=res.res_norm, dx_norm=res.dx_norm)


def newton_step(F, G, gamma, k: int, t: float, x: np.ndarray):
    """One Newton iteration without tests; returns (rc, x_new, [res, dx])."""
    rf, rg = _ref(F), _ref(G)
    x = np.array(x, dtype=np.float64, copy=True)
    gam = np.ascontiguousarray(gamma if gamma is not None else np.zeros((2, rf.P)), dtype=np.float64)
    norms = np.zeros(2)
    rc = lib().ora_newton_step(_sp(rf), _sp(rg), _p(gam), int(k), float(t), _p(x), _p(norms))
    return rc, x, norms


DEFAULT_TRACK = dict(max_iter=3, tol_res=1e-12, tol_dx=1e-12, max_eq_val=1.0,
                     max_dt=2.0 ** -4, min_dt=2.0 ** -40, max_steps=1500,
                     end_iters=10, end_tol=None, predictor_order=1)


END_TOL = {1: 1e-14, 2: 1e-28, 4: 1e-58}


def predict(P: int, ts, xs: np.ndarray, t: float) -> np.ndarray:
    """The predictor: the interpolating polynomial of degree len(ts) - 1
    through (ts[j], xs[j]) at t; xs [d+1][n][2][P], newest first."""
    ts = np.ascontiguousarray(ts, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    d = ts.size - 1
    n = xs.shape[1]
    out = np.zeros((n, 2, P))
    rc = lib().ora_predict(P, n, d, _p(ts), _p(xs), float(t), _p(out))
    if rc:
        raise ValueError(f"ora_predict rc={rc}")
    return out


def track(F, G, gamma, k: int, x0: np.ndarray, trace: bool = False, **kw):
    """Track one path (Fig. 3).  trace=True also returns the per-step rows
    (trial t, dt, accepted, corrector evaluations) as a third value."""
    rf, rg = _ref(F), _ref(G)
    p = dict(DEFAULT_TRACK)
    p.update(kw)
    if p["end_tol"] is None:
        p["end_tol"] = END_TOL[rf.P]
    prm = _TrackParams(int(p["max_iter"]), float(p["tol_res"]), float(p["tol_dx"]),
                       float(p["max_eq_val"]), float(p["max_dt"]), float(p["min_dt"]),
                       int(p["max_steps"]), int(p["end_iters"]), float(p["end_tol"]),
                       int(p["predictor_order"]))
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    gam = np.ascontiguousarray(gamma, dtype=np.float64)
    xo = np.zeros_like(x0)
    out = _PathResult()
    cap = int(p["max_steps"]) + 2 if trace else 0
    rows = np.zeros((max(cap, 1), 4))
    lib().ora_track_trace(_sp(rf), _sp(rg), _p(gam), int(k), _p(x0), ctypes.byref(prm), _p(xo),
                          ctypes.byref(out), _p(rows) if trace else None, cap)
    r = SimpleNamespace(status=out.status, steps=out.steps, newton_iters=out.newton_iters,
                        end_iters=out.end_iters, end_status=out.end_status,
                        accepted=out.accepted, t=out.t, res_norm=out.res_norm,
                        dx_norm=out.dx_norm)
    if trace:
        return xo, r, rows[:min(out.steps, cap)]
    return xo, r


def total_degree_start(F):
    """The start system g_i = x_i^{d_i} - 1 with d_i the total degree of f_i,
    as explicit tables (the oracle's own construction)."""
    N, n, P = int(F.N), int(F.n), int(F.P)
    if N != n:
        raise ValueError("total-degree start system needs N == n")
    eq_ptr = np.asarray(F.eq_ptr)
    mon_ptr = np.asarray(F.mon_ptr)
    ex = np.asarray(F.exp)
    d = []
    for i in range(N):
        best = 0
        for m in range(int(eq_ptr[i]), int(eq_ptr[i + 1])):
            best = max(best, int(ex[int(mon_ptr[m]):int(mon_ptr[m + 1])].sum()))
        d.append(best)
    coef = np.zeros((2 * n, 2, P))
    coef[0::2, 0, 0] = 1.0
    coef[1::2, 0, 0] = -1.0
    return SimpleNamespace(N=n, n=n, P=P,
                           eq_ptr=np.arange(0, 2 * n + 1, 2, dtype=np.int32),
                           mon_ptr=_td_mon_ptr(n),
                           var=np.arange(n, dtype=np.int32),
                           exp=np.asarray(d, dtype=np.int32),
                           coef=coef, degrees=np.asarray(d))


def _td_mon_ptr(n: int) -> np.ndarray:
    # monomial 2i = x_i^{d_i} (one pair), monomial 2i+1 = constant (no pair)
    ptr = [0]
    for i in range(n):
        ptr.append(i + 1)
        ptr.append(i + 1)
    return np.asarray(ptr, dtype=np.int32)
