"""Python binding of libhcn.so (ctypes; argument marshalling only).

Every computation runs in the HIP kernels of libhcn.so.  torch provides
device memory and streams: arrays are torch CUDA float64 / int32 tensors,
passed by data pointer together with the current stream.  The library is
loaded from this package directory; there is no fallback: a missing or
unloadable library raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhcn.so")

OK, EINVAL, ENOMEM, EDEVICE, ESINGULAR = 0, -1, -2, -3, -4
NOT_CONVERGED, DIVERGED, MAX_STEPS, STEP_TOO_SMALL, NAN = 1, 2, 3, 4, 5

OPS = dict(add=0, sub=1, mul=2, div=3, sqrt=4, mul_d=5, cadd=10, csub=11, cmul=12,
           cmul_conj=13, cnorm2=14, cscale=15, two_sum=20, fast_two_sum=21, two_prod=22)


class HcnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hcn error {code}: {msg}")
        self.code = code


class _SysInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("n", ctypes.c_int), ("P", ctypes.c_int),
                ("nmon", ctypes.c_int), ("max_k", ctypes.c_int), ("nslots", ctypes.c_int),
                ("nnz_jac", ctypes.c_int), ("device_bytes", ctypes.c_size_t)]


class _NewtonParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("tol_res", ctypes.c_double),
                ("tol_dx", ctypes.c_double), ("max_eq_val", ctypes.c_double)]


class _TrackParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("tol_res", ctypes.c_double),
                ("tol_dx", ctypes.c_double), ("max_eq_val", ctypes.c_double),
                ("max_dt", ctypes.c_double), ("min_dt", ctypes.c_double),
                ("max_steps", ctypes.c_int), ("end_iters", ctypes.c_int),
                ("end_tol", ctypes.c_double), ("predictor_order", ctypes.c_int)]


PATH_RESULT_DTYPE = np.dtype([("status", np.int32), ("steps", np.int32),
                              ("newton_iters", np.int32), ("end_iters", np.int32),
                              ("end_status", np.int32), ("accepted", np.int32),
                              ("t", np.float64), ("res_norm", np.float64),
                              ("dx_norm", np.float64)])
assert PATH_RESULT_DTYPE.itemsize == 48

# every symbol the header declares
EXPORTS = ["hcn_last_error", "hcn_version", "hcn_sys_load", "hcn_sys_free", "hcn_sys_info",
           "hcn_sys_degrees", "hcn_eval_ws_bytes", "hcn_eval_jac", "hcn_mgs_ws_bytes",
           "hcn_mgs_solve", "hcn_newton_ws_bytes", "hcn_newton_step", "hcn_newton_step_static",
           "hcn_newton",
           "hcn_track_ws_bytes", "hcn_track_paths", "hcn_elementwise", "hcn_profile_enable",
           "hcn_set_mgs_variant", "hcn_set_mgs_panel", "hcn_set_mgs_wait_limit", "hcn_set_chunk_bytes", "hcn_set_mon_uniform", "hcn_set_mon_tree", "hcn_newton_mixed_ws_bytes", "hcn_newton_mixed",
           "hcn_tune_set", "hcn_tune_get", "hcn_tune_save", "hcn_tune_load", "hcn_autotune",
           "hcn_batch_create", "hcn_batch_destroy", "hcn_batch_device_bytes",
           "hcn_batch_last_error", "hcn_batch_add", "hcn_batch_release", "hcn_batch_set_split", "hcn_batch_set_persistent", "hcn_batch_step",
           "hcn_batch_poll", "hcn_batch_result", "hcn_batch_run", "hcn_batch_counts",
           "hcn_server_create", "hcn_server_destroy", "hcn_server_last_error", "hcn_server_now",
           "hcn_server_capacity", "hcn_server_submit", "hcn_server_pump", "hcn_server_fetch",
           "hcn_server_queued",
           "hcn_profile_reset", "hcn_profile_query"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1501_06625_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cd, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.hcn_last_error.restype = ctypes.c_char_p
    lib.hcn_sys_load.argtypes = [ctypes.POINTER(vp), ci, ci, ci, vp, vp, vp, vp, vp]
    lib.hcn_sys_free.argtypes = [vp]
    lib.hcn_sys_info.argtypes = [vp, ctypes.POINTER(_SysInfo)]
    lib.hcn_sys_degrees.argtypes = [vp, vp]
    lib.hcn_eval_ws_bytes.argtypes = [vp, ci]
    lib.hcn_eval_ws_bytes.restype = sz
    lib.hcn_eval_jac.argtypes = [vp, ci, vp, vp, vp, vp, sz, vp]
    lib.hcn_mgs_ws_bytes.argtypes = [ci, ci, ci, ci]
    lib.hcn_mgs_ws_bytes.restype = sz
    lib.hcn_mgs_solve.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.hcn_newton_ws_bytes.argtypes = [vp, ci]
    lib.hcn_newton_ws_bytes.restype = sz
    lib.hcn_newton_step.argtypes = [vp, vp, ci, ci, vp, vp, vp, vp, vp, sz, vp]
    lib.hcn_newton_step_static.argtypes = [vp, vp, ci, ci, vp, vp, vp, vp, vp]
    lib.hcn_newton.argtypes = [vp, vp, ci, ci, vp, vp, ctypes.POINTER(_NewtonParams), vp, vp, vp,
                               vp, sz, vp]
    lib.hcn_track_ws_bytes.argtypes = [vp, ci]
    lib.hcn_track_ws_bytes.restype = sz
    lib.hcn_track_paths.argtypes = [vp, vp, ci, ci, vp, ctypes.POINTER(_TrackParams), vp, vp, vp,
                                    sz, vp]
    lib.hcn_elementwise.argtypes = [ci, ci, ci, vp, vp, vp, vp]
    lib.hcn_profile_enable.argtypes = [ci]
    lib.hcn_set_mgs_variant.argtypes = [ci]
    lib.hcn_set_mgs_panel.argtypes = [ci]
    lib.hcn_set_mgs_wait_limit.argtypes = [ctypes.c_longlong]
    lib.hcn_set_chunk_bytes.argtypes = [sz]
    lib.hcn_set_mon_uniform.argtypes = [ci]
    lib.hcn_set_mon_tree.argtypes = [ci]
    lib.hcn_newton_mixed_ws_bytes.argtypes = [vp, ci]
    lib.hcn_newton_mixed_ws_bytes.restype = sz
    lib.hcn_newton_mixed.argtypes = lib.hcn_newton.argtypes
    lib.hcn_tune_set.argtypes = [ci, ci, ci, ci]
    lib.hcn_tune_get.argtypes = [ci, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    lib.hcn_tune_save.argtypes = [ctypes.c_char_p]
    lib.hcn_tune_load.argtypes = [ctypes.c_char_p]
    lib.hcn_autotune.argtypes = [vp, ci, vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci),
                                 ctypes.POINTER(cd), vp]
    lib.hcn_batch_create.argtypes = [ctypes.POINTER(vp), ci, ci, ci, ci, ci,
                                     ctypes.POINTER(_TrackParams), ci, ci]
    lib.hcn_batch_destroy.argtypes = [vp]
    lib.hcn_batch_device_bytes.argtypes = [vp]
    lib.hcn_batch_device_bytes.restype = sz
    lib.hcn_batch_last_error.restype = ctypes.c_char_p
    lib.hcn_batch_add.argtypes = [vp, ci, vp, vp, vp, vp]
    lib.hcn_batch_release.argtypes = [vp, ci]
    lib.hcn_batch_set_split.argtypes = [vp, ci]
    lib.hcn_batch_set_persistent.argtypes = [vp, ci]
    lib.hcn_batch_step.argtypes = [vp, ci, vp]
    lib.hcn_batch_poll.argtypes = [vp, vp, vp]
    lib.hcn_batch_result.argtypes = [vp, ci, vp, vp, vp]
    lib.hcn_batch_run.argtypes = [vp, ci, vp]
    lib.hcn_batch_counts.argtypes = [vp, vp, vp]
    lib.hcn_server_create.argtypes = [ctypes.POINTER(vp), sz, cd, ci, ci, ctypes.POINTER(_TrackParams),
                                      ctypes.POINTER(_TrackParams), ci, ci]
    lib.hcn_server_destroy.argtypes = [vp]
    lib.hcn_server_last_error.restype = ctypes.c_char_p
    lib.hcn_server_now.argtypes = [vp]
    lib.hcn_server_now.restype = cd
    lib.hcn_server_capacity.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    lib.hcn_server_submit.argtypes = [vp, ctypes.c_int64, vp, vp, vp, cd]
    lib.hcn_server_pump.argtypes = [vp]
    lib.hcn_server_fetch.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), vp, vp,
                                     ctypes.POINTER(cd), ctypes.POINTER(cd), ctypes.POINTER(cd)]
    lib.hcn_server_queued.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    lib.hcn_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(cd),
                                      ctypes.POINTER(ctypes.c_int64)]
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise HcnError(rc, _lib.hcn_last_error().decode())
    return rc


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class SysInfo:
    N: int
    n: int
    P: int
    nmon: int
    max_k: int
    nslots: int
    nnz_jac: int
    device_bytes: int


class System:
    """A polynomial system loaded on the current device (hcn_sys_load)."""

    def __init__(self, ps):
        self.N, self.n, self.P = int(ps.N), int(ps.n), int(ps.P)
        eq_ptr = np.ascontiguousarray(ps.eq_ptr, dtype=np.int32)
        mon_ptr = np.ascontiguousarray(ps.mon_ptr, dtype=np.int32)
        var = np.ascontiguousarray(ps.var, dtype=np.int32)
        exp = np.ascontiguousarray(ps.exp, dtype=np.int32)
        coef = np.ascontiguousarray(ps.coef, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(_lib.hcn_sys_load(ctypes.byref(h), self.N, self.n, self.P, _np_ptr(eq_ptr),
                                 _np_ptr(mon_ptr), _np_ptr(var), _np_ptr(exp), _np_ptr(coef)))
        self.handle = h
        self.device = torch.device("cuda", torch.cuda.current_device())

    def info(self) -> SysInfo:
        i = _SysInfo()
        _check(_lib.hcn_sys_info(self.handle, ctypes.byref(i)))
        return SysInfo(i.N, i.n, i.P, i.nmon, i.max_k, i.nslots, i.nnz_jac, i.device_bytes)

    def degrees(self) -> np.ndarray:
        d = np.zeros(self.N, dtype=np.int32)
        _check(_lib.hcn_sys_degrees(self.handle, _np_ptr(d)))
        return d

    def free(self):
        if self.handle:
            _lib.hcn_sys_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _batched(x: torch.Tensor, tail: int):
    """Return (tensor with a batch axis, had_batch)."""
    if x.dim() == tail:
        return x.unsqueeze(0), False
    return x, True


def eval_jac(sys: System, x: torch.Tensor, want_jac: bool = True):
    """f [B][N][2][P] and column-major J [B][n][N][2][P] at x [B][n][2][P]."""
    xb, batched = _batched(x.contiguous(), 3)
    B = xb.shape[0]
    f = torch.empty((B, sys.N, 2, sys.P), dtype=torch.float64, device=x.device)
    J = torch.empty((B, sys.n, sys.N, 2, sys.P), dtype=torch.float64, device=x.device) if want_jac else None
    ws = _workspace(_lib.hcn_eval_ws_bytes(sys.handle, B), x.device)
    _check(_lib.hcn_eval_jac(sys.handle, B, _ptr(xb), _ptr(f), _ptr(J), _ptr(ws), ws.numel(),
                             _stream()))
    if not batched:
        return f[0], (J[0] if J is not None else None)
    return f, J


def mgs_solve(A: torch.Tensor, b: torch.Tensor, want_R: bool = True):
    """Solve A dx = b by MGS; A [B][n][N][2][P] (column-major) is overwritten
    by Q and b by its residual.  Returns (dx, R or None, status)."""
    Ab, batched = _batched(A, 4)
    bb, _ = _batched(b, 3)
    if not (Ab.is_contiguous() and bb.is_contiguous()):
        raise ValueError("A and b must be contiguous (they are overwritten)")
    B, n, N, _, P = Ab.shape
    dx = torch.empty((B, n, 2, P), dtype=torch.float64, device=A.device)
    R = torch.zeros((B, n + 1, n, 2, P), dtype=torch.float64, device=A.device) if want_R else None
    status = torch.empty(B, dtype=torch.int32, device=A.device)
    ws = _workspace(_lib.hcn_mgs_ws_bytes(B, N, n, P), A.device)
    _check(_lib.hcn_mgs_solve(B, N, n, P, _ptr(Ab), _ptr(bb), _ptr(dx), _ptr(R), _ptr(status),
                              _ptr(ws), ws.numel(), _stream()))
    if not batched:
        return dx[0], (R[0] if R is not None else None), status[0]
    return dx, R, status


def _gamma_arg(gamma, P):
    if gamma is None:
        return None, None
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(2, P))
    return g, _np_ptr(g)


def newton_step(sys: System, x: torch.Tensor, gamma=None, t: Optional[torch.Tensor] = None,
                relax_k: int = 1, ws: Optional[torch.Tensor] = None):
    """One Newton iteration in place on x [B][n][2][P]; returns (norms [B][2], status [B])."""
    xb, batched = _batched(x, 3)
    if not xb.is_contiguous():
        raise ValueError("x must be contiguous (updated in place)")
    B = xb.shape[0]
    norms = torch.empty((B, 2), dtype=torch.float64, device=x.device)
    status = torch.empty(B, dtype=torch.int32, device=x.device)
    g, gp = _gamma_arg(gamma, sys.P)
    need = _lib.hcn_newton_ws_bytes(sys.handle, B)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, x.device)
    _check(_lib.hcn_newton_step(sys.handle, gp, relax_k, B, _ptr(t), _ptr(xb), _ptr(norms),
                                _ptr(status), _ptr(ws), ws.numel(), _stream()))
    if not batched:
        return norms[0], status[0]
    return norms, status


# bytes of the fixed device workspace of hcn_newton_step_static
STATIC_WS_BYTES = 64 << 20


def newton_step_static(sys: System, x: torch.Tensor, gamma=None,
                       t: Optional[torch.Tensor] = None, relax_k: int = 1):
    """newton_step on the library's fixed device workspace (no allocation by
    the library; norms and status are the caller's outputs, allocated here)."""
    xb, batched = _batched(x, 3)
    if not xb.is_contiguous():
        raise ValueError("x must be contiguous (updated in place)")
    B = xb.shape[0]
    norms = torch.empty((B, 2), dtype=torch.float64, device=x.device)
    status = torch.empty(B, dtype=torch.int32, device=x.device)
    g, gp = _gamma_arg(gamma, sys.P)
    _check(_lib.hcn_newton_step_static(sys.handle, gp, relax_k, B, _ptr(t), _ptr(xb),
                                       _ptr(norms), _ptr(status), _stream()))
    if not batched:
        return norms[0], status[0]
    return norms, status


def newton_ws(sys: System, B: int, device=None) -> torch.Tensor:
    return _workspace(_lib.hcn_newton_ws_bytes(sys.handle, B), device or sys.device)


def newton(sys: System, x: torch.Tensor, gamma=None, t: Optional[torch.Tensor] = None,
           relax_k: int = 1, max_iter: int = 3, tol_res: float = 1e-12, tol_dx: float = 1e-12,
           max_eq_val: float = 1.0, mixed: bool = False, ws: Optional[torch.Tensor] = None):
    """Fig. 2 corrector in place on x; returns (status [B], iters [B], norms [B][2]).
    mixed=True: FP64 Jacobian and solve, residual and update in DD/QD."""
    xb, batched = _batched(x, 3)
    if not xb.is_contiguous():
        raise ValueError("x must be contiguous (updated in place)")
    B = xb.shape[0]
    norms = torch.empty((B, 2), dtype=torch.float64, device=x.device)
    status = torch.empty(B, dtype=torch.int32, device=x.device)
    iters = torch.empty(B, dtype=torch.int32, device=x.device)
    g, gp = _gamma_arg(gamma, sys.P)
    prm = _NewtonParams(max_iter, tol_res, tol_dx, max_eq_val)
    need = (_lib.hcn_newton_mixed_ws_bytes if mixed else _lib.hcn_newton_ws_bytes)(sys.handle, B)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, x.device)
    fn = _lib.hcn_newton_mixed if mixed else _lib.hcn_newton
    _check(fn(sys.handle, gp, relax_k, B, _ptr(t), _ptr(xb), ctypes.byref(prm),
              _ptr(norms), _ptr(status), _ptr(iters), _ptr(ws), ws.numel(), _stream()))
    if not batched:
        return status[0], iters[0], norms[0]
    return status, iters, norms


# refinement tolerance at t = 1 per precision (double, double-double, quad-double)
END_TOL = {1: 1e-14, 2: 1e-28, 4: 1e-58}

DEFAULT_TRACK = dict(max_iter=3, tol_res=1e-12, tol_dx=1e-12, max_eq_val=1.0,
                     max_dt=2.0 ** -4, min_dt=2.0 ** -40, max_steps=1500,
                     end_iters=10, end_tol=None, predictor_order=1)


def track_paths(sys: System, gamma, x0: torch.Tensor, relax_k: int = 1, **kw):
    """Track paths from start solutions x0 [B][n][2][P]; returns (x_out, results)
    with results a numpy structured array (PATH_RESULT_DTYPE)."""
    p = dict(DEFAULT_TRACK)
    p.update(kw)
    if p["end_tol"] is None:
        p["end_tol"] = END_TOL[sys.P]
    x0b, batched = _batched(x0.contiguous(), 3)
    B = x0b.shape[0]
    xo = torch.empty_like(x0b)
    res = torch.zeros(B * PATH_RESULT_DTYPE.itemsize, dtype=torch.uint8, device=x0.device)
    g, gp = _gamma_arg(gamma, sys.P)
    prm = _TrackParams(int(p["max_iter"]), float(p["tol_res"]), float(p["tol_dx"]),
                       float(p["max_eq_val"]), float(p["max_dt"]), float(p["min_dt"]),
                       int(p["max_steps"]), int(p["end_iters"]), float(p["end_tol"]),
                       int(p["predictor_order"]))
    ws = _workspace(_lib.hcn_track_ws_bytes(sys.handle, B), x0.device)
    _check(_lib.hcn_track_paths(sys.handle, gp, relax_k, B, _ptr(x0b), ctypes.byref(prm),
                                _ptr(xo), _ptr(res), _ptr(ws), ws.numel(), _stream()))
    results = res.cpu().numpy().view(PATH_RESULT_DTYPE)
    if not batched:
        return xo[0], results[0]
    return xo, results


def elementwise(op: str, P: int, a: torch.Tensor, b: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Elementwise DD/QD operation on device arrays (layouts as hcn_elementwise)."""
    code = OPS[op]
    a = a.contiguous()
    if code >= 20:
        count = a.numel()
        out = torch.empty((count, 2), dtype=torch.float64, device=a.device)
    elif code >= 10:
        count = a.shape[0]
        shape = (count, P) if op == "cnorm2" else (count, 2, P)
        out = torch.empty(shape, dtype=torch.float64, device=a.device)
    else:
        count = a.shape[0]
        out = torch.empty((count, P), dtype=torch.float64, device=a.device)
    bb = b.contiguous() if b is not None else None
    _check(_lib.hcn_elementwise(code, P, count, _ptr(a), _ptr(bb), _ptr(out), _stream()))
    return out


def profile_enable(on: bool = True) -> None:
    _check(_lib.hcn_profile_enable(1 if on else 0))


def profile_reset() -> None:
    _check(_lib.hcn_profile_reset())


def profile_query(kernel: str):
    """(summed event milliseconds, launches) of one kernel name."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(_lib.hcn_profile_query(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


MGS_AUTO, MGS_WORKGROUP, MGS_RIGHT_LOOKING, MGS_TILED, MGS_PIPELINED = 0, 1, 2, 4, 5


def set_mgs_variant(variant: int) -> None:
    """Process-wide MGS variant (see hcn_set_mgs_variant)."""
    _check(_lib.hcn_set_mgs_variant(int(variant)))


def set_mgs_panel(T: int) -> None:
    """Panel width of the tiled MGS variant (see hcn_set_mgs_panel)."""
    _check(_lib.hcn_set_mgs_panel(int(T)))


MGS_WAIT_LIMIT = 1 << 22


def set_mgs_wait_limit(polls: int) -> None:
    """Bound on each wait of the pipelined MGS (see hcn_set_mgs_wait_limit)."""
    _check(_lib.hcn_set_mgs_wait_limit(int(polls)))


def set_mon_uniform(on: bool) -> None:
    """Uniform (1) or branching (0) common factor in the monomial kernels (see hcn_set_mon_uniform)."""
    _check(_lib.hcn_set_mon_uniform(1 if on else 0))


def set_mon_tree(on: bool) -> None:
    """Tree mode (1) or reverse mode (0) for the monomials (see hcn_set_mon_tree)."""
    _check(_lib.hcn_set_mon_tree(1 if on else 0))


def set_chunk_bytes(nbytes: int) -> None:
    """Point chunking of the Newton and tracking launches (see hcn_set_chunk_bytes)."""
    _check(_lib.hcn_set_chunk_bytes(int(nbytes)))


def tune_set(P: int, N: int, mgs_group: int, mgs_lds: int) -> None:
    """Kernel-variant choice for problems of precision P and N rows."""
    _check(_lib.hcn_tune_set(P, N, mgs_group, mgs_lds))


def autotune(sys: System, x: torch.Tensor, reps: int = 5):
    """Time every MGS variant on a Newton step at x [B][n][2][P]; keep the
    fastest for (P, N).  Returns (group, lds, ms per step)."""
    xb, _ = _batched(x.contiguous(), 3)
    g, l, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(_lib.hcn_autotune(sys.handle, xb.shape[0], _ptr(xb), reps, ctypes.byref(g),
                             ctypes.byref(l), ctypes.byref(ms), _stream()))
    return g.value, l.value, ms.value


def tune_save(path: str) -> None:
    _check(_lib.hcn_tune_save(path.encode()))


def tune_load(path: str) -> None:
    _check(_lib.hcn_tune_load(path.encode()))


def tune_get(P: int, N: int):
    g, l = ctypes.c_int(), ctypes.c_int()
    _check(_lib.hcn_tune_get(P, N, ctypes.byref(g), ctypes.byref(l)))
    return g.value, l.value


def _bcheck(rc: int) -> int:
    if rc < 0:
        raise HcnError(rc, _lib.hcn_batch_last_error().decode())
    return rc


def track_params(P: int, **kw) -> _TrackParams:
    p = dict(DEFAULT_TRACK)
    p.update(kw)
    if p["end_tol"] is None:
        p["end_tol"] = END_TOL[P]
    return _TrackParams(int(p["max_iter"]), float(p["tol_res"]), float(p["tol_dx"]),
                        float(p["max_eq_val"]), float(p["max_dt"]), float(p["min_dt"]),
                        int(p["max_steps"]), int(p["end_iters"]), float(p["end_tol"]),
                        int(p["predictor_order"]))


class Batch:
    """Slot table of paths of many systems (hcn_batch_*)."""

    def __init__(self, P: int, capacity: int, max_n: int, max_nslots: int,
                 max_systems: int = 256, relax_k: int = 1, mixed: bool = False,
                 split_n: int = 0, persistent: bool = False, **track_kw):
        self.P = P
        self.capacity = capacity
        self.prm = track_params(P, **track_kw)
        h = ctypes.c_void_p()
        _bcheck(_lib.hcn_batch_create(ctypes.byref(h), P, capacity, max_n, max_nslots,
                                      max_systems, ctypes.byref(self.prm), relax_k,
                                      1 if mixed else 0))
        self.handle = h
        if split_n:
            _bcheck(_lib.hcn_batch_set_split(h, int(split_n)))
        if persistent:
            _bcheck(_lib.hcn_batch_set_persistent(h, 1))
        self._keep = {}
        self.device = torch.device("cuda", torch.cuda.current_device())

    def add(self, slot: int, sys: System, gamma, x0: torch.Tensor):
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(2, self.P))
        x0 = x0.contiguous()
        self._keep[slot] = (sys, x0)
        _bcheck(_lib.hcn_batch_add(self.handle, slot, sys.handle, _np_ptr(g), _ptr(x0), _stream()))

    def release(self, slot: int):
        self._keep.pop(slot, None)
        _bcheck(_lib.hcn_batch_release(self.handle, slot))

    def step(self, steps: int = 1):
        _bcheck(_lib.hcn_batch_step(self.handle, steps, _stream()))

    def poll(self):
        """(number of unfinished occupied slots, done flags [capacity])."""
        done = np.zeros(self.capacity, dtype=np.int32)
        n = _bcheck(_lib.hcn_batch_poll(self.handle, _np_ptr(done), _stream()))
        return n, done

    def result(self, slot: int, n: int):
        x = torch.empty((n, 2, self.P), dtype=torch.float64, device=self.device)
        res = np.zeros(1, dtype=PATH_RESULT_DTYPE)
        _bcheck(_lib.hcn_batch_result(self.handle, slot, _ptr(x), _np_ptr(res), _stream()))
        return x, res[0]

    def run(self, chunk: int = 8):
        _bcheck(_lib.hcn_batch_run(self.handle, chunk, _stream()))

    def counts(self):
        """[capacity][2] int32: residual evaluations and solves per slot."""
        c = np.zeros((self.capacity, 2), dtype=np.int32)
        _bcheck(_lib.hcn_batch_counts(self.handle, _np_ptr(c), _stream()))
        return c

    def device_bytes(self) -> int:
        return int(_lib.hcn_batch_device_bytes(self.handle))

    def free(self):
        if self.handle:
            _lib.hcn_batch_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _scheck(rc: int) -> int:
    if rc < 0:
        raise HcnError(rc, _lib.hcn_server_last_error().decode())
    return rc


class Server:
    """Continuous-batching server of path-tracking requests (hcn_server_*)."""

    def __init__(self, budget_bytes: int, max_n: int, max_nslots: int, qd_share: float = 0.2,
                 steps_per_round: int = 4, serial: bool = False, **track_kw):
        self.dd_prm = track_params(2, **track_kw)
        self.qd_prm = track_params(4, **track_kw)
        h = ctypes.c_void_p()
        _scheck(_lib.hcn_server_create(ctypes.byref(h), int(budget_bytes), float(qd_share), max_n,
                                       max_nslots, ctypes.byref(self.dd_prm),
                                       ctypes.byref(self.qd_prm), steps_per_round,
                                       1 if serial else 0))
        self.handle = h
        self._n = {}

    def now(self) -> float:
        return float(_lib.hcn_server_now(self.handle))

    def capacity(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _scheck(_lib.hcn_server_capacity(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def submit(self, rid: int, sys: System, gamma, x0: np.ndarray, t_arrival: float):
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(2, sys.P))
        x = np.ascontiguousarray(x0, dtype=np.float64)
        self._n[int(rid)] = (sys.n, sys.P)
        _scheck(_lib.hcn_server_submit(self.handle, int(rid), sys.handle, _np_ptr(g), _np_ptr(x),
                                       float(t_arrival)))

    def pump(self) -> int:
        return _scheck(_lib.hcn_server_pump(self.handle))

    def fetch(self):
        """One completed request as (id, x_out, result, t_arrival, t_admit, t_done) or None."""
        rid = ctypes.c_int64()
        ta, tb, tc = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        # sizes are known only after the id; fetch into the largest buffer
        x = np.zeros((4096, 2, 4))
        res = np.zeros(1, dtype=PATH_RESULT_DTYPE)
        got = _scheck(_lib.hcn_server_fetch(self.handle, ctypes.byref(rid), _np_ptr(x),
                                            _np_ptr(res), ctypes.byref(ta), ctypes.byref(tb),
                                            ctypes.byref(tc)))
        if not got:
            return None
        n, P = self._n.pop(rid.value)
        xo = x.reshape(-1)[:n * 2 * P].reshape(n, 2, P).copy()
        return rid.value, xo, res[0], ta.value, tb.value, tc.value

    def queued(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _scheck(_lib.hcn_server_queued(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def free(self):
        if self.handle:
            _lib.hcn_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
