"""mpmath helpers for pinning the oracle (320-bit arithmetic).

TEST INFRASTRUCTURE ONLY.  Conversions between limb arrays and mpmath
numbers, matrix helpers for the QR invariants, and input builders that need
exact arithmetic (planted roots).  Nothing here is used by the GPU path.
"""
from __future__ import annotations

import mpmath
import numpy as np

PREC = 320
# tests compare at this precision throughout
mpmath.mp.prec = PREC


def mp_real(limbs) -> mpmath.mpf:
    with mpmath.workprec(PREC):
        s = mpmath.mpf(0)
        for d in np.asarray(limbs, dtype=np.float64).ravel().tolist():
            s += mpmath.mpf(d)
        return s


def mp_complex(z) -> mpmath.mpc:
    z = np.asarray(z, dtype=np.float64)
    with mpmath.workprec(PREC):
        return mpmath.mpc(mp_real(z[0]), mp_real(z[1]))


def to_limbs(x, P: int):
    out = []
    with mpmath.workprec(PREC):
        r = mpmath.mpf(x)
        for _ in range(P):
            d = float(r)
            out.append(d)
            r -= mpmath.mpf(d)
    return out


def complex_limbs(z, P: int) -> np.ndarray:
    z = mpmath.mpc(z)
    return np.array([to_limbs(z.real, P), to_limbs(z.imag, P)])


def vec(a) -> list:
    """[len][2][P] limbs -> list of mpc."""
    a = np.asarray(a)
    return [mp_complex(a[i]) for i in range(a.shape[0])]


def colmajor(J) -> mpmath.matrix:
    """[n][N][2][P] column-major limbs -> N x n mpmath matrix."""
    J = np.asarray(J)
    n, N = J.shape[0], J.shape[1]
    with mpmath.workprec(PREC):
        M = mpmath.matrix(N, n)
        for k in range(n):
            for i in range(N):
                M[i, k] = mp_complex(J[k, i])
    return M


def rel_err(a, b) -> float:
    """|a - b| / |b| (|a - b| when b == 0)."""
    with mpmath.workprec(PREC):
        d = abs(a - b)
        s = abs(b)
        return float(d / s) if s != 0 else float(d)


def eval_system(sys, x):
    """f and J by the textbook formulas, at 320 bits (x: list of mpc)."""
    with mpmath.workprec(PREC):
        f = [mpmath.mpc(0)] * sys.N
        J = [[mpmath.mpc(0)] * sys.n for _ in range(sys.N)]
        for i in range(sys.N):
            acc = mpmath.mpc(0)
            for m in range(int(sys.eq_ptr[i]), int(sys.eq_ptr[i + 1])):
                a, b = int(sys.mon_ptr[m]), int(sys.mon_ptr[m + 1])
                pairs = list(zip(sys.var[a:b].tolist(), sys.exp[a:b].tolist()))
                c = mp_complex(sys.coef[m])
                term = c
                for v, e in pairs:
                    term *= x[v] ** e
                acc += term
                for q, (v, e) in enumerate(pairs):
                    d = c * e * x[v] ** (e - 1)
                    for r, (w, g) in enumerate(pairs):
                        if r != q:
                            d *= x[w] ** g
                    J[i][v] += d
            f[i] = acc
        return f, J


def planted_constant_terms(sys, root):
    """Append a constant term to every equation so that `root` ([n][2][P])
    is a root to within the rounding of the constant."""
    from types import SimpleNamespace
    P = sys.P
    xs = vec(root)
    with mpmath.workprec(PREC):
        consts = []
        for i in range(sys.N):
            acc = mpmath.mpc(0)
            for m in range(int(sys.eq_ptr[i]), int(sys.eq_ptr[i + 1])):
                a, b = int(sys.mon_ptr[m]), int(sys.mon_ptr[m + 1])
                term = mp_complex(sys.coef[m])
                for v, e in zip(sys.var[a:b].tolist(), sys.exp[a:b].tolist()):
                    term *= xs[v] ** e
                acc += term
            consts.append(-acc)
    eq_ptr, mon_ptr, coefs = [0], [0], []
    var, exp = [], []
    for i in range(sys.N):
        for m in range(int(sys.eq_ptr[i]), int(sys.eq_ptr[i + 1])):
            a, b = int(sys.mon_ptr[m]), int(sys.mon_ptr[m + 1])
            var.extend(sys.var[a:b].tolist())
            exp.extend(sys.exp[a:b].tolist())
            mon_ptr.append(len(var))
            coefs.append(np.asarray(sys.coef[m]))
        mon_ptr.append(len(var))
        coefs.append(complex_limbs(consts[i], P))
        eq_ptr.append(len(mon_ptr) - 1)
    return SimpleNamespace(N=sys.N, n=sys.n, P=P,
                           eq_ptr=np.asarray(eq_ptr, dtype=np.int32),
                           mon_ptr=np.asarray(mon_ptr, dtype=np.int32),
                           var=np.asarray(var, dtype=np.int32),
                           exp=np.asarray(exp, dtype=np.int32),
                           coef=np.asarray(coefs, dtype=np.float64))


def closed_form_endpoint(gamma, c, d: int, x0, steps: int = 4000):
    """Endpoint at t = 1 of the path x(t)^d = (gamma (1-t) + t c) / (gamma (1-t) + t)
    that starts at x0 (a d-th root of unity): follow the right-hand side on a
    fine t-grid and take at every point the d-th root nearest to the previous
    one."""
    with mpmath.workprec(PREC):
        x = mpmath.mpc(x0)
        g = mpmath.mpc(gamma)
        c = mpmath.mpc(c)
        for s in range(1, steps + 1):
            t = mpmath.mpf(s) / steps
            w = (g * (1 - t) + t * c) / (g * (1 - t) + t)
            r = mpmath.root(w, d)
            best = None
            for j in range(d):
                cand = r * mpmath.expjpi(mpmath.mpf(2 * j) / d)
                if best is None or abs(cand - x) < abs(best - x):
                    best = cand
            x = best
        # polish on the exact equation x^d = c
        for _ in range(8):
            x = x - (x ** d - c) / (d * x ** (d - 1))
        return x
