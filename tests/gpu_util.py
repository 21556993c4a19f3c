"""Shared helpers for the GPU parity tests (tolerances and scales)."""
import numpy as np

# reduction / solve gates: 1e-28 (DD), 1e-58 (QD)
GATE = {2: 1e-28, 4: 1e-58}
# working unit roundoff of the formats
UNIT = {2: 2.0 ** -104, 4: 2.0 ** -209}


def limb_diff(a, b):
    """Complex difference of two limb arrays [..., 2, P] as complex128; the
    leading limbs are subtracted first (exact when they are close)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = (a[..., 0] - b[..., 0])
    for j in range(1, a.shape[-1]):
        d = d + (a[..., j] - b[..., j])
    return d[..., 0] + 1j * d[..., 1]


def lead_complex(a):
    a = np.asarray(a)
    return a[..., 0, 0] + 1j * a[..., 1, 0]


def term_scales(ps, x):
    """S = sum of |terms| for every output of f and J at x (double is enough
    for a scale): Sf [N], SJ [n][N]."""
    xa = np.abs(lead_complex(x))
    Sf = np.zeros(ps.N)
    SJ = np.zeros((ps.n, ps.N))
    for i in range(ps.N):
        for m in range(int(ps.eq_ptr[i]), int(ps.eq_ptr[i + 1])):
            a, b = int(ps.mon_ptr[m]), int(ps.mon_ptr[m + 1])
            vs = ps.var[a:b]
            es = ps.exp[a:b]
            c = abs(lead_complex(ps.coef[m]))
            term = c * np.prod(xa[vs] ** es) if b > a else c
            Sf[i] += term
            for v, e in zip(vs, es):
                others = np.prod([xa[w] ** g for w, g in zip(vs, es) if w != v]) if b - a > 1 else 1.0
                SJ[v, i] += c * e * xa[v] ** (e - 1) * others
    return Sf, SJ


def random_points(rng, B, n, P):
    from paper_1501_06625_amd import systems as S
    return S.unit_complex(rng.uniform(0, 2 * np.pi, B * n), P).reshape(B, n, 2, P)


def update_bound(tol, dx_norm, x_ref, P):
    """Bound on |x_gpu - x_oracle| after one Newton update x + dx: the
    solves' difference tol |dx|, plus the rounding of the sum x + dx on each
    side (at most 2 UNIT |x|, UNIT at least three units of the last place of
    the accurate double-word / quad-word sum)."""
    return tol * dx_norm + 2.0 * UNIT[P] * max(1.0, float(np.abs(lead_complex(x_ref)).max()))
