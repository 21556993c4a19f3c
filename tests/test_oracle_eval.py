"""Pins of the oracle's evaluation and differentiation (plain definition).

* closed forms at special points: all ones (value sum c, partial sum a_k c),
  the imaginary unit and powers of two (dyadic: every product and sum is
  exact, so the oracle must agree bitwise with exact rational arithmetic);
* Table 1's four monomials: each partial is the product of the variables the
  table lists (the closed-form Speelpenning gradient);
* Euler's identity for homogeneous equations: sum_k x_k J_ik = d f_i;
* the Jacobian equals central finite differences of the oracle's own f in
  quad-double (h = 2^-70, error far below the check);
* the homotopy reduces to gamma g at t = 0 and to f at t = 1.
"""
import json
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from oracle import mpref as M
from paper_1501_06625_amd import systems as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _system(P, seed=3, N=6, n=6, M_=5, k=(1, 4), exps=(1, 2, 3)):
    rng = np.random.default_rng(seed)
    return S.random_system(rng, N, n, M_, k, exps, P)


@pytest.mark.parametrize("P", [2, 4])
def test_all_ones_point(P):
    s = _system(P)
    x = S.ones_point(s.n, P)
    f, J = O.eval_jac(s, x)
    with mpmath.workprec(320):
        for i in range(s.N):
            fi = mpmath.mpc(0)
            Ji = [mpmath.mpc(0)] * s.n
            for m, mon in s.monomials(i):
                c = M.mp_complex(s.coef[m])
                fi += c
                for v, e in mon:
                    Ji[v] += e * c
            assert abs(M.mp_complex(f[i]) - fi) <= 1e-28 * (1 + abs(fi))
            for k in range(s.n):
                assert abs(M.mp_complex(J[k, i]) - Ji[k]) <= 1e-28 * (1 + abs(Ji[k]))


def _dyadic_system(P, rng, N=5, n=5):
    units = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    eqs, coefs = [], []
    for _ in range(N):
        mons = []
        for _ in range(4):
            k = int(rng.integers(1, 4))
            vs = sorted(rng.choice(n, size=k, replace=False).tolist())
            mons.append([(v, int(rng.integers(1, 4))) for v in vs])
            c = np.zeros((2, P))
            re, im = units[int(rng.integers(0, 4))]
            c[0, 0], c[1, 0] = re, im
            coefs.append(c)
        eqs.append(mons)
    return S.system_from_monomials(N, n, P, eqs, np.array(coefs))


@pytest.mark.parametrize("P", [2, 4])
def test_dyadic_points_bitwise_exact(P):
    """x_l in {+-2^e, +-i 2^e}, c in {+-1, +-i}: all exact; compare the
    limbs with exact Gaussian-rational arithmetic."""
    rng = np.random.default_rng(21 + P)
    s = _dyadic_system(P, rng)
    xq = []
    x = np.zeros((s.n, 2, P))
    for j in range(s.n):
        e = int(rng.integers(-3, 4))
        sg = float(rng.choice([-1.0, 1.0]))
        if rng.integers(0, 2):
            x[j, 0, 0] = sg * 2.0 ** e
            xq.append((Fraction(sg * 2.0 ** e), Fraction(0)))
        else:
            x[j, 1, 0] = sg * 2.0 ** e
            xq.append((Fraction(0), Fraction(sg * 2.0 ** e)))

    def cm(a, b):
        return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])

    f, J = O.eval_jac(s, x)
    for i in range(s.N):
        fi = (Fraction(0), Fraction(0))
        Ji = [(Fraction(0), Fraction(0))] * s.n
        for m, mon in s.monomials(i):
            c = (Fraction(float(s.coef[m, 0, 0])), Fraction(float(s.coef[m, 1, 0])))
            t = c
            for v, e in mon:
                for _ in range(e):
                    t = cm(t, xq[v])
            fi = (fi[0] + t[0], fi[1] + t[1])
            for q, (v, e) in enumerate(mon):
                d = (c[0] * e, c[1] * e)
                for r, (w, g) in enumerate(mon):
                    for _ in range(g - (1 if r == q else 0)):
                        d = cm(d, xq[w])
                Ji[v] = (Ji[v][0] + d[0], Ji[v][1] + d[1])
        assert Fraction(float(f[i, 0, 0])) == fi[0] and np.all(f[i, 0, 1:] == 0)
        assert Fraction(float(f[i, 1, 0])) == fi[1] and np.all(f[i, 1, 1:] == 0)
        for k in range(s.n):
            assert Fraction(float(J[k, i, 0, 0])) == Ji[k][0]
            assert Fraction(float(J[k, i, 1, 0])) == Ji[k][1]


@pytest.mark.parametrize("P", [2, 4])
def test_table1_speelpenning_partials(P):
    fx = json.load(open(os.path.join(GOLDEN, "table1_monomials.json")))
    mons = fx["monomials"]
    n = 6
    one = np.zeros((2, P))
    one[0, 0] = 1.0
    eqs = [[[(v, 1) for v in m["vars"]]] for m in mons]
    s = S.system_from_monomials(len(mons), n, P, eqs, np.array([one] * len(mons)))
    rng = S.rng_for(9, P)
    x = S.random_unit_point(rng, n, P)
    f, J = O.eval_jac(s, x)
    xs = M.vec(x)
    tol = 1e-30 if P == 2 else 1e-62
    with mpmath.workprec(320):
        for i, m in enumerate(mons):
            val = mpmath.mpc(1)
            for v in m["vars"]:
                val *= xs[v]
            assert abs(M.mp_complex(f[i]) - val) <= tol
            for k in range(n):
                if str(k) in m["partials"]:
                    ref = mpmath.mpc(1)
                    for v in m["partials"][str(k)]:
                        ref *= xs[v]
                else:
                    ref = mpmath.mpc(0)
                assert abs(M.mp_complex(J[k, i]) - ref) <= tol, (i, k)


@pytest.mark.parametrize("P", [2, 4])
def test_euler_identity_homogeneous(P):
    rng = S.rng_for(8, P)
    deg = 4
    N = n = 7
    eqs = []
    for _ in range(N):
        mons = []
        for _ in range(6):
            k = int(rng.integers(1, 4))
            vs = sorted(rng.choice(n, size=k, replace=False).tolist())
            es = [1] * k
            for _ in range(deg - k):
                es[int(rng.integers(0, k))] += 1
            mons.append(list(zip(vs, es)))
        eqs.append(mons)
    coefs = S.unit_complex(rng.uniform(0, 6.28, N * 6), P)
    s = S.system_from_monomials(N, n, P, eqs, coefs)
    x = S.random_unit_point(rng, n, P)
    f, J = O.eval_jac(s, x)
    xs = M.vec(x)
    tol = 1e-29 if P == 2 else 1e-60
    with mpmath.workprec(320):
        for i in range(N):
            lhs = sum((xs[k] * M.mp_complex(J[k, i]) for k in range(n)), mpmath.mpc(0))
            assert abs(lhs - deg * M.mp_complex(f[i])) <= tol * 6 * deg


def test_jacobian_matches_finite_differences():
    """Central differences of the oracle's own f, in quad-double."""
    P = 4
    s = _system(P, seed=12)
    rng = S.rng_for(7, 1)
    x = S.random_unit_point(rng, s.n, P)
    f, J = O.eval_jac(s, x)
    h = 2.0 ** -70
    with mpmath.workprec(320):
        for k in range(s.n):
            for dirn, scale in ((0, 1), (1, 1j)):
                xp = x.copy()
                xm = x.copy()
                xp[k, dirn] = M.to_limbs(M.mp_real(x[k, dirn]) + h, P)
                xm[k, dirn] = M.to_limbs(M.mp_real(x[k, dirn]) - h, P)
                fp, _ = O.eval_jac(s, xp)
                fm, _ = O.eval_jac(s, xm)
                for i in range(s.N):
                    fd = (M.mp_complex(fp[i]) - M.mp_complex(fm[i])) / (2 * h)
                    ref = M.mp_complex(J[k, i]) * scale
                    assert abs(fd - ref) <= 1e-30 * (1 + abs(ref)), (k, i, dirn)


@pytest.mark.parametrize("P", [2, 4])
def test_homotopy_endpoints(P):
    s = _system(P, seed=5)
    g = O.total_degree_start(s)
    rng = S.rng_for(7, 2)
    x = S.random_unit_point(rng, s.n, P)
    gam = S.random_unit_gamma(rng, P)
    f, Jf = O.eval_jac(s, x)
    gv, Jg = O.eval_jac(g, x)
    h1, Jh1 = O.eval_h(s, g, gam, 1, 1.0, x)
    assert np.array_equal(h1, f) and np.array_equal(Jh1, Jf)
    h0, Jh0 = O.eval_h(s, g, gam, 1, 0.0, x)
    gm = M.mp_complex(gam)
    tol = 1e-30 if P == 2 else 1e-62
    for i in range(s.N):
        assert abs(M.mp_complex(h0[i]) - gm * M.mp_complex(gv[i])) <= tol * 10
    # start system: g_i = x_i^{d_i} - 1 with d_i the total degree of f_i
    d = S.degrees(s)
    xs = M.vec(x)
    for i in range(s.N):
        assert abs(M.mp_complex(gv[i]) - (xs[i] ** int(d[i]) - 1)) <= tol * 10
        assert abs(M.mp_complex(Jg[i, i]) - int(d[i]) * xs[i] ** int(d[i] - 1)) <= tol * 10 * d[i]
