"""Pins of the paper's two benchmark families as built here (Section 4),
and of the oracle's complex-double mode.

* cyclic n-roots (Section 4.2): the root found by substitution
  (x_j = w^j for odd n, e^{i pi/n} w^j for even n) makes every equation
  vanish, so the oracle's residual there is at rounding level; Euler's
  identity sum_k x_k df_i/dx_k = i f_i holds for the homogeneous equations
  f_1 .. f_{n-1} at any point; the equation sizes are those of the formula.
* minor expansions (Section 4.1): each equation is det(K_i^T X) for the
  pattern matrix X of the unknowns; the oracle's value at a point equals
  the determinant formed directly (to the double-precision rounding of the
  coefficients, which are double minors).
* complex double (P = 1): the oracle's arithmetic is IEEE double (each
  operation correctly rounded), its MGS solves a random system to the
  backward-stability bound, and its Newton step is the double version of
  the DD one.
"""
import mpmath
import numpy as np
import pytest

from oracle import mpref as M
from oracle import oracle as O
from paper_1501_06625_amd import systems as S

TOL = {1: 1e-14, 2: 1e-28, 4: 1e-58}


@pytest.mark.parametrize("n", [5, 8, 13, 16])
@pytest.mark.parametrize("P", [2, 4])
def test_cyclic_root_residual(n, P):
    ps = S.cyclic_system(n, P)
    assert ps.N == n and ps.nmon == n * (n - 1) + 2
    x = S.cyclic_root(n, P)
    f, _ = O.eval_jac(ps, x)
    # each f_i sums n terms of modulus one
    res = np.abs(f[:, :, 0]).max()
    assert res <= n * TOL[P], res


@pytest.mark.parametrize("n", [6, 9])
def test_cyclic_euler_identity(n):
    P = 2
    ps = S.cyclic_system(n, P)
    x = S.random_unit_point(S.rng_for(4, n), n, P)
    f, J = O.eval_jac(ps, x)
    xs = M.vec(x)
    for i in range(n - 1):
        lhs = sum(xs[k] * M.mp_complex(J[k, i]) for k in range(n))
        rhs = (i + 1) * M.mp_complex(f[i])
        assert abs(lhs - rhs) <= 50 * n * n * TOL[P]


def test_cyclic_structure():
    n = 7
    ps = S.cyclic_system(n, 2)
    for i in range(n - 1):
        mons = list(ps.monomials(i))
        assert len(mons) == n and all(len(m) == i + 1 for _, m in mons)
        # the windows of consecutive indices mod n, one starting at each j
        starts = sorted(m[0][0] for _, m in mons)
        assert starts == list(range(n))
    last = list(ps.monomials(n - 1))
    assert len(last) == 2 and len(last[0][1]) == n and last[1][1] == []


def _pattern_matrix(m, p, k, x):
    """X (m+p) x p with its pivots, the first k unknowns from x (mpc) and
    zeros elsewhere."""
    X = mpmath.matrix(m + p, p)
    for c in range(p):
        X[c, c] = 1
    for q, (r, c) in enumerate(S.pieri_variables(m, p)[:k]):
        X[r, c] = x[q]
    return X


@pytest.mark.parametrize("m,p,k", [(2, 2, 4), (3, 2, 5), (3, 3, 7)])
def test_determinantal_equations_are_determinants(m, p, k):
    ps = S.determinantal_system(m, p, k, seed=1, P=2)
    assert ps.N == k and ps.n == k
    assert max(int(ps.mon_ptr[q + 1] - ps.mon_ptr[q]) for q in range(ps.nmon)) <= p
    rng = S.rng_for(5, 1)
    K = rng.standard_normal((k, m + p, p)) + 1j * rng.standard_normal((k, m + p, p))
    x = S.random_unit_point(S.rng_for(4, 77 + k), k, 2)
    f, _ = O.eval_jac(ps, x)
    X = _pattern_matrix(m, p, k, M.vec(x))
    for i in range(k):
        Ki = mpmath.matrix([[complex(K[i, r, c]) for c in range(p)] for r in range(m + p)])
        ref = mpmath.det(Ki.T * X)
        assert abs(M.mp_complex(f[i]) - ref) <= 1e-12 * max(1.0, abs(ref))


def test_determinantal_pieri_order():
    # the example of Section 4.1: m = p = 2, the last column first
    assert S.pieri_variables(2, 2) == [(2, 1), (3, 1), (1, 0), (2, 0)]


# ---------------------------------------------------------------------------
# complex double (P = 1)
# ---------------------------------------------------------------------------

def test_double_arithmetic_is_ieee():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((50, 1)) * 10.0 ** rng.integers(-5, 5, (50, 1))
    b = rng.standard_normal((50, 1))
    assert np.array_equal(O.elementwise("add", 1, a, b), a + b)
    assert np.array_equal(O.elementwise("mul", 1, a, b), a * b)
    assert np.array_equal(O.elementwise("div", 1, a, b), a / b)
    assert np.array_equal(O.elementwise("sqrt", 1, np.abs(a)), np.sqrt(np.abs(a)))
    za = rng.standard_normal((20, 2, 1))
    zb = rng.standard_normal((20, 2, 1))
    out = O.elementwise("cmul", 1, za, zb)
    re = za[:, 0, 0] * zb[:, 0, 0] - za[:, 1, 0] * zb[:, 1, 0]
    im = za[:, 0, 0] * zb[:, 1, 0] + za[:, 1, 0] * zb[:, 0, 0]
    assert np.array_equal(out[:, 0, 0], re) and np.array_equal(out[:, 1, 0], im)


def test_double_mgs_backward_stable():
    rng = np.random.default_rng(4)
    N, n = 30, 20
    A = rng.standard_normal((n, N, 2, 1))
    b = rng.standard_normal((N, 2, 1))
    rc, dx, Q, R, _ = O.mgs_solve(1, A, b)
    assert rc == 0
    Ac = A[:, :, 0, 0].T + 1j * A[:, :, 1, 0].T
    bc = b[:, 0, 0] + 1j * b[:, 1, 0]
    xc = dx[:, 0, 0] + 1j * dx[:, 1, 0]
    ref = np.linalg.lstsq(Ac, bc, rcond=None)[0]
    kappa = np.linalg.cond(Ac)
    assert np.abs(xc - ref).max() <= 16 * n * kappa * 2.0 ** -53 * np.abs(ref).max()


def test_double_newton_converges_to_planted_root():
    rng = S.rng_for(5, 30)
    base = S.random_system(rng, 6, 6, 6, (2, 4), (1, 2), 2)
    root = S.random_unit_point(rng, 6, 2)
    f2 = M.planted_constant_terms(base, root)
    f1 = S.PolySystem(N=f2.N, n=f2.n, P=1, eq_ptr=f2.eq_ptr, mon_ptr=f2.mon_ptr, var=f2.var,
                      exp=f2.exp, coef=np.ascontiguousarray(f2.coef[:, :, :1]))
    x = np.ascontiguousarray(root[:, :, :1]).copy()
    x[:, 0, 0] += 1e-4 * rng.standard_normal(6)
    for _ in range(6):
        rc, x, norms = O.newton_step(f1, None, None, 1, 1.0, x)
        assert rc == 0
    err = np.abs((x[:, 0, 0] - root[:, 0, 0]) + 1j * (x[:, 1, 0] - root[:, 1, 0])).max()
    assert err <= 1e-13


def test_finite_roots_variant():
    """The finite-roots variant of a random system: x = 1 is a root (the
    oracle's residual there is at rounding level), every equation holds the
    pure power of its own variable at its degree, and total-degree paths of
    a small such system end at finite, refined roots (the literal system's
    end at the step limit or shrink below the smallest step)."""
    P = 2
    base = S.batch_systems(1, seed=11, P=P, n_range=(10, 10))[0]
    fin = S.with_finite_roots(base, 3)
    degs = S.degrees(base)
    assert np.array_equal(S.degrees(fin), degs)
    for i in range(fin.N):
        mons = [m for _, m in fin.monomials(i)]
        assert [(i, int(degs[i]))] in mons and [] in mons
    f, _ = O.eval_jac(fin, S.ones_point(fin.n, P))
    assert np.abs(f[:, :, 0]).max() <= 100 * TOL[P]
    rng = S.rng_for(9, 77)
    gam = S.random_unit_gamma(rng, P)
    g = O.total_degree_start(fin)
    for _ in range(2):
        x0 = S.start_solution(rng, degs, P)
        _, r = O.track(fin, g, gam, 1, x0, predictor_order=4)
        assert r.status == O.OK and r.end_status == O.OK and r.steps < 1500
