"""Pins of the oracle's DD/QD arithmetic against exact rational arithmetic
and 400-bit mpmath (independent of the oracle's own code).

Bounds, with u = 2^-53:
* error-free transformations are exact (checked with fractions.Fraction);
* DD (Joldes, Muller & Popescu 2017): sum 3u^2, product 4u^2, product by a
  double 2u^2, quotient 15u^2; square root (one Newton correction of the
  double square root) 4u^2;
* QD (Hida, Li & Bailey 2001): results within 8u^4 (2^-209) relative error
  (square root 16u^4), including sums under heavy cancellation.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from oracle import mpref as M

U = 2.0 ** -53
BOUND = {
    2: dict(add=3 * U ** 2, mul=4 * U ** 2, mul_d=2 * U ** 2, div=15 * U ** 2, sqrt=4 * U ** 2),
    4: dict(add=8 * U ** 4, mul=8 * U ** 4, mul_d=8 * U ** 4, div=8 * U ** 4, sqrt=16 * U ** 4),
}


def _rand_numbers(rng, P, cnt, spread=20):
    out = np.zeros((cnt, P))
    with mpmath.workprec(400):
        for q in range(cnt):
            x = mpmath.mpf(rng.uniform(-1, 1)) * mpmath.mpf(2) ** int(rng.integers(-spread, spread))
            for sh in (-60, -125, -185, -240):
                x += mpmath.mpf(rng.uniform(-1, 1)) * mpmath.mpf(2) ** sh * x
            out[q] = M.to_limbs(x, P)
    return out


def _exact(op, x, y):
    if op == "add":
        return x + y
    if op == "sub":
        return x - y
    if op == "mul":
        return x * y
    if op == "div":
        return x / y
    raise ValueError(op)


def _max_rel(P, a, b, r, op):
    worst = 0.0
    with mpmath.workprec(400):
        for q in range(a.shape[0]):
            x = M.mp_real(a[q])
            if op == "sqrt":
                ex = mpmath.sqrt(x)
            elif op == "mul_d":
                ex = x * mpmath.mpf(float(b[q]))
            else:
                ex = _exact(op, x, M.mp_real(b[q]))
            e = abs(M.mp_real(r[q]) - ex)
            worst = max(worst, float(e / abs(ex)) if ex != 0 else float(e))
    return worst


def test_eft_exact_fraction():
    rng = np.random.default_rng(11)
    a = rng.standard_normal(4000) * np.exp2(rng.integers(-40, 40, 4000))
    b = rng.standard_normal(4000) * np.exp2(rng.integers(-40, 40, 4000))
    ts = O.elementwise("two_sum", 2, a, b)
    tp = O.elementwise("two_prod", 2, a, b)
    big = np.where(np.abs(a) >= np.abs(b), a, b)
    small = np.where(np.abs(a) >= np.abs(b), b, a)
    fs = O.elementwise("fast_two_sum", 2, big, small)
    for q in range(a.size):
        A, B = Fraction(float(a[q])), Fraction(float(b[q]))
        assert Fraction(float(ts[q, 0])) + Fraction(float(ts[q, 1])) == A + B
        assert ts[q, 0] == float(a[q] + b[q])
        assert Fraction(float(tp[q, 0])) + Fraction(float(tp[q, 1])) == A * B
        assert tp[q, 0] == float(a[q] * b[q])
        assert Fraction(float(fs[q, 0])) + Fraction(float(fs[q, 1])) == A + B


@pytest.mark.parametrize("P", [2, 4])
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_binary_ops_within_bound(P, op):
    rng = np.random.default_rng(100 + P * 10 + len(op))
    a = _rand_numbers(rng, P, 600)
    b = _rand_numbers(rng, P, 600)
    r = O.elementwise(op, P, a, b)
    bound = BOUND[P]["add" if op == "sub" else op]
    assert _max_rel(P, a, b, r, op) <= bound


@pytest.mark.parametrize("P", [2, 4])
def test_sum_under_cancellation(P):
    """b = -a + c * 2^-s: the accurate sums keep a relative error bound."""
    rng = np.random.default_rng(7 + P)
    a = _rand_numbers(rng, P, 600)
    c = _rand_numbers(rng, P, 600)
    b = np.zeros_like(a)
    with mpmath.workprec(400):
        for q in range(a.shape[0]):
            s = int(rng.integers(1, 50 * P))
            b[q] = M.to_limbs(-M.mp_real(a[q]) + M.mp_real(c[q]) * mpmath.mpf(2) ** -s, P)
    r = O.elementwise("add", P, a, b)
    assert _max_rel(P, a, b, r, "add") <= BOUND[P]["add"]


def test_double_double_add_commutes_bitwise():
    """The double-double sum does not depend on the order of its operands,
    bit for bit (each of its error-free sums yields the same pair either
    way), also under cancellation, with signed zeros and with exact sums:
    the GPU's butterfly reductions in FP64 and DD rely on it to skip the
    lane-order select."""
    rng = np.random.default_rng(12)
    a = _rand_numbers(rng, 2, 400)
    b = _rand_numbers(rng, 2, 400)
    b[:100] = -a[:100]                       # exact cancellation
    b[100:200, 0] = -a[100:200, 0]           # leading limbs cancel
    a[200:220] = 0.0
    b[210:230] = -0.0
    b[230:260] = a[230:260] * 2.0 ** -30     # different magnitudes
    for x, y in ((a, b), (b, a)):
        r1 = O.elementwise("add", 2, x, y)
        r2 = O.elementwise("add", 2, y, x)
        assert np.array_equal(r1.view(np.uint64), r2.view(np.uint64))
    # the plain double sum as well (the degenerate case P = 1)
    r1 = O.elementwise("add", 1, a[:, :1], b[:, :1])
    r2 = O.elementwise("add", 1, b[:, :1], a[:, :1])
    assert np.array_equal(r1.view(np.uint64), r2.view(np.uint64))


@pytest.mark.parametrize("P", [2, 4])
def test_mul_d_and_sqrt(P):
    rng = np.random.default_rng(33 + P)
    a = _rand_numbers(rng, P, 600)
    d = rng.uniform(-8, 8, 600)
    r = O.elementwise("mul_d", P, a, d)
    assert _max_rel(P, a, d, r, "mul_d") <= BOUND[P]["mul_d"]
    pos = np.where(a[:, :1] < 0, -a, a)
    r = O.elementwise("sqrt", P, pos)
    assert _max_rel(P, pos, None, r, "sqrt") <= BOUND[P]["sqrt"]


@pytest.mark.parametrize("P", [2, 4])
def test_special_values(P):
    z = np.zeros((1, P))
    one = np.zeros((1, P))
    one[0, 0] = 1.0
    two = 2 * one
    # x + (-x) == 0, 1 * x == x, x / 1 == x, sqrt(4) == 2, sqrt(0) == 0
    rng = np.random.default_rng(5)
    x = _rand_numbers(rng, P, 50)
    assert np.all(O.elementwise("add", P, x, -x) == 0)
    assert np.array_equal(O.elementwise("mul", P, x, np.repeat(one, 50, 0)), x)
    assert np.array_equal(O.elementwise("div", P, x, np.repeat(one, 50, 0)), x)
    assert np.array_equal(O.elementwise("sqrt", P, 4 * one), two)
    assert np.array_equal(O.elementwise("sqrt", P, z), z)
    assert np.array_equal(O.elementwise("add", P, x, np.zeros_like(x)), x)
    # exact powers of two multiply exactly
    assert np.array_equal(O.elementwise("mul", P, x, np.repeat(two, 50, 0)), 2 * x)
    # limbs of results are non-overlapping: |lo| <= ulp(hi)/2
    y = _rand_numbers(rng, P, 200)
    for op in ("add", "mul", "div"):
        r = O.elementwise(op, P, x[np.arange(200) % 50], y)
        for q in range(200):
            for j in range(P - 1):
                if r[q, j] != 0:
                    assert abs(r[q, j + 1]) <= np.spacing(abs(r[q, j])) / 2 * (1 + 1e-15)


@pytest.mark.parametrize("P", [2, 4])
def test_complex_ops(P):
    rng = np.random.default_rng(77 + P)
    cnt = 200
    a = _rand_numbers(rng, P, 2 * cnt).reshape(cnt, 2, P)
    b = _rand_numbers(rng, P, 2 * cnt).reshape(cnt, 2, P)
    cm = O.elementwise("cmul", P, a, b)
    cj = O.elementwise("cmul_conj", P, a, b)
    n2 = O.elementwise("cnorm2", P, a)
    ca = O.elementwise("cadd", P, a, b)
    tol = 8 * BOUND[P]["add"] + 8 * BOUND[P]["mul"]
    with mpmath.workprec(400):
        for q in range(cnt):
            x, y = M.mp_complex(a[q]), M.mp_complex(b[q])
            s = (abs(x.real) + abs(x.imag)) * (abs(y.real) + abs(y.imag))
            assert abs(M.mp_complex(cm[q]) - x * y) <= tol * s
            assert abs(M.mp_complex(cj[q]) - mpmath.conj(x) * y) <= tol * s
            assert abs(M.mp_real(n2[q]) - abs(x) ** 2) <= tol * abs(x) ** 2
            assert abs(M.mp_complex(ca[q]) - (x + y)) <= tol * (abs(x) + abs(y))
    # the imaginary unit squares to -1 exactly
    i = np.zeros((1, 2, P))
    i[0, 1, 0] = 1.0
    m1 = O.elementwise("cmul", P, i, i)
    assert m1[0, 0, 0] == -1.0 and np.all(m1[0, 0, 1:] == 0) and np.all(m1[0, 1] == 0)


@pytest.mark.parametrize("P", [2, 4])
def test_products_by_one_and_small_scalings_exact(P):
    """Facts the uniform monomial kernel relies on: a complex product by 1
    (on either side) returns a normalised operand bit for bit, also a
    product's result, and the product by the double 1 or 2 equals the operand
    or its exact double (so scaling by an exponent 1 or 2 through mul_d
    changes no bit)."""
    rng = np.random.default_rng(2024 + P)
    cnt = 300
    a = _rand_numbers(rng, P, 2 * cnt).reshape(cnt, 2, P)
    a[:20] = 0.0                       # zeros and single-limb values too
    a[20:40, :, 1:] = 0.0
    one = np.zeros((cnt, 2, P))
    one[:, 0, 0] = 1.0
    a[40:60, :, 2:] = 0.0
    assert np.array_equal(O.elementwise("cmul", P, a, one), a)
    assert np.array_equal(O.elementwise("cmul", P, one, a), a)
    b = _rand_numbers(rng, P, 2 * cnt).reshape(cnt, 2, P)
    ab = O.elementwise("cmul", P, a, b)
    assert np.array_equal(O.elementwise("cmul", P, ab, one), ab)
    re = a[:, 0, :].copy()
    assert np.array_equal(O.elementwise("mul_d", P, re, np.ones(cnt)), re)
    assert np.array_equal(O.elementwise("mul_d", P, re, np.full(cnt, 2.0)), 2.0 * re)
