"""Algorithmic FP64 operation counts of the kernels (a fused multiply-add
counts as two operations; comparisons and selects are not counted).

Per real operation (double-double, from the operation sequences of the
arithmetic layer): TwoSum 6, FastTwoSum 3, TwoProd 3; add 20, mul 12,
mul by a double 8, div 16, sqrt 12.  Quad-double: renormalisation 48, add
144, mul 130, mul by a double 85, div 739, sqrt 2421.  Complex: add 2A,
mul 4M + 2A, |z|^2 2M + A, real scaling 2M, scaling by a double 2D.

Reductions are counted as a sequential algorithm needs them (n terms:
n - 1 additions), not as the butterflies compute them.
"""
from __future__ import annotations

import numpy as np

REAL = {
    1: dict(add=1, mul=1, mul_d=1, div=1, sqrt=1),
    2: dict(add=20, mul=12, mul_d=8, div=16, sqrt=12),
    4: dict(add=144, mul=130, mul_d=85, div=739, sqrt=2421),
}


def complex_costs(P: int) -> dict:
    r = REAL[P]
    return dict(cadd=2 * r["add"], cmul=4 * r["mul"] + 2 * r["add"],
                cnorm2=2 * r["mul"] + r["add"], cscale=2 * r["mul"], cscale_d=2 * r["mul_d"],
                add=r["add"], sqrt=r["sqrt"], div=r["div"])


def eval_monomials(ps, P: int) -> int:
    """Reverse-mode evaluation of every monomial with its coefficient:
    3k - 3 complex products for k >= 2 (3k - 5 for the product and its
    gradient, two more to carry the coefficient), powers for exponents above
    one, and a scaling by exponents above two (doubling is exact and not
    counted)."""
    c = complex_costs(P)
    total = 0
    for m in range(ps.nmon):
        a, b = int(ps.mon_ptr[m]), int(ps.mon_ptr[m + 1])
        k = b - a
        if k == 0:
            continue
        es = [int(e) for e in ps.exp[a:b]]
        hi = [e for e in es if e >= 2]
        cm = sum(e - 2 for e in hi) + max(len(hi) - 1, 0) + (1 if hi else 0)
        cm += 1 if k == 1 else 3 * k - 3
        total += cm * c["cmul"] + sum(1 for e in es if e > 2) * c["cscale_d"]
    return total


def eval_values(ps, P: int) -> int:
    """Values only (the residual of the mixed-precision step): k - 1 complex
    products for the product, the powers, the common factor and the
    coefficient."""
    c = complex_costs(P)
    total = 0
    for m in range(ps.nmon):
        a, b = int(ps.mon_ptr[m]), int(ps.mon_ptr[m + 1])
        k = b - a
        if k == 0:
            continue
        es = [int(e) for e in ps.exp[a:b]]
        hi = [e for e in es if e >= 2]
        cm = sum(e - 2 for e in hi) + max(len(hi) - 1, 0) + (1 if hi else 0)
        cm += 1 if k == 1 else k  # (k - 1) for S, one for c' S
        total += cm * c["cmul"]
    return total


def eval_sums_values(ps, P: int) -> int:
    c = complex_costs(P)
    return int(sum(max(int(ps.eq_ptr[i + 1] - ps.eq_ptr[i]) - 1, 0) for i in range(ps.N))) * c["cadd"]


def mixed_step(ps, P: int) -> dict:
    """One mixed-precision iteration: the residual in P, the Jacobian and the
    solve in FP64, the update in P."""
    d = dict(residual=eval_values(ps, P) + eval_sums_values(ps, P),
             jacobian=eval_monomials(ps, 1) + eval_sums(ps, 1),
             mgs=mgs_solve(ps.N, ps.n, 1), update=newton_update(ps.n, P))
    d["total"] = sum(d.values())
    return d


def eval_sums(ps, P: int) -> int:
    """Summation: every output with L contributions costs L - 1 additions."""
    c = complex_costs(P)
    N, n = ps.N, ps.n
    counts = np.zeros(n * N, dtype=np.int64)
    for i in range(N):
        for m in range(int(ps.eq_ptr[i]), int(ps.eq_ptr[i + 1])):
            for v in ps.var[int(ps.mon_ptr[m]):int(ps.mon_ptr[m + 1])]:
                counts[int(v) * N + i] += 1
    adds = int(np.maximum(counts - 1, 0).sum())
    adds += int(sum(max(int(ps.eq_ptr[i + 1] - ps.eq_ptr[i]) - 1, 0) for i in range(N)))
    return adds * c["cadd"]


def mgs_solve(N: int, n: int, P: int) -> int:
    """MGS on [A | b] (n+1 columns) and back substitution."""
    c = complex_costs(P)
    cmadd = c["cmul"] + c["cadd"]
    per_k = N * c["cnorm2"] + (N - 1) * c["add"] + c["sqrt"] + c["div"] + N * c["cscale"]
    per_kj = N * c["cmul"] + (N - 1) * c["cadd"] + N * cmadd
    pairs = n * (n + 1) // 2
    back = n * c["cscale"] + (n * (n - 1) // 2) * cmadd
    return n * per_k + pairs * per_kj + back


def newton_update(n: int, P: int) -> int:
    return n * complex_costs(P)["cadd"]


def newton_step(ps, P: int) -> dict:
    d = dict(eval_monomials=eval_monomials(ps, P), eval_sums=eval_sums(ps, P),
             mgs=mgs_solve(ps.N, ps.n, P) + newton_update(ps.n, P))
    d["total"] = sum(d.values())
    return d
