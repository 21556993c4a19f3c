"""Seeded synthetic polynomial systems and points (input generation only).

This module draws the random inputs that both the GPU path and the CPU
oracle consume.  It holds none of the method's arithmetic: it only draws
supports, exponents and angles, and rounds unit complex numbers to
double-double / quad-double limbs with mpmath at 320 bits.

Input format (the fully expanded distributed representation of a list of
polynomials, Section 3.1 "Accelerated Predictor-Corrector"):

* equations ``i = 0..N-1`` are a CSR over monomials (``eq_ptr``),
* monomials are a CSR over (variable, exponent) pairs (``mon_ptr``,
  ``var``, ``exp``); a monomial with no pair is a constant term,
* ``coef`` is ``[nmon][2][P]`` float64: real limbs then imaginary limbs,
  most significant limb first, ``P = 2`` (double-double) or ``4``
  (quad-double).

Recipes follow the workloads of the path tracker: random dense systems of
products of distinct variables with small exponents and unit-circle
coefficients, and sparse low-degree systems where linear algebra
dominates (Section 1, the discussion of sparse versus dense systems).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import mpmath
import numpy as np

DD = 2
QD = 4

_MP_PREC = 320


@dataclasses.dataclass
class PolySystem:
    """A polynomial system in the CSR tables described in the module doc."""

    N: int
    n: int
    P: int
    eq_ptr: np.ndarray   # int32 [N+1]
    mon_ptr: np.ndarray  # int32 [nmon+1]
    var: np.ndarray      # int32 [npairs]
    exp: np.ndarray      # int32 [npairs]
    coef: np.ndarray     # float64 [nmon][2][P]
    name: str = ""

    @property
    def nmon(self) -> int:
        return int(self.mon_ptr.shape[0] - 1)

    def with_precision(self, P: int, coef: np.ndarray) -> "PolySystem":
        return dataclasses.replace(self, P=P, coef=coef)

    def monomials(self, i: int):
        """Yield (coef_index, [(var, exp), ...]) for equation i."""
        for m in range(int(self.eq_ptr[i]), int(self.eq_ptr[i + 1])):
            a, b = int(self.mon_ptr[m]), int(self.mon_ptr[m + 1])
            yield m, list(zip(self.var[a:b].tolist(), self.exp[a:b].tolist()))


# ---------------------------------------------------------------------------
# limb rounding (greedy: each limb is the double nearest to what is left)
# ---------------------------------------------------------------------------

def mp_to_limbs(x, P: int) -> List[float]:
    """Round an mpmath real to P non-overlapping double limbs."""
    out = []
    with mpmath.workprec(_MP_PREC):
        r = mpmath.mpf(x)
        for _ in range(P):
            d = float(r)
            out.append(d)
            r = r - mpmath.mpf(d)
    return out


def limbs_to_mp(limbs: Sequence[float]):
    with mpmath.workprec(_MP_PREC):
        s = mpmath.mpf(0)
        for d in limbs:
            s += mpmath.mpf(float(d))
        return s


def complex_to_limbs(z, P: int) -> np.ndarray:
    """[2][P] limbs of an mpmath complex (or real)."""
    z = mpmath.mpc(z)
    return np.array([mp_to_limbs(z.real, P), mp_to_limbs(z.imag, P)], dtype=np.float64)


def limbs_to_complex(a: np.ndarray):
    a = np.asarray(a, dtype=np.float64)
    with mpmath.workprec(_MP_PREC):
        return mpmath.mpc(limbs_to_mp(a[0]), limbs_to_mp(a[1]))


def unit_complex(thetas: np.ndarray, P: int) -> np.ndarray:
    """exp(i*theta) for double angles theta, rounded to P limbs: [len][2][P]."""
    thetas = np.asarray(thetas, dtype=np.float64).ravel()
    out = np.zeros((thetas.size, 2, P), dtype=np.float64)
    with mpmath.workprec(_MP_PREC):
        for j, th in enumerate(thetas.tolist()):
            c, s = mpmath.cos_sin(mpmath.mpf(th))
            out[j, 0] = mp_to_limbs(c, P)
            out[j, 1] = mp_to_limbs(s, P)
    return out


def roots_of_unity(js: np.ndarray, ds: np.ndarray, P: int) -> np.ndarray:
    """exp(2*pi*i*j/d) rounded to P limbs for integer pairs (j, d): [len][2][P]."""
    js = np.asarray(js).ravel()
    ds = np.asarray(ds).ravel()
    out = np.zeros((js.size, 2, P), dtype=np.float64)
    with mpmath.workprec(_MP_PREC):
        for q, (j, d) in enumerate(zip(js.tolist(), ds.tolist())):
            ang = 2 * mpmath.pi * mpmath.mpf(int(j)) / int(d)
            c, s = mpmath.cos_sin(ang)
            out[q, 0] = mp_to_limbs(c, P)
            out[q, 1] = mp_to_limbs(s, P)
    return out


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    """numpy PCG64 generator seeded with 1000*config + instance."""
    return np.random.Generator(np.random.PCG64(1000 * config + instance))


# ---------------------------------------------------------------------------
# system recipes
# ---------------------------------------------------------------------------

def _build(N, n, P, eqs, thetas, name="") -> PolySystem:
    """eqs: list over equations of lists of monomials [(var, exp), ...]."""
    eq_ptr = [0]
    mon_ptr = [0]
    var: List[int] = []
    exp: List[int] = []
    for mons in eqs:
        for mon in mons:
            for v, e in mon:
                var.append(v)
                exp.append(e)
            mon_ptr.append(len(var))
        eq_ptr.append(len(mon_ptr) - 1)
    nmon = len(mon_ptr) - 1
    coef = unit_complex(thetas[:nmon], P)
    return PolySystem(N=N, n=n, P=P,
                      eq_ptr=np.asarray(eq_ptr, dtype=np.int32),
                      mon_ptr=np.asarray(mon_ptr, dtype=np.int32),
                      var=np.asarray(var, dtype=np.int32),
                      exp=np.asarray(exp, dtype=np.int32),
                      coef=coef, name=name)


def random_system(rng: np.random.Generator, N: int, n: int, mons_per_eq,
                  vars_per_mon, exps: Sequence[int], P: int = DD,
                  const_term: bool = False, name: str = "") -> PolySystem:
    """Random system: per equation ``mons_per_eq`` distinct monomials, each the
    product of ``vars_per_mon`` distinct variables drawn uniformly, exponents
    iid uniform over ``exps``, coefficients exp(i*theta) with theta ~ U[0, 2pi).

    ``mons_per_eq`` / ``vars_per_mon`` are ints or (lo, hi) inclusive ranges
    drawn per equation / per monomial.  ``const_term`` appends a constant
    monomial to every equation.
    """
    def draw(spec):
        if isinstance(spec, (tuple, list)):
            return int(rng.integers(spec[0], spec[1] + 1))
        return int(spec)

    exps = list(exps)
    eqs = []
    for _ in range(N):
        M = draw(mons_per_eq)
        seen = set()
        mons = []
        while len(mons) < M:
            k = min(draw(vars_per_mon), n)
            vs = np.sort(rng.choice(n, size=k, replace=False))
            es = rng.choice(exps, size=k)
            key = tuple(zip(vs.tolist(), es.tolist()))
            if key in seen:
                continue
            seen.add(key)
            mons.append(list(key))
        if const_term:
            mons.append([])
        eqs.append(mons)
    nmon = sum(len(m) for m in eqs)
    thetas = rng.uniform(0.0, 2.0 * math.pi, size=nmon)
    return _build(N, n, P, eqs, thetas, name=name)


def degrees(sys: PolySystem) -> np.ndarray:
    """Total degree of each equation."""
    d = np.zeros(sys.N, dtype=np.int64)
    for i in range(sys.N):
        best = 0
        for _, mon in sys.monomials(i):
            best = max(best, sum(e for _, e in mon))
        d[i] = best
    return d


def random_unit_point(rng: np.random.Generator, n: int, P: int) -> np.ndarray:
    """x_j = exp(i*phi_j), phi_j ~ U[0, 2pi): [n][2][P]."""
    return unit_complex(rng.uniform(0.0, 2.0 * math.pi, size=n), P)


def random_unit_gamma(rng: np.random.Generator, P: int) -> np.ndarray:
    """gamma = exp(i*theta), theta ~ U[0, 2pi): [2][P]."""
    return unit_complex(rng.uniform(0.0, 2.0 * math.pi, size=1), P)[0]


def start_solution(rng: np.random.Generator, degs: np.ndarray, P: int) -> np.ndarray:
    """A random solution of g_i = x_i^{d_i} - 1: x_i = exp(2 pi i j_i / d_i)."""
    degs = np.asarray(degs)
    js = np.array([int(rng.integers(0, int(d))) for d in degs])
    return roots_of_unity(js, degs, P)


def ones_point(n: int, P: int) -> np.ndarray:
    x = np.zeros((n, 2, P))
    x[:, 0, 0] = 1.0
    return x


def convert_precision(a: np.ndarray, P_from: int, P_to: int) -> np.ndarray:
    """Re-round limb arrays [..., 2, P_from] to P_to limbs (exact when widening)."""
    a = np.asarray(a, dtype=np.float64)
    if P_to >= P_from:
        out = np.zeros(a.shape[:-1] + (P_to,))
        out[..., :P_from] = a
        return out
    flat = a.reshape(-1, P_from)
    out = np.zeros((flat.shape[0], P_to))
    for q in range(flat.shape[0]):
        out[q] = mp_to_limbs(limbs_to_mp(flat[q]), P_to)
    return out.reshape(a.shape[:-1] + (P_to,))


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def small_track_system(seed: int = 0, P: int = DD) -> PolySystem:
    """n = N = 8; 8 monomials per equation, each a product of 3 distinct
    variables with exponents uniform in {1, 2}; unit-circle coefficients."""
    rng = rng_for(0, seed)
    return random_system(rng, 8, 8, 8, 3, (1, 2), P, name=f"track8-s{seed}")


def dense32_system(seed: int = 0, P: int = DD) -> PolySystem:
    """n = N = 32 dense: 32 monomials per equation over 16 distinct variables,
    exponents uniform in {1, 2, 3}, unit-circle coefficients."""
    rng = rng_for(1, seed)
    return random_system(rng, 32, 32, 32, 16, (1, 2, 3), P, name=f"dense32-s{seed}")


def dense32_points(seed: int, B: int, P: int = DD) -> np.ndarray:
    """B random unit-modulus points for the dense n = 32 system: [B][32][2][P]."""
    rng = rng_for(1, 500 + seed)
    phis = rng.uniform(0.0, 2.0 * math.pi, size=(B, 32))
    return unit_complex(phis.ravel(), P).reshape(B, 32, 2, P)


def sparse512_system(seed: int = 0, P: int = DD, n: int = 512) -> PolySystem:
    """n = N = 512 sparse: 4 monomials per equation, each the product of 2
    distinct variables with exponent 1, plus a constant term.  Redrawn until
    every variable occurs (otherwise the Jacobian is structurally singular)."""
    inst = seed
    while True:
        rng = rng_for(2, inst)
        s = random_system(rng, n, n, 4, 2, (1,), P, const_term=True,
                          name=f"sparse{n}-s{seed}")
        if np.unique(s.var).size == n:
            return s
        inst += 7919


def batch_systems(count: int = 64, seed: int = 0, P: int = DD,
                  n_range=(16, 96), log_uniform_n: bool = False) -> List[PolySystem]:
    """Heterogeneous systems for batched tracking: n uniform in n_range (or
    log-uniform), monomials per equation uniform in [16, 64], 4..12 distinct
    variables per monomial (capped at n), exponents in {1, 2, 3}."""
    out = []
    for s in range(count):
        rng = rng_for(3, seed * 1000 + s)
        if log_uniform_n:
            n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        else:
            n = int(rng.integers(n_range[0], n_range[1] + 1))
        out.append(random_system(rng, n, n, (16, 64), (4, 12), (1, 2, 3), P,
                                 name=f"batch-n{n}-s{seed * 1000 + s}"))
    return out


def with_root_at_ones(sys: PolySystem) -> PolySystem:
    """Append to every equation the constant term minus the sum of its
    coefficients, so that x = (1, ..., 1) is a root (the sum is formed at
    320 bits and rounded to the system's limbs)."""
    P = sys.P
    eqs, coefs = [], []
    for i in range(sys.N):
        mons = []
        with mpmath.workprec(_MP_PREC):
            acc = mpmath.mpc(0)
            for m, mon in sys.monomials(i):
                mons.append(mon)
                coefs.append(np.asarray(sys.coef[m]))
                acc += limbs_to_complex(sys.coef[m])
            mons.append([])
            coefs.append(complex_to_limbs(-acc, P))
        eqs.append(mons)
    return system_from_monomials(sys.N, sys.n, P, eqs, np.asarray(coefs),
                                 name=sys.name + "+root1")


def diagonal_power_system(cs: np.ndarray, d: int, P: int) -> PolySystem:
    """f_i = x_i^d - c_i, i = 0..n-1 (coefficient of x_i^d is 1); cs: [n][2][P]."""
    n = cs.shape[0]
    eq_ptr = [0]
    mon_ptr = [0]
    var, exp, coefs = [], [], []
    one = np.zeros((2, P))
    one[0, 0] = 1.0
    for i in range(n):
        var.append(i)
        exp.append(d)
        mon_ptr.append(len(var))
        coefs.append(one)
        mon_ptr.append(len(var))
        coefs.append(-np.asarray(cs[i]))
        eq_ptr.append(len(mon_ptr) - 1)
    return PolySystem(N=n, n=n, P=P,
                      eq_ptr=np.asarray(eq_ptr, dtype=np.int32),
                      mon_ptr=np.asarray(mon_ptr, dtype=np.int32),
                      var=np.asarray(var, dtype=np.int32),
                      exp=np.asarray(exp, dtype=np.int32),
                      coef=np.asarray(coefs, dtype=np.float64),
                      name=f"diagpow{n}-d{d}")


def system_from_monomials(N: int, n: int, P: int, eqs, coefs: np.ndarray,
                          name: str = "") -> PolySystem:
    """Build a system from explicit monomial lists and coefficient limbs."""
    eq_ptr = [0]
    mon_ptr = [0]
    var: List[int] = []
    exp: List[int] = []
    for mons in eqs:
        for mon in mons:
            for v, e in mon:
                var.append(v)
                exp.append(e)
            mon_ptr.append(len(var))
        eq_ptr.append(len(mon_ptr) - 1)
    return PolySystem(N=N, n=n, P=P,
                      eq_ptr=np.asarray(eq_ptr, dtype=np.int32),
                      mon_ptr=np.asarray(mon_ptr, dtype=np.int32),
                      var=np.asarray(var, dtype=np.int32),
                      exp=np.asarray(exp, dtype=np.int32),
                      coef=np.asarray(coefs, dtype=np.float64).reshape(-1, 2, P),
                      name=name)
