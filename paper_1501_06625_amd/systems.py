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


def with_finite_roots(sys: PolySystem, seed: int = 0) -> PolySystem:
    """Append to every equation i a pure power c_i x_i^{d_i} (d_i the
    equation's degree, c_i = exp(i theta), theta ~ U[0, 2 pi) seeded), then
    the constant term minus the sum of all its coefficients, so that
    x = (1, ..., 1) is a root (the sum formed at 320 bits).  The pure powers
    put x_i^{d_i} in the leading form of equation i, so (for random
    coefficients) the leading forms have no common zero: the system has no
    roots at infinity and every path of the total-degree homotopy ends at a
    finite root.  The literal random systems have no constant term and
    far fewer finite roots than the total degree, so most of their paths
    diverge."""
    P = sys.P
    rng = rng_for(8, seed)
    degs = degrees(sys)
    eqs, coefs = [], []
    for i in range(sys.N):
        mons = []
        with mpmath.workprec(_MP_PREC):
            acc = mpmath.mpc(0)
            for m, mon in sys.monomials(i):
                mons.append(mon)
                coefs.append(np.asarray(sys.coef[m]))
                acc += limbs_to_complex(sys.coef[m])
            c = unit_complex(np.array([rng.uniform(0.0, 2.0 * math.pi)]), P)[0]
            mons.append([(i, int(degs[i]))])
            coefs.append(c)
            acc += limbs_to_complex(c)
            mons.append([])
            coefs.append(complex_to_limbs(-acc, P))
        eqs.append(mons)
    return system_from_monomials(sys.N, sys.n, P, eqs, np.asarray(coefs),
                                 name=sys.name + "+finite")


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


# ---------------------------------------------------------------------------
# the paper's two benchmark families, as structure (Section 4)
# ---------------------------------------------------------------------------

def cyclic_system(n: int, P: int = DD) -> PolySystem:
    """The cyclic n-roots system (Section 4.2): f_1 = x_0 + ... + x_{n-1};
    f_i = sum_{j=0}^{n-1} prod_{k=j}^{j+i-1} x_{k mod n} for i = 2..n-1;
    f_n = x_0 x_1 ... x_{n-1} - 1.  Equation i has n monomials of i
    variables (its degree is i), so the system has monomials of every size
    1..n; coefficients are 1 (and -1 for the constant)."""
    eqs, coefs = [], []
    one = np.zeros((2, P))
    one[0, 0] = 1.0
    for i in range(1, n):
        mons = []
        for j in range(n):
            mons.append([((j + q) % n, 1) for q in range(i)])
            coefs.append(one)
        eqs.append(mons)
    eqs.append([[(q, 1) for q in range(n)], []])
    coefs.append(one)
    coefs.append(-one)
    return system_from_monomials(n, n, P, eqs, np.asarray(coefs), name=f"cyclic{n}")


def cyclic_root(n: int, P: int = DD) -> np.ndarray:
    """A root of the cyclic n-roots system found by substitution:
    x_j = w^j for odd n and x_j = e^{i pi / n} w^j for even n, w = e^{2 pi i / n}
    (then every f_i, i < n, is a multiple of sum_j w^{ij} = 0 and the product
    of all x_j is 1); rounded to P limbs at 320 bits: [n][2][P]."""
    out = np.zeros((n, 2, P))
    with mpmath.workprec(_MP_PREC):
        for j in range(n):
            ang = 2 * mpmath.pi * mpmath.mpf(j) / n
            if n % 2 == 0:
                ang += mpmath.pi / n
            c, s_ = mpmath.cos_sin(ang)
            out[j, 0] = mp_to_limbs(c, P)
            out[j, 1] = mp_to_limbs(s_, P)
    return out


def pieri_variables(m: int, p: int):
    """Positions (row, column) of the unknowns of the (m+p) x p localization
    pattern (Section 4.1): column c has its 1 at row c and unknowns at rows
    c+1 .. c+m; they are introduced one at a time, the last column first,
    top to bottom within a column."""
    order = []
    for c in range(p - 1, -1, -1):
        for r in range(c + 1, c + m + 1):
            order.append((r, c))
    return order


def determinantal_system(m: int, p: int, k: int, seed: int = 0, P: int = DD) -> PolySystem:
    """A system of minor expansions (Section 4.1, equation (5)): the unknowns
    are the first k entries of the Pieri pattern of an (m+p) x p matrix X
    (pieri_variables; later pattern entries are 0), and equation i is
    det(K_i^T X) = 0 for a random complex (m+p) x p matrix K_i, i = 1..k,
    which is det(A_i | X) = 0 for an A_i whose columns span the orthogonal
    complement of K_i's.  By Cauchy-Binet,
        det(K^T X) = sum over p-row subsets S of det(K[S]) det(X[S]),
    and det(X[S]) expands by Leibniz into products of entries from distinct
    rows and columns: every monomial is a product of at most p distinct
    unknowns.  The coefficients (sums of signed p x p minors of K_i, in
    double precision: the K_i are random draws) are exact doubles in limb
    0.  Seeded with 1000*5 + seed."""
    from itertools import combinations, permutations
    n = m + p
    order = pieri_variables(m, p)
    if not 1 <= k <= len(order):
        raise ValueError("k out of range")
    var_at = {pos: q for q, pos in enumerate(order[:k])}
    # terms (S, sign, monomial) of det(X[S]) with every entry nonzero
    subsets = list(combinations(range(n), p))
    perms = list(permutations(range(p)))

    def sign(pm):
        s_, seen = 1, list(pm)
        for a in range(len(seen)):
            for b in range(a + 1, len(seen)):
                if seen[a] > seen[b]:
                    s_ = -s_
        return s_

    mono_index = {}
    t_sub, t_sign, t_mono = [], [], []
    for si, S in enumerate(subsets):
        for pm in perms:
            vs = []
            ok = True
            for c in range(p):
                r = S[pm[c]]
                if r == c:
                    continue  # the pivot 1
                if (r, c) in var_at:
                    vs.append(var_at[(r, c)])
                else:
                    ok = False
                    break
            if not ok:
                continue
            key = tuple(sorted(vs))
            if key not in mono_index:
                mono_index[key] = len(mono_index)
            t_sub.append(si)
            t_sign.append(sign(pm))
            t_mono.append(mono_index[key])
    monos = sorted(mono_index, key=lambda key: (len(key), key))
    rank = {key: q for q, key in enumerate(monos)}
    remap = np.array([rank[key] for key in mono_index], dtype=np.int64)
    t_mono = remap[np.array(t_mono, dtype=np.int64)]
    rng = rng_for(5, seed)
    K = rng.standard_normal((k, n, p)) + 1j * rng.standard_normal((k, n, p))
    idx = np.array(subsets, dtype=np.int64)              # [nsub][p]
    minors = np.linalg.det(K[:, idx, :])                 # [k][nsub]
    coef = np.zeros((k, len(monos)), dtype=np.complex128)
    contrib = minors[:, np.array(t_sub)] * np.array(t_sign)[None, :]
    for i in range(k):
        np.add.at(coef[i], t_mono, contrib[i])
    # every equation has the same support (the coefficients are nonzero with
    # probability one): the tables of one equation repeated k times
    M = len(monos)
    lens = np.array([len(key) for key in monos], dtype=np.int64)
    flat = np.array([v for key in monos for v in key], dtype=np.int32)
    mon_ptr = np.zeros(k * M + 1, dtype=np.int64)
    mon_ptr[1:] = np.cumsum(np.tile(lens, k))
    coefs = np.zeros((k * M, 2, P))
    coefs[:, 0, 0] = coef.real.ravel()
    coefs[:, 1, 0] = coef.imag.ravel()
    return PolySystem(N=k, n=k, P=P,
                      eq_ptr=np.arange(0, k * M + 1, M, dtype=np.int32),
                      mon_ptr=mon_ptr.astype(np.int32),
                      var=np.tile(flat, k).astype(np.int32),
                      exp=np.ones(k * flat.size, dtype=np.int32),
                      coef=coefs, name=f"det-m{m}-p{p}-k{k}")
