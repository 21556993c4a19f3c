"""GPU parity on the paper's benchmark families and in complex double, all
through the C ABI:

* cyclic n-roots (Section 4.2; the shapes of Tables 2-3): element by element
  against the oracle at n = 32 (every monomial size 1..32, ragged lanes);
  at n = 128 and 352 (monomials of up to 352 variables, the loop form of
  the reverse mode): the closed-form root gives f = 0 to rounding, Euler's
  identity holds for the homogeneous equations, and the Jacobian rows of
  sampled equations equal the oracle's (a one-equation system each); the
  loop form gives the bits of the unrolled forms;
* minor expansions (Section 4.1): against the oracle;
* complex double (the third mode of Section 3.1): arithmetic bit for bit,
  evaluation, MGS and Newton against the oracle in double;
* tree mode (Section 3.2) in double, DD and QD against the oracle.
"""
import numpy as np
import pytest

from oracle import mpref as M
from oracle import oracle as O
from paper_1501_06625_amd import systems as S
from tests.gpu_util import GATE, UNIT, lead_complex, limb_diff, term_scales

pytestmark = pytest.mark.gpu

GATE1 = {1: 1e-14, **GATE}
UNIT1 = {1: 2.0 ** -53, **UNIT}


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06625_amd import hcn
    return hcn


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _unit_scales(ps):
    """Sum of |terms| of every f and J entry when every coefficient and every
    coordinate has modulus one (each term then has modulus |exponent|):
    Sf [N], SJ [n][N]."""
    Sf = np.zeros(ps.N)
    SJ = np.zeros((ps.n, ps.N))
    eq = np.repeat(np.arange(ps.N), np.diff(ps.eq_ptr))
    np.add.at(Sf, eq, 1.0)
    mon_of_pair = np.repeat(np.arange(ps.nmon), np.diff(ps.mon_ptr))
    np.add.at(SJ, (ps.var, eq[mon_of_pair]), ps.exp.astype(float))
    return Sf, SJ


def _compare(f, J, fo, Jo, Sf, SJ, P):
    ef = np.abs(limb_diff(f, fo)) / np.maximum(Sf, 1e-300)
    eJ = np.abs(limb_diff(J, Jo)) / np.maximum(SJ, 1e-300)
    assert ef.max() <= GATE1[P] and eJ.max() <= GATE1[P], (ef.max(), eJ.max())


# ---------------------------------------------------------------------------
# cyclic n-roots
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("P", [2, 4])
def test_cyclic32_vs_oracle(H, P):
    ps = S.cyclic_system(32, P)
    xs = np.stack([S.random_unit_point(S.rng_for(4, 300 + q), 32, P) for q in range(2)])
    sysd = H.System(ps)
    f, J = H.eval_jac(sysd, dev(xs))
    f, J = host(f), host(J)
    Sf, SJ = _unit_scales(ps)
    for q in range(2):
        fo, Jo = O.eval_jac(ps, xs[q])
        _compare(f[q], J[q], fo, Jo, Sf, SJ, P)


def _one_equation(ps, i):
    """Equation i of ps as a system of one equation in the same unknowns."""
    a, b = int(ps.eq_ptr[i]), int(ps.eq_ptr[i + 1])
    p0, p1 = int(ps.mon_ptr[a]), int(ps.mon_ptr[b])
    return S.PolySystem(N=ps.n, n=ps.n, P=ps.P,
                        eq_ptr=np.array([0] + [b - a] * ps.n, dtype=np.int32),
                        mon_ptr=(ps.mon_ptr[a:b + 1] - p0).astype(np.int32),
                        var=ps.var[p0:p1].copy(), exp=ps.exp[p0:p1].copy(),
                        coef=ps.coef[a:b].copy())


@pytest.mark.parametrize("n", [128, 352])
def test_cyclic_large_properties(H, n):
    """DD at the sizes of Tables 2-3: f vanishes at the closed-form root
    (n terms of modulus one per equation); at a random unit point Euler's
    identity sum_k x_k J_ik = i f_i holds for i < n, and the Jacobian rows
    of sampled equations (sizes 1, 2, 25 and n) equal the oracle's."""
    P = 2
    ps = S.cyclic_system(n, P)
    sysd = H.System(ps)
    assert sysd.info().max_k == n
    root = S.cyclic_root(n, P)
    x = S.random_unit_point(S.rng_for(4, 400 + n), n, P)
    f, J = H.eval_jac(sysd, dev(np.stack([root, x])))
    f, J = host(f), host(J)
    assert np.abs(lead_complex(f[0])).max() <= n * 1e-30
    Sf, SJ = _unit_scales(ps)
    xc = lead_complex(x)
    for i in range(n - 1):
        lhs = (xc[:, None] * lead_complex(J[1][:, i:i + 1])).sum()
        # double is enough to catch a wrong term: the gate is a few ulps of
        # double on sums of i n terms of modulus one
        assert abs(lhs - (i + 1) * lead_complex(f[1][i])) <= 1e-12 * (i + 1) * Sf[i]
    for i in (0, 1, 24, n - 1):
        one = _one_equation(ps, i)
        fo, Jo = O.eval_jac(one, x)
        e = np.abs(limb_diff(J[1][:, i], Jo[:, 0])) / np.maximum(SJ[:, i], 1e-300)
        assert e.max() <= GATE[P], (i, e.max())
        assert abs(limb_diff(f[1][i], fo[0])) / Sf[i] <= GATE[P]


@pytest.mark.parametrize("P", [2, 4])
def test_long_form_bitwise(H, P):
    """A monomial of more than 64 variables sends every monomial of its
    system to the loop form of the reverse mode (loads issued a group of
    positions ahead).  A random system with such a monomial added to its
    last equation gives, in every other equation, the bits of f and J of the
    system without it, whose monomials take the unrolled forms (exponents up
    to 3: the staged powers of the uniform form; DD keeps its forward
    products in registers, QD in the slots)."""
    n = 70
    rng = np.random.default_rng(31 + P)
    A = S.random_system(rng, n, n, (2, 6), (1, 8), (1, 2, 3), P=P)
    lv = np.sort(rng.choice(n, size=66, replace=False)).astype(np.int32)
    le = rng.choice([1, 2, 3], size=66).astype(np.int32)
    coef = S.unit_complex(rng.uniform(0.0, 6.283, size=1), P).reshape(1, 2, P)
    B = S.PolySystem(N=n, n=n, P=P,
                     eq_ptr=np.concatenate([A.eq_ptr[:-1], [A.eq_ptr[-1] + 1]]).astype(np.int32),
                     mon_ptr=np.concatenate([A.mon_ptr, [A.mon_ptr[-1] + 66]]).astype(np.int32),
                     var=np.concatenate([A.var, lv]).astype(np.int32),
                     exp=np.concatenate([A.exp, le]).astype(np.int32),
                     coef=np.concatenate([A.coef, coef]))
    sa, sb = H.System(A), H.System(B)
    assert sa.info().max_k <= 8 and sb.info().max_k == 66
    x = np.stack([S.random_unit_point(S.rng_for(4, 700 + q), n, P) for q in range(3)])
    fa, Ja = H.eval_jac(sa, dev(x))
    fb, Jb = H.eval_jac(sb, dev(x))
    fa, Ja, fb, Jb = (np.asarray(v.cpu().numpy()) for v in (fa, Ja, fb, Jb))
    assert np.array_equal(fa[:, :n - 1].view(np.uint64), fb[:, :n - 1].view(np.uint64))
    assert np.array_equal(Ja[:, :, :n - 1].view(np.uint64), Jb[:, :, :n - 1].view(np.uint64))
    sa.free()
    sb.free()


# ---------------------------------------------------------------------------
# minor expansions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("P", [2, 4])
def test_determinantal_vs_oracle(H, P):
    ps = S.determinantal_system(6, 3, 14, seed=2, P=P)
    xs = np.stack([S.random_unit_point(S.rng_for(5, 500 + q), ps.n, P) for q in range(2)])
    sysd = H.System(ps)
    f, J = H.eval_jac(sysd, dev(xs))
    f, J = host(f), host(J)
    for q in range(2):
        fo, Jo = O.eval_jac(ps, xs[q])
        Sf, SJ = term_scales(ps, xs[q])
        _compare(f[q], J[q], fo, Jo, Sf, SJ, P)


# ---------------------------------------------------------------------------
# complex double
# ---------------------------------------------------------------------------

def _to_double(ps):
    return S.PolySystem(N=ps.N, n=ps.n, P=1, eq_ptr=ps.eq_ptr, mon_ptr=ps.mon_ptr, var=ps.var,
                        exp=ps.exp, coef=np.ascontiguousarray(ps.coef[:, :, :1]))


def test_double_arithmetic_bitwise(H):
    rng = np.random.default_rng(11)
    a = rng.standard_normal((4096, 1)) * 10.0 ** rng.integers(-8, 8, (4096, 1))
    b = rng.standard_normal((4096, 1))
    for op in ("add", "sub", "mul", "div"):
        assert np.array_equal(host(H.elementwise(op, 1, dev(a), dev(b))), O.elementwise(op, 1, a, b))
    za = rng.standard_normal((2048, 2, 1))
    zb = rng.standard_normal((2048, 2, 1))
    for op in ("cadd", "csub", "cmul", "cmul_conj"):
        assert np.array_equal(host(H.elementwise(op, 1, dev(za), dev(zb))), O.elementwise(op, 1, za, zb))


@pytest.mark.parametrize("tree", [False, True])
def test_double_eval_dense32(H, tree):
    ps = _to_double(S.dense32_system(0, 2))
    xs = S.dense32_points(3, 3, 2)[:, :, :, :1].copy()
    sysd = H.System(ps)
    H.set_mon_tree(tree)
    try:
        f, J = H.eval_jac(sysd, dev(xs))
    finally:
        H.set_mon_tree(False)
    f, J = host(f), host(J)
    for q in range(3):
        fo, Jo = O.eval_jac(ps, xs[q])
        Sf, SJ = term_scales(ps, xs[q])
        # a sum of M terms of up to 49 factors in double: (M + 3 deg) u
        e_gate = 200 * 2.0 ** -53
        ef = np.abs(limb_diff(f[q], fo)) / Sf
        eJ = np.abs(limb_diff(J[q], Jo)) / np.maximum(SJ, 1e-300)
        assert ef.max() <= e_gate and eJ.max() <= e_gate


def test_double_newton_and_tracking(H):
    ps2 = S.small_track_system(3, 2)
    ps = _to_double(ps2)
    g = O.total_degree_start(ps)
    gam = S.random_unit_gamma(S.rng_for(0, 103), 2)[:, :1].copy()
    x0 = S.ones_point(ps.n, 1)
    sysd = H.System(ps)
    # one Newton step on the homotopy
    xs = S.start_solution(S.rng_for(5, 9), S.degrees(ps), 2)[:, :, :1].copy()
    xs[:, 0, 0] += 1e-3
    xd = dev(xs[None])
    ts = dev(np.array([0.25]))
    H.newton_step(sysd, xd, gamma=gam, t=ts)
    rc, xo, no = O.newton_step(ps, g, gam, 1, 0.25, xs)
    h, Jh = O.eval_h(ps, g, gam, 1, 0.25, xs)
    kappa = np.linalg.cond(lead_complex(Jh).T)
    assert np.abs(limb_diff(host(xd)[0], xo)).max() <= 16 * ps.n * kappa * 2.0 ** -53 * no[1]
    # tracking: the same decisions as the oracle in double
    xg, res = H.track_paths(sysd, gam, dev(x0[None]), max_steps=400)
    xr, r = O.track(ps, g, gam, 1, x0, max_steps=400)
    assert (res[0]["status"], res[0]["steps"], res[0]["accepted"]) == (r.status, r.steps, r.accepted)


@pytest.mark.parametrize("P", [1, 2, 4])
def test_double_mgs(H, P):
    rng = np.random.default_rng(20 + P)
    N, n = 40, 33
    A = rng.standard_normal((1, n, N, 2, P))
    A[..., 1:] = 0.0
    b = rng.standard_normal((1, N, 2, P))
    b[..., 1:] = 0.0
    dx, R, status = H.mgs_solve(dev(A), dev(b))
    assert int(host(status)[0]) == 0
    rc, dxo, _, _, _ = O.mgs_solve(P, A[0], b[0])
    Ac = lead_complex(A[0]).T
    kappa = np.linalg.cond(Ac)
    tol = max(GATE1[P], 16 * n * kappa * UNIT1[P])
    assert np.abs(limb_diff(host(dx)[0], dxo)).max() <= tol * np.abs(lead_complex(dxo)).max()


# ---------------------------------------------------------------------------
# tree mode
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("P", [2, 4])
def test_tree_mode_vs_oracle(H, P):
    """Tree mode on the dense system (16 variables, exponents to 3: the power
    table path) and on a ragged system (1..7 variables, exponents to 2, a
    constant term): within the reduction gate of the plain definition."""
    H.set_mon_tree(True)
    try:
        for ps in (S.dense32_system(0, P),
                   S.random_system(S.rng_for(7, 200 + P), 12, 12, (1, 9), (1, 7), (1, 2), P,
                                   const_term=True)):
            xs = np.stack([S.random_unit_point(S.rng_for(7, 210 + q), ps.n, P) for q in range(2)])
            sysd = H.System(ps)
            f, J = H.eval_jac(sysd, dev(xs))
            f, J = host(f), host(J)
            for q in range(2):
                fo, Jo = O.eval_jac(ps, xs[q])
                Sf, SJ = term_scales(ps, xs[q])
                _compare(f[q], J[q], fo, Jo, Sf, SJ, P)
    finally:
        H.set_mon_tree(False)
