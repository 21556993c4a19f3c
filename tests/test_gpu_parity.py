"""GPU (HIP, through the C ABI) against the CPU oracle.

Bars: elementwise DD/QD operations bit for bit; reductions (f, J) within
1e-28 (DD) / 1e-58 (QD) of the sum of the magnitudes of their terms; solves
by normwise backward error <= 1e-28 / 1e-58 and forward difference to the
oracle <= max(1e-28, 16 n kappa u); Newton and tracking decisions equal.
"""
import contextlib
import time

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from oracle import mpref as M
from paper_1501_06625_amd import systems as S
from tests.gpu_util import GATE, UNIT, limb_diff, lead_complex, term_scales, random_points, update_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1501_06625_amd import hcn
    return hcn


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------------------
# arithmetic layer: bit for bit
# ---------------------------------------------------------------------------

def _rand_reals(rng, cnt, P, spread=30):
    hi = rng.standard_normal(cnt) * np.exp2(rng.integers(-spread, spread, cnt))
    out = np.zeros((cnt, P))
    out[:, 0] = hi
    prev = hi
    for j in range(1, P):
        nxt = np.spacing(np.abs(prev)) * rng.uniform(-0.5, 0.5, cnt)
        out[:, j] = nxt
        prev = np.where(nxt == 0, prev, nxt)
    # edge cases: zeros, powers of two, exact negatives
    out[:8] = 0.0
    out[8:16, 0] = np.exp2(np.arange(8) - 4)
    out[8:16, 1:] = 0.0
    return out


def _bitwise_equal(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.array_equal(a, b) or bool(np.all((a == b) | (np.isnan(a) & np.isnan(b))))


@pytest.mark.parametrize("P", [2, 4])
def test_elementwise_bitwise(H, P):
    rng = np.random.default_rng(1000 + P)
    cnt = 20000
    a = _rand_reals(rng, cnt, P)
    b = _rand_reals(rng, cnt, P)
    # cancellation partners: b = -a + tiny
    b[100:600] = -a[100:600]
    b[100:600, P - 1] += np.spacing(np.abs(a[100:600, P - 1])) * 3
    bsafe = np.where(np.abs(b[:, :1]) > 0, b, 1.0)
    for op, x, y in (("add", a, b), ("sub", a, b), ("mul", a, b), ("div", a, bsafe)):
        g = host(H.elementwise(op, P, dev(x), dev(y)))
        o = O.elementwise(op, P, x, y)
        assert _bitwise_equal(g, o), op
    pos = np.where(a[:, :1] < 0, -a, a)
    assert _bitwise_equal(host(H.elementwise("sqrt", P, dev(pos))), O.elementwise("sqrt", P, pos))
    d = rng.standard_normal(cnt) * np.exp2(rng.integers(-10, 10, cnt))
    assert _bitwise_equal(host(H.elementwise("mul_d", P, dev(a), dev(d))),
                          O.elementwise("mul_d", P, a, d))
    ca = _rand_reals(rng, 2 * cnt, P).reshape(cnt, 2, P)
    cb = _rand_reals(rng, 2 * cnt, P).reshape(cnt, 2, P)
    for op in ("cadd", "csub", "cmul", "cmul_conj"):
        assert _bitwise_equal(host(H.elementwise(op, P, dev(ca), dev(cb))),
                              O.elementwise(op, P, ca, cb)), op
    assert _bitwise_equal(host(H.elementwise("cnorm2", P, dev(ca))), O.elementwise("cnorm2", P, ca))
    assert _bitwise_equal(host(H.elementwise("cscale", P, dev(ca), dev(a))),
                          O.elementwise("cscale", P, ca, a))


def test_eft_bitwise(H):
    rng = np.random.default_rng(7)
    a = rng.standard_normal(50000) * np.exp2(rng.integers(-60, 60, 50000))
    b = rng.standard_normal(50000) * np.exp2(rng.integers(-60, 60, 50000))
    for op in ("two_sum", "two_prod"):
        assert _bitwise_equal(host(H.elementwise(op, 2, dev(a), dev(b))), O.elementwise(op, 2, a, b))
    big = np.where(np.abs(a) >= np.abs(b), a, b)
    sm = np.where(np.abs(a) >= np.abs(b), b, a)
    assert _bitwise_equal(host(H.elementwise("fast_two_sum", 2, dev(big), dev(sm))),
                          O.elementwise("fast_two_sum", 2, big, sm))


# ---------------------------------------------------------------------------
# evaluation and differentiation
# ---------------------------------------------------------------------------

def _ragged_system(P, seed=4):
    """Monomials of 0..20 variables (several k-groups, constants, k = 1,
    and more than 16 variables), exponents 1..3."""
    rng = np.random.default_rng(seed)
    n = N = 24
    eqs = []
    for i in range(N):
        mons = [[]]  # a constant term
        seen = set()
        for _ in range(int(rng.integers(3, 12))):
            k = int(rng.choice([1, 2, 3, 5, 8, 13, 17, 20]))
            vs = tuple(sorted(rng.choice(n, size=k, replace=False).tolist()))
            if vs in seen:
                continue
            seen.add(vs)
            mons.append([(v, int(rng.integers(1, 4))) for v in vs])
        eqs.append(mons)
    nmon = sum(len(m) for m in eqs)
    coefs = S.unit_complex(rng.uniform(0, 6.28, nmon), P)
    return S.system_from_monomials(N, n, P, eqs, coefs, name="ragged")


def _check_eval(H, ps, xs):
    P = ps.P
    sysd = H.System(ps)
    f, J = H.eval_jac(sysd, dev(xs))
    f, J = host(f), host(J)
    for b in range(xs.shape[0]):
        fo, Jo = O.eval_jac(ps, xs[b])
        Sf, SJ = term_scales(ps, xs[b])
        ef = np.abs(limb_diff(f[b], fo))
        eJ = np.abs(limb_diff(J[b], Jo))
        assert np.all(ef <= GATE[P] * Sf + 1e-300), (b, ef.max())
        assert np.all(eJ <= GATE[P] * SJ + 1e-300), (b, eJ.max())
        # structural zeros are exact zeros
        assert np.all(J[b][SJ == 0] == 0)
    sysd.free()


@pytest.mark.parametrize("P", [2, 4])
def test_eval_small_track_system(H, P):
    ps = S.small_track_system(1, P)
    xs = random_points(np.random.default_rng(3), 5, ps.n, P)
    _check_eval(H, ps, xs)


@pytest.mark.parametrize("P", [2, 4])
def test_eval_dense32(H, P):
    ps = S.dense32_system(0, P)
    xs = S.dense32_points(0, 2, P)
    _check_eval(H, ps, xs)


@pytest.mark.parametrize("P", [2, 4])
def test_eval_ragged(H, P):
    ps = _ragged_system(P)
    xs = random_points(np.random.default_rng(5), 3, ps.n, P)
    # also a non-unit point to exercise magnitudes
    xs[2] *= 1.3
    _check_eval(H, ps, xs)


def test_eval_sparse512_sampled(H):
    """Full-size sparse system: every output checked (the oracle's plain
    evaluation of this system is cheap)."""
    ps = S.sparse512_system(0, 2)
    xs = random_points(np.random.default_rng(9), 1, ps.n, 2)
    _check_eval(H, ps, xs)


@pytest.mark.parametrize("P", [2, 4])
def test_monomials_uniform_form_bitwise(H, P):
    """The uniform form of the common factor (same products in every lane,
    powers tabulated per point) gives bitwise the f and J of the branching
    form: largest exponent 3 with 16 and with up to 20 variables per
    monomial (registers and output-slot forward products), largest exponent
    2, exponents up to 5, the FP64 Jacobian of the mixed-precision step, and
    a slot-table batch."""
    import torch
    rng = np.random.default_rng(31 + P)
    cases = [(S.dense32_system(0, P), S.dense32_points(2, 3, P)),
             (_ragged_system(P), random_points(rng, 3, 24, P)),
             (S.small_track_system(2, P), random_points(rng, 3, 8, P)),
             (S.random_system(S.rng_for(3, 901), 12, 12, (3, 8), (1, 6), (1, 2, 3, 4, 5), P),
              random_points(rng, 3, 12, P))]
    try:
        for ps, xs in cases:
            sysd = H.System(ps)
            out = {}
            for uni in (True, False):
                H.set_mon_uniform(uni)
                f, J = H.eval_jac(sysd, dev(xs))
                xd = dev(xs)
                st, it, nm = H.newton(sysd, xd, mixed=True, max_iter=2)
                out[uni] = [host(f), host(J), host(xd), host(st), host(nm)]
            for a, b in zip(out[True], out[False]):
                assert _bitwise_equal(a, b), ps.name
            sysd.free()
        cases_b = _batch_cases(P)
        systems = {id(c[0]): H.System(c[0]) for c in cases_b}
        maxs = max(sd.info().nslots for sd in systems.values())
        res = {}
        for uni in (True, False):
            H.set_mon_uniform(uni)
            bt = H.Batch(P, capacity=len(cases_b), max_n=8, max_nslots=maxs, max_steps=30)
            for slot, (ps, gam, x0) in enumerate(cases_b):
                bt.add(slot, systems[id(ps)], gam, dev(x0))
            bt.run()
            res[uni] = [bt.result(slot, ps.n) for slot, (ps, _, _) in enumerate(cases_b)]
            bt.free()
        for (xa, ra), (xb, rb) in zip(res[True], res[False]):
            assert _bitwise_equal(host(xa), host(xb)) and ra.tobytes() == rb.tobytes()
    finally:
        H.set_mon_uniform(True)


def test_empty_batches_are_noops(H):
    """Zero points: every entry point returns at once with empty outputs."""
    import torch
    for P in (2, 4):
        ps = S.small_track_system(3, P)
        sysd = H.System(ps)
        x = torch.zeros((0, ps.n, 2, P), dtype=torch.float64, device="cuda")
        f, J = H.eval_jac(sysd, x)
        assert f.shape[0] == 0 and J.shape[0] == 0
        norms, st = H.newton_step(sysd, x)
        assert norms.shape[0] == 0 and st.shape[0] == 0
        for mixed in (False, True):
            st, it, nm = H.newton(sysd, x, mixed=mixed)
            assert st.shape[0] == 0
        xo, res = H.track_paths(sysd, S.random_unit_gamma(S.rng_for(0, 1), P), x)
        assert xo.shape[0] == 0 and len(res) == 0
        sysd.free()


def test_points_beyond_one_grid_row(H):
    """More points than one grid dimension holds (65535): the launches loop
    over the rest, and every point gets bitwise what it gets in a small
    batch (evaluation, one Newton step, the Fig. 2 loop)."""
    P = 2
    ps = S.small_track_system(5, P)
    rng = np.random.default_rng(65536)
    B = 70000
    xs = random_points(rng, B, ps.n, P)
    sysd = H.System(ps)
    f, J = H.eval_jac(sysd, dev(xs))
    xd = dev(xs)
    nm1, st1 = H.newton_step(sysd, xd)
    xl = dev(xs)
    st, it, nm = H.newton(sysd, xl)
    f, J, xd, nm1, xl, st = host(f), host(J), host(xd), host(nm1), host(xl), host(st)
    for lo in (0, 65530, B - 7):
        sl = slice(lo, lo + 7)
        fs, Js = H.eval_jac(sysd, dev(xs[sl]))
        assert _bitwise_equal(host(fs), f[sl]) and _bitwise_equal(host(Js), J[sl]), lo
        xq = dev(xs[sl])
        nq, _ = H.newton_step(sysd, xq)
        assert _bitwise_equal(host(xq), xd[sl]) and _bitwise_equal(host(nq), nm1[sl]), lo
        xq = dev(xs[sl])
        sq, _, _ = H.newton(sysd, xq)
        assert _bitwise_equal(host(xq), xl[sl]) and np.array_equal(host(sq), st[sl]), lo
    sysd.free()


def test_eval_batch_independent_and_deterministic(H):
    ps = S.dense32_system(0, 2)
    xs = S.dense32_points(1, 6, 2)
    sysd = H.System(ps)
    f, J = H.eval_jac(sysd, dev(xs))
    f2, J2 = H.eval_jac(sysd, dev(xs))
    assert _bitwise_equal(host(f), host(f2)) and _bitwise_equal(host(J), host(J2))
    f1, J1 = H.eval_jac(sysd, dev(xs[3]))
    assert _bitwise_equal(host(f1), host(f)[3]) and _bitwise_equal(host(J1), host(J)[3])


# ---------------------------------------------------------------------------
# modified Gram-Schmidt solve
# ---------------------------------------------------------------------------

def _rand_matrix(rng, N, n, P):
    return random_points(rng, n, N, P) * rng.uniform(0.3, 1.0, (n, N, 1, 1))


def _backward_error(A, b, dx):
    """||A dx - b||_inf / (||A||_inf ||dx||_inf + ||b||_inf) at 320 bits."""
    Am, xm = M.colmajor(A), mpmath.matrix(M.vec(dx))
    bm = mpmath.matrix(M.vec(b))
    r = Am * xm - bm
    num = max(abs(r[i]) for i in range(r.rows))
    nA = max(sum(abs(Am[i, j]) for j in range(Am.cols)) for i in range(Am.rows))
    nx = max(abs(xm[i]) for i in range(xm.rows))
    nb = max(abs(bm[i]) for i in range(bm.rows))
    return float(num / (nA * nx + nb))


@pytest.mark.parametrize("P,N,n", [(2, 8, 8), (2, 32, 32), (2, 40, 24), (4, 16, 16), (2, 1, 1),
                                   (4, 33, 33)])
def test_mgs_parity(H, P, N, n):
    rng = np.random.default_rng(N * 7 + n + P)
    B = 3
    A = np.stack([_rand_matrix(rng, N, n, P) for _ in range(B)])
    b = random_points(rng, B, N, P)
    Ad, bd = dev(A), dev(b)
    dx, R, status = H.mgs_solve(Ad, bd)
    dx, R, status = host(dx), host(R), host(status)
    assert np.all(status == 0)
    for q in range(B):
        rc, dxo, Qo, Ro, _ = O.mgs_solve(P, A[q], b[q])
        assert rc == 0
        if N == n:
            assert _backward_error(A[q], b[q], dx[q]) <= GATE[P]
        Z = lead_complex(A[q]).T
        kappa = np.linalg.cond(Z)
        tol = max(GATE[P], 16 * n * kappa * UNIT[P])
        scale = np.abs(lead_complex(dxo)).max()
        assert np.abs(limb_diff(dx[q], dxo)).max() <= tol * scale
        assert np.abs(limb_diff(R[q], Ro)).max() <= tol * np.abs(lead_complex(Ro)).max()


def test_mgs_singular_and_empty(H):
    import torch
    rng = np.random.default_rng(2)
    A = np.stack([_rand_matrix(rng, 6, 6, 2) for _ in range(2)])
    A[1, 3] = 0.0
    b = random_points(rng, 2, 6, 2)
    dx, R, status = H.mgs_solve(dev(A), dev(b))
    st = host(status)
    assert st[0] == H.OK and st[1] == H.ESINGULAR
    # an empty batch is a no-op
    dx, R, status = H.mgs_solve(torch.zeros((0, 2, 2, 2, 2), dtype=torch.float64, device="cuda"),
                                torch.zeros((0, 2, 2, 2), dtype=torch.float64, device="cuda"))
    assert dx.shape[0] == 0


# ---------------------------------------------------------------------------
# Newton
# ---------------------------------------------------------------------------

def _kappa_at(ps, x):
    _, J = O.eval_jac(ps, x)
    return np.linalg.cond(lead_complex(J).T)


@pytest.mark.parametrize("P", [2, 4])
def test_newton_step_dense32(H, P):
    ps = S.dense32_system(0, P)
    xs = S.dense32_points(2, 2, P)
    sysd = H.System(ps)
    xd = dev(xs)
    norms, status = H.newton_step(sysd, xd)
    xg, norms, status = host(xd), host(norms), host(status)
    assert np.all(status == 0)
    for q in range(xs.shape[0]):
        rc, xo, no = O.newton_step(ps, None, None, 1, 1.0, xs[q])
        assert rc == 0
        kappa = _kappa_at(ps, xs[q])
        tol = max(GATE[P], 16 * ps.n * kappa * UNIT[P])
        assert np.abs(limb_diff(xg[q], xo)).max() <= update_bound(tol, no[1], xo, P)
        assert abs(norms[q, 0] - no[0]) <= 1e-14 * no[0]
        assert abs(norms[q, 1] - no[1]) <= 1e-10 * no[1]


@pytest.mark.parametrize("P", [2, 4])
def test_newton_step_homotopy(H, P):
    ps = S.small_track_system(2, P)
    g = O.total_degree_start(ps)
    rng = S.rng_for(0, 77)
    gam = S.random_unit_gamma(rng, P)
    xs = S.start_solution(rng, S.degrees(ps), P)[None].repeat(3, 0)
    xs[:, :, 0, 0] += 1e-3 * rng.standard_normal((3, ps.n))
    ts = np.array([0.0, 0.25, 0.6])
    import torch
    sysd = H.System(ps)
    xd = dev(xs)
    norms, status = H.newton_step(sysd, xd, gamma=gam, t=dev(ts))
    xg = host(xd)
    for q in range(3):
        rc, xo, no = O.newton_step(ps, g, gam, 1, float(ts[q]), xs[q])
        h, Jh = O.eval_h(ps, g, gam, 1, float(ts[q]), xs[q])
        kappa = np.linalg.cond(lead_complex(Jh).T)
        tol = max(GATE[P], 16 * ps.n * kappa * UNIT[P])
        assert np.abs(limb_diff(xg[q], xo)).max() <= tol * max(no[1], 1e-300)


def _iterate_bound(ps, g, gam, t, x0, iters, P):
    """Bound on the difference between two runs of `iters` Newton iterations
    from x0 whose solves are each backward stable: every solve may differ by
    16 n kappa u |dx| (normwise), kappa taken at each iterate of the oracle's
    run; the differences add up (near a regular root the Newton map shrinks
    them further).  Returns sum_k max(GATE, 16 n kappa_k u) |dx_k| plus GATE
    for the last update's rounding."""
    x = x0.copy()
    total = 0.0
    for _ in range(iters):
        h, Jh = O.eval_h(ps, g, gam, 1, t, x)
        kappa = np.linalg.cond(lead_complex(Jh).T)
        rc, x, no = O.newton_step(ps, g, gam, 1, t, x)
        if rc:
            break
        total += max(GATE[P], 16 * ps.n * kappa * UNIT[P]) * no[1]
    return total + GATE[P] * max(1.0, np.abs(lead_complex(x)).max())


def test_newton_fig2_decisions(H):
    """Fig. 2 on the device takes the oracle's decisions (status and
    evaluations) over a range of distances from the path; the iterates agree
    within the bound of _iterate_bound for the updates actually applied."""
    P = 2
    ps = S.small_track_system(3, P)
    g = O.total_degree_start(ps)
    rng = S.rng_for(0, 78)
    gam = S.random_unit_gamma(rng, P)
    B = 12
    base = S.start_solution(rng, S.degrees(ps), P)
    xs = base[None].repeat(B, 0)
    scale = np.logspace(-8, -1, B)
    xs[:, :, 0, 0] += scale[:, None] * rng.standard_normal((B, ps.n))
    ts = np.linspace(0.0, 0.05, B)
    sysd = H.System(ps)
    xd = dev(xs)
    status, iters, norms = H.newton(sysd, xd, gamma=gam, t=dev(ts), max_iter=4)
    status, iters, xg = host(status), host(iters), host(xd)
    for q in range(B):
        xo, r = O.newton(ps, g, gam, 1, float(ts[q]), xs[q], max_iter=4)
        assert status[q] == r.status and iters[q] == r.iters, (q, status[q], r.status)
        # an upper bound: one update per evaluation
        bound = _iterate_bound(ps, g, gam, float(ts[q]), xs[q], r.iters, P)
        assert np.abs(limb_diff(xg[q], xo)).max() <= bound, q


# ---------------------------------------------------------------------------
# tracking
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("P", [2, 4])
@pytest.mark.parametrize("n,d", [(4, 3), (1, 5)])
def test_track_closed_form_powers(H, P, n, d):
    """x_i^d = c_i (one variable, or several uncoupled ones): the endpoints
    are the closed-form ones and the step decisions the oracle's."""
    rng = S.rng_for(6, 50 + P + (0 if n == 4 else 100))
    cs = S.unit_complex(rng.uniform(0, 6.28, n), P)
    ps = S.diagonal_power_system(cs, d, P)
    gam = S.random_unit_gamma(rng, P)
    x0 = np.stack([S.start_solution(rng, np.full(n, d), P) for _ in range(3)])
    sysd = H.System(ps)
    xo, res = H.track_paths(sysd, gam, dev(x0))
    xo = host(xo)
    for q in range(3):
        assert res[q]["status"] == H.OK and res[q]["t"] == 1.0
        for i in range(n):
            ref = M.closed_form_endpoint(M.mp_complex(gam), M.mp_complex(cs[i]), d,
                                         M.mp_complex(x0[q, i]), steps=1500)
            assert abs(M.mp_complex(xo[q, i]) - ref) <= GATE[P]
        # and the same decisions as the oracle
        xr, r = O.track(ps, O.total_degree_start(ps), gam, 1, x0[q])
        assert (res[q]["steps"], res[q]["accepted"], res[q]["newton_iters"]) == \
               (r.steps, r.accepted, r.newton_iters)


@pytest.mark.parametrize("seed", [0, 3, 5, 6])
def test_track_small_system_parity(H, seed):
    P = 2
    ps = S.small_track_system(seed, P)
    g = O.total_degree_start(ps)
    rng = S.rng_for(0, 100 + seed)
    gam = S.random_unit_gamma(rng, P)
    x0 = S.ones_point(ps.n, P)
    sysd = H.System(ps)
    xg, res = H.track_paths(sysd, gam, dev(x0[None]))
    xg, res = host(xg)[0], res[0]
    xo, r = O.track(ps, g, gam, 1, x0)
    assert res["status"] == r.status
    assert (res["steps"], res["accepted"], res["newton_iters"]) == (r.steps, r.accepted, r.newton_iters)
    assert res["end_status"] == r.end_status and res["end_iters"] == r.end_iters
    if r.status == O.OK and r.end_status == O.OK:
        # two refined roots of the same regular solution: each is within
        # ||J^-1|| ||h|| of the root, plus the solves' 16 n kappa u
        _endpoint_close(ps, xg, xo, res["res_norm"], r.res_norm, P)


def _endpoint_close(ps, xg, xo, res_g, res_o, P):
    """|xg - xo| <= ||J^-1||_inf (||h(xg)|| + ||h(xo)||) + 16 n kappa u |x|,
    J the Jacobian of f at the oracle's endpoint (double is enough for the
    bound); the residual norms are those the refinement reported."""
    _, J = O.eval_jac(ps, xo)
    Jc = lead_complex(J).T
    kappa = np.linalg.cond(Jc)
    jinv = np.abs(np.linalg.inv(Jc)).sum(axis=1).max()
    scale = max(1.0, np.abs(lead_complex(xo)).max())
    bound = 2.0 * jinv * (res_g + res_o) + max(GATE[P], 16 * ps.n * kappa * UNIT[P]) * scale
    assert np.abs(limb_diff(xg, xo)).max() <= bound


def test_track_batch_matches_single(H):
    """Paths of one system tracked together give the same results as alone."""
    P = 2
    ps = S.small_track_system(5, P)
    rng = S.rng_for(0, 200)
    gam = S.random_unit_gamma(rng, P)
    degs = S.degrees(ps)
    x0 = np.stack([S.start_solution(rng, degs, P) for _ in range(4)])
    sysd = H.System(ps)
    xb, rb = H.track_paths(sysd, gam, dev(x0))
    xb = host(xb)
    for q in (0, 3):
        x1, r1 = H.track_paths(sysd, gam, dev(x0[q:q + 1]))
        assert _bitwise_equal(host(x1)[0], xb[q])
        assert r1[0].tobytes() == rb[q].tobytes()


# ---------------------------------------------------------------------------
# large systems: multi-workgroup MGS variants
# ---------------------------------------------------------------------------

def _solve_variant(H, variant, A, b):
    H.set_mgs_variant(variant)
    try:
        dx, R, status = H.mgs_solve(dev(A), dev(b))
        return host(dx), host(R), host(status)
    finally:
        H.set_mgs_variant(H.MGS_AUTO)


def _solve_variant_q(H, variant, A, b):
    """As _solve_variant, also returning Q (A overwritten) and the projected b."""
    H.set_mgs_variant(variant)
    try:
        Ad, bd = dev(A), dev(b)
        dx, R, status = H.mgs_solve(Ad, bd)
        return host(dx), host(R), host(status), host(Ad), host(bd)
    finally:
        H.set_mgs_variant(H.MGS_AUTO)


@pytest.mark.parametrize("P,N,n,B", [(2, 512, 512, 1), (2, 300, 257, 1), (4, 200, 200, 1),
                                     (2, 700, 300, 2), (4, 96, 600, 1)])
def test_mgs_big_variants_bitwise(H, P, N, n, B):
    """Right-looking and pipelined variants: identical bits in dx, R, Q and
    the projected right-hand side (the pipelined one with its columns
    resident in LDS, one or two problems per launch, more columns than
    workgroups, N > n); the one-workgroup variant within the solve
    tolerance."""
    if n > N:
        n, N = N, n
    rng = np.random.default_rng(N + n + P + B)
    A = np.stack([_rand_matrix(rng, N, n, P) for _ in range(B)])
    b = random_points(rng, B, N, P)
    print(f"mgs variants P={P} N={N} n={n} B={B}", flush=True)
    d2, R2, s2, Q2, b2 = _solve_variant_q(H, 2, A, b)
    d5, R5, s5, Q5, b5 = _solve_variant_q(H, 5, A, b)
    assert np.all(s2 == 0) and np.all(s5 == 0)
    for u, v in ((d2, d5), (R2, R5), (Q2, Q5), (b2, b5)):
        assert _bitwise_equal(u, v)
    d1, R1, s1 = _solve_variant(H, 1, A, b)
    for q in range(B):
        kappa = np.linalg.cond(lead_complex(A[q]).T)
        tol = max(GATE[P], 16 * n * kappa * UNIT[P])
        assert np.abs(limb_diff(d1[q], d2[q])).max() <= tol * np.abs(lead_complex(d2[q])).max()


@pytest.mark.parametrize("P,N,n,T", [(2, 300, 257, 3), (4, 200, 200, 8), (4, 256, 100, 16),
                                     (2, 64, 64, 16), (2, 65, 1, 1), (4, 40, 33, 5), (2, 129, 96, 7)])
def test_mgs_tiled_vs_oracle(H, P, N, n, T):
    """Tiled variant (panel width T: ragged last panel, rows not a multiple
    of 64, QD panels capped at eight columns) on two problems at once,
    against the oracle's MGS."""
    rng = np.random.default_rng(N * 3 + n + T + P)
    A = np.stack([_rand_matrix(rng, N, n, P) for _ in range(2)])
    b = random_points(rng, 2, N, P)
    H.set_mgs_panel(T)
    try:
        dx, R, st = _solve_variant(H, H.MGS_TILED, A, b)
    finally:
        H.set_mgs_panel(16)
    assert np.all(st == 0)
    for q in range(2):
        rc, dxo, _, Ro, _ = O.mgs_solve(P, A[q], b[q])
        assert rc == 0
        kappa = np.linalg.cond(lead_complex(A[q]).T)
        tol = max(GATE[P], 16 * n * kappa * UNIT[P])
        assert np.abs(limb_diff(dx[q], dxo)).max() <= tol * np.abs(lead_complex(dxo)).max()
        assert np.abs(limb_diff(R[q], Ro)).max() <= tol * np.abs(lead_complex(Ro)).max()


@pytest.mark.parametrize("T", [16, 8])
def test_mgs_tiled_512_vs_right_looking(H, T):
    """The full n = 512 size: tiled against right-looking (which the
    variants test ties to the other two), within the solve tolerance."""
    P, N, n = 2, 512, 512
    rng = np.random.default_rng(512 + T)
    A = _rand_matrix(rng, N, n, P)[None]
    b = random_points(rng, 1, N, P)
    d2, R2, s2 = _solve_variant(H, 2, A, b)
    H.set_mgs_panel(T)
    try:
        d4, R4, s4 = _solve_variant(H, H.MGS_TILED, A, b)
    finally:
        H.set_mgs_panel(16)
    assert s2[0] == 0 and s4[0] == 0
    kappa = np.linalg.cond(lead_complex(A[0]).T)
    tol = max(GATE[P], 16 * n * kappa * UNIT[P])
    assert np.abs(limb_diff(d4, d2)).max() <= tol * np.abs(lead_complex(d2)).max()
    assert np.abs(limb_diff(R4, R2)).max() <= tol * np.abs(lead_complex(R2)).max()


def test_mgs_big_backward_error(H):
    P, n = 2, 160
    rng = np.random.default_rng(160)
    A = _rand_matrix(rng, n, n, P)[None]
    b = random_points(rng, 1, n, P)
    for v in (2, 4, 5):
        d, _, s = _solve_variant(H, v, A, b)
        assert s[0] == 0
        assert _backward_error(A[0], b[0], d[0]) <= GATE[P]


def test_mgs_big_singular(H):
    P = 2
    rng = np.random.default_rng(5)
    A = _rand_matrix(rng, 200, 200, P)[None]
    A[0, 150] = 0.0
    b = random_points(rng, 1, 200, P)
    for v in (2, 4, 5):
        _, _, s = _solve_variant(H, v, A, b)
        assert s[0] == H.ESINGULAR
    # and a first column of zeros (the pipelined variant stops before it publishes any column)
    A[0, 0] = 0.0
    for v in (2, 5):
        _, _, s = _solve_variant(H, v, A, b)
        assert s[0] == H.ESINGULAR


def test_mgs_pipelined_wait_limit(H):
    """A pipelined solve whose waits run out (a bound of zero polls, set from
    the host, so that every kernel still ends normally) reports HCN_EDEVICE
    for its problem; with the default bound back, the next solve is whole
    and gives the right-looking bits."""
    P = 2
    rng = np.random.default_rng(11)
    A = _rand_matrix(rng, 300, 300, P)[None]
    b = random_points(rng, 1, 300, P)
    H.set_mgs_wait_limit(0)
    try:
        _, _, s = _solve_variant(H, 5, A, b)
    finally:
        H.set_mgs_wait_limit(H.MGS_WAIT_LIMIT)
    assert s[0] == H.EDEVICE
    d5, R5, s5 = _solve_variant(H, 5, A, b)
    d2, R2, s2 = _solve_variant(H, 2, A, b)
    assert s5[0] == 0 and s2[0] == 0
    assert _bitwise_equal(d2, d5) and _bitwise_equal(R2, R5)


def test_newton_step_sparse512_vs_oracle(H):
    """The full-size sparse n = 512 Newton step (every solve variant, the
    configurations the benchmark times) against the oracle's plain step;
    right-looking and pipelined bit for bit."""
    P = 2
    ps = S.sparse512_system(0, P)
    x = random_points(np.random.default_rng(12), 1, ps.n, P)
    sysd = H.System(ps)
    out = {}
    for v in (1, 2, 4, 5):
        H.set_mgs_variant(v)
        xd = dev(x)
        norms, status = H.newton_step(sysd, xd)
        H.set_mgs_variant(H.MGS_AUTO)
        assert host(status)[0] == 0
        out[v] = host(xd)[0]
    rc, xo, no = O.newton_step(ps, None, None, 1, 1.0, x[0])
    assert rc == 0
    f, J = O.eval_jac(ps, x[0])
    kappa = np.linalg.cond(lead_complex(J).T)
    tol = max(GATE[P], 16 * ps.n * kappa * UNIT[P])
    for v in (1, 2, 4, 5):
        assert np.abs(limb_diff(out[v], xo)).max() <= update_bound(tol, no[1], xo, P), v
    assert _bitwise_equal(out[2], out[5])


# ---------------------------------------------------------------------------
# mixed precision: FP64 Jacobian and solve, DD/QD residual and update
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("P", [2, 4])
def test_mixed_newton_reaches_extended_accuracy(H, P):
    """From near a planted root, the mixed-precision corrector reaches the
    root to DD/QD accuracy (checked in mpmath) and agrees with plain DD/QD
    Newton to the same tolerance."""
    rng = S.rng_for(3, 70 + P)
    base = S.random_system(rng, 12, 12, 10, (3, 6), (1, 2, 3), P)
    root = S.random_unit_point(rng, 12, P)
    f = M.planted_constant_terms(base, root)
    B = 4
    x0 = np.stack([root.copy() for _ in range(B)])
    x0[:, :, 0, 0] += 1e-6 * rng.standard_normal((B, 12))
    sysd = H.System(f)
    tol = GATE[P]
    xm = dev(x0)
    st_m, it_m, nm = H.newton(sysd, xm, max_iter=30, tol_res=tol, tol_dx=tol, max_eq_val=1.0,
                              mixed=True)
    xp = dev(x0)
    st_p, it_p, npn = H.newton(sysd, xp, max_iter=10, tol_res=tol, tol_dx=tol, max_eq_val=1.0)
    st_m, it_m, st_p = host(st_m), host(it_m), host(st_p)
    assert np.all(st_m == 0), st_m
    assert np.all(st_p == 0), st_p
    xm, xp = host(xm), host(xp)
    for q in range(B):
        err = max(abs(M.mp_complex(xm[q, i]) - M.mp_complex(root[i])) for i in range(12))
        assert err <= 100 * tol
        assert np.abs(limb_diff(xm[q], xp[q])).max() <= 100 * tol
        # residual at the result, at 320 bits
        fv, _ = M.eval_system(f, M.vec(xm[q]))
        assert max(abs(v) for v in fv) <= 100 * tol


def test_mixed_newton_fig2_branches(H):
    P = 2
    f = S.random_system(S.rng_for(3, 90), 6, 6, 5, (2, 3), (1, 2), P, const_term=True)
    x = random_points(np.random.default_rng(4), 2, 6, P)
    sysd = H.System(f)
    xd = dev(x)
    st, it, nr = H.newton(sysd, xd, max_eq_val=1e-30, mixed=True)
    assert np.all(host(st) == H.DIVERGED) and np.all(host(it) == 1)
    assert _bitwise_equal(host(xd), x)
    xd = dev(x)
    st, it, nr = H.newton(sysd, xd, max_iter=1, tol_res=1e-300, tol_dx=1e-300,
                          max_eq_val=1e300, mixed=True)
    assert np.all(host(st) == H.NOT_CONVERGED) and np.all(host(it) == 1)


# ---------------------------------------------------------------------------
# kernel variants from the tuning table
# ---------------------------------------------------------------------------

@contextlib.contextmanager
def _tune_restored(H, P, *Ns):
    """Restore the table entries of (P, N) for every N on exit."""
    saved = [(N, H.tune_get(P, N)) for N in Ns]
    try:
        yield
    finally:
        for N, (g, l) in saved:
            H.tune_set(P, N, g, l)


@pytest.mark.parametrize("P", [2, 4])
def test_tuned_variants(H, P):
    """LDS staging and register residency do not change a bit; other
    lane-group widths stay within the solve tolerance of the oracle."""
    ps = S.dense32_system(0, P)
    xs = S.dense32_points(3, 2, P)
    sysd = H.System(ps)
    out = {}
    with _tune_restored(H, P, ps.N):
        for grp in (8, 16, 32):
            for lds in (0, 1, 2):
                H.tune_set(P, ps.N, grp, lds)
                xd = dev(xs)
                _, status = H.newton_step(sysd, xd)
                assert np.all(host(status) == 0)
                out[(grp, lds)] = host(xd)
    for grp in (8, 16, 32):
        assert _bitwise_equal(out[(grp, 0)], out[(grp, 1)])
        assert _bitwise_equal(out[(grp, 0)], out[(grp, 2)])
    for q in range(2):
        rc, xo, no = O.newton_step(ps, None, None, 1, 1.0, xs[q])
        kappa = _kappa_at(ps, xs[q])
        tol = max(GATE[P], 16 * ps.n * kappa * UNIT[P])
        for grp in (8, 32):
            assert np.abs(limb_diff(out[(grp, 1)][q], xo)).max() <= update_bound(tol, no[1], xo, P)


def test_point_chunking_bitwise(H):
    """Launches over chunks of 64 points (the last one ragged) give bitwise
    the results of launches over the whole batch: one Newton step, the Fig. 2
    loop, the mixed-precision loop and path tracking."""
    import torch
    P = 2
    ps = S.dense32_system(0, P)
    xs = S.dense32_points(5, 200, P)
    sysd = H.System(ps)
    tp = S.small_track_system(3, P)
    tsys = H.System(tp)
    gam = S.random_unit_gamma(S.rng_for(0, 103), P)
    x0 = np.stack([S.ones_point(tp.n, P)] * 70)
    x0[1:] += S.random_unit_point(S.rng_for(0, 7), tp.n, P)[None] * 1e-3 * np.arange(1, 70)[:, None, None, None]
    out = {}
    try:
        for cb in (0, 1):
            H.set_chunk_bytes(cb)
            xd = dev(xs)
            norms, st = H.newton_step(sysd, xd)
            r = [host(xd), host(norms), host(st)]
            for mixed in (False, True):
                xd = dev(xs)
                st, it, nm = H.newton(sysd, xd, mixed=mixed)
                r += [host(xd), host(st), host(it), host(nm)]
            xo, res = H.track_paths(tsys, gam, dev(x0), max_steps=60)
            r += [host(xo), res.tobytes()]
            out[cb] = r
    finally:
        H.set_chunk_bytes(0)
    for a, b in zip(out[0], out[1]):
        if isinstance(a, bytes):
            assert a == b
        else:
            assert _bitwise_equal(a, b)


@pytest.mark.parametrize("P,N,n", [(2, 24, 24), (2, 32, 31), (2, 40, 24), (2, 64, 40), (2, 7, 5),
                                   (2, 97, 96), (2, 130, 100), (4, 24, 24), (4, 32, 20), (4, 9, 9)])
def test_mgs_register_storage_bitwise(H, P, N, n):
    """[A | b] held in registers (all columns, or a panel at a time,
    left-looking) gives bitwise the Q, R, projected b and dx of the
    global-memory form, for every lane-group width where it fits (ragged
    rows and columns, least squares, several panels), on three problems at
    once; a problem with a zero column stays singular."""
    rng = np.random.default_rng(N * 11 + n + P)
    A = np.stack([_rand_matrix(rng, N, n, P) for _ in range(3)])
    A[2, n // 2] = 0.0
    b = random_points(rng, 3, N, P)
    with _tune_restored(H, P, N):
        for grp in (8, 16, 32):
            res = {}
            for mode in (0, 2, 3):
                H.tune_set(P, N, grp, mode)
                Ad, bd = dev(A), dev(b)
                dx, R, st = H.mgs_solve(Ad, bd)
                res[mode] = (host(dx), host(R), host(st), host(Ad), host(bd))
            assert list(res[0][2]) == [H.OK, H.OK, H.ESINGULAR]
            for mode in (2, 3):
                assert list(res[mode][2]) == list(res[0][2])
                for q in range(2):
                    for a0, am in zip(res[0], res[mode]):
                        if np.ndim(a0) > 1:
                            assert _bitwise_equal(a0[q], am[q]), (grp, mode, q)


# ---------------------------------------------------------------------------
# slot-table batches of many systems
# ---------------------------------------------------------------------------

def _batch_cases(P):
    """(system, gamma, start point) for paths of several different systems."""
    cases = []
    for seed in (3, 5, 6):
        ps = S.small_track_system(seed, P)
        rng = S.rng_for(0, 100 + seed)
        gam = S.random_unit_gamma(rng, P)
        cases.append((ps, gam, S.ones_point(ps.n, P)))
    rng = S.rng_for(6, 11)
    cs = S.unit_complex(rng.uniform(0, 6.28, 5), P)
    ps = S.diagonal_power_system(cs, 3, P)
    gam = S.random_unit_gamma(rng, P)
    for _ in range(2):
        cases.append((ps, gam, S.start_solution(rng, np.full(5, 3), P)))
    return cases


@pytest.mark.parametrize("P", [2, 4])
def test_batch_matches_single_system_tracking(H, P):
    """Paths of several systems in one batch give bitwise the results of
    tracking each system on its own, alone or in any mix."""
    cases = _batch_cases(P)
    systems = {}
    for ps, _, _ in cases:
        if id(ps) not in systems:
            systems[id(ps)] = H.System(ps)
    # each path alone through the single-system tracker
    ref = []
    for ps, gam, x0 in cases:
        xo, res = H.track_paths(systems[id(ps)], gam, dev(x0[None]))
        ref.append((host(xo)[0], res[0]))
    maxs = max(systems[id(ps)].info().nslots for ps, _, _ in cases)
    bt = H.Batch(P, capacity=8, max_n=8, max_nslots=maxs)
    slots = [0, 2, 3, 5, 7]
    for slot, (ps, gam, x0) in zip(slots, cases):
        bt.add(slot, systems[id(ps)], gam, dev(x0))
    bt.run()
    n, done = bt.poll()
    assert n == 0 and all(done[s] == 1 for s in slots)
    for slot, (ps, gam, x0), (xr, rr) in zip(slots, cases, ref):
        x, r = bt.result(slot, ps.n)
        assert _bitwise_equal(host(x), xr)
        assert r.tobytes() == rr.tobytes()
    # a released slot takes a new path; the old paths are unaffected
    bt.release(2)
    ps, gam, x0 = cases[0]
    bt.add(2, systems[id(ps)], gam, dev(x0))
    bt.run()
    x, r = bt.result(2, ps.n)
    assert _bitwise_equal(host(x), ref[0][0]) and r.tobytes() == ref[0][1].tobytes()
    # one path alone in a batch
    bt2 = H.Batch(P, capacity=2, max_n=8, max_nslots=maxs)
    ps, gam, x0 = cases[3]
    bt2.add(1, systems[id(ps)], gam, dev(x0))
    bt2.run()
    x, r = bt2.result(1, ps.n)
    assert _bitwise_equal(host(x), ref[3][0]) and r.tobytes() == ref[3][1].tobytes()
    bt.free()
    bt2.free()


@pytest.mark.parametrize("P", [2, 4])
def test_batch_persistent_bitwise(H, P):
    """One persistent workgroup per slot gives bitwise the endpoints, step
    counts and work counters of the captured graph, for paths of several
    systems (some finishing long before others), stepped a few steps at a
    time or run to the end, and for a single path alone."""
    cases = _batch_cases(P)
    systems = {id(c[0]): H.System(c[0]) for c in cases}
    maxs = max(sd.info().nslots for sd in systems.values())
    out = {}
    for persistent in (False, True):
        bt = H.Batch(P, capacity=len(cases) + 1, max_n=8, max_nslots=maxs, persistent=persistent)
        for slot, (ps, gam, x0) in enumerate(cases):
            bt.add(slot + 1, systems[id(ps)], gam, dev(x0))
        bt.step(3)
        mid = bt.poll()
        bt.run(chunk=5)
        res = [bt.result(slot + 1, ps.n) for slot, (ps, _, _) in enumerate(cases)]
        out[persistent] = (mid[0], [(host(x), r.tobytes()) for x, r in res], bt.counts().tobytes())
        bt.free()
        b1 = H.Batch(P, capacity=1, max_n=8, max_nslots=maxs, persistent=persistent)
        ps, gam, x0 = cases[2]
        b1.add(0, systems[id(ps)], gam, dev(x0))
        b1.run(chunk=64)
        x, r = b1.result(0, ps.n)
        out[persistent] += ((host(x), r.tobytes()),)
        b1.free()
    g, p = out[False], out[True]
    assert g[0] == p[0] and g[2] == p[2]
    for (xg, rg), (xp, rp) in zip(g[1] + [g[3]], p[1] + [p[3]]):
        assert rg == rp and _bitwise_equal(xg, xp)


def test_batch_persistent_falls_back_to_graph(H):
    """A persistent batch in mixed precision, or with slots on the tiled
    solve, runs the captured graph: bitwise the results of a batch that never
    asked for the persistent form."""
    P = 2
    cases = _split_cases(P)
    systems = [H.System(ps) for ps, _, _ in cases]
    maxs = max(sd.info().nslots for sd in systems)
    for kw in (dict(mixed=True), dict(split_n=16)):
        out = {}
        for persistent in (False, True):
            bt = H.Batch(P, capacity=len(cases), max_n=40, max_nslots=maxs, max_steps=20,
                         persistent=persistent, **kw)
            for slot, ((ps, gam, x0), sd) in enumerate(zip(cases, systems)):
                bt.add(slot, sd, gam, dev(x0))
            bt.run()
            out[persistent] = [(host(x), r.tobytes()) for x, r in
                               (bt.result(slot, ps.n) for slot, (ps, _, _) in enumerate(cases))]
            bt.free()
        for (xa, ra), (xb, rb) in zip(out[False], out[True]):
            assert ra == rb and _bitwise_equal(xa, xb), kw


def test_batch_step_by_step_polling(H):
    """Stepping a few steps at a time and polling reports progress."""
    P = 2
    cases = _batch_cases(P)[:3]
    systems = [H.System(ps) for ps, _, _ in cases]
    maxs = max(s.info().nslots for s in systems)
    bt = H.Batch(P, capacity=4, max_n=8, max_nslots=maxs)
    for slot, ((ps, gam, x0), sd) in enumerate(zip(cases, systems)):
        bt.add(slot, sd, gam, dev(x0))
    n0, _ = bt.poll()
    assert n0 == 3
    bt.step(2)
    n1, done = bt.poll()
    assert n1 == 3 and not done.any()
    bt.run(chunk=16)
    n2, done = bt.poll()
    assert n2 == 0 and done[:3].all() and not done[3]
    for slot, (ps, gam, x0) in enumerate(cases):
        _, r = bt.result(slot, ps.n)
        xo, ro = O.track(ps, O.total_degree_start(ps), gam, 1, x0)
        assert (r["status"], r["steps"], r["accepted"]) == (ro.status, ro.steps, ro.accepted)


def _split_cases(P):
    """Paths of random systems of 20 and 40 unknowns (2..4 monomials of one
    or two variables, exponents 1..2, a constant term per equation) from
    total-degree start points, and one small system below the split."""
    cases = []
    for q, n in enumerate((20, 40, 20)):
        rng = S.rng_for(3, 900 + 10 * P + q)
        ps = S.random_system(rng, n, n, (2, 4), (1, 2), (1, 2), P, const_term=True)
        gam = S.random_unit_gamma(rng, P)
        cases.append((ps, gam, S.start_solution(rng, S.degrees(ps), P)))
    cases.append(_batch_cases(P)[0])
    return cases


@pytest.mark.parametrize("P", [2, 4])
def test_batch_split_alone_mix_and_oracle(H, P):
    """Slots of systems with n >= split_n solve with the tiled MGS (two and
    three panels, a ragged last one): each path gives the same bits alone
    and in a mix with a small system, and takes the oracle's step decisions
    (status, steps, accepted) to an endpoint within tolerance of the
    oracle's."""
    cases = _split_cases(P)
    systems = [H.System(ps) for ps, _, _ in cases]
    maxs = max(sd.info().nslots for sd in systems)
    kw = dict(max_steps=40)
    bt = H.Batch(P, capacity=6, max_n=40, max_nslots=maxs, split_n=16, **kw)
    slots = [5, 0, 3, 1]
    for slot, (ps, gam, x0), sd in zip(slots, cases, systems):
        bt.add(slot, sd, gam, dev(x0))
    bt.run()
    mix = [bt.result(slot, ps.n) for slot, (ps, _, _) in zip(slots, cases)]
    bt.free()
    for q, ((ps, gam, x0), sd) in enumerate(zip(cases, systems)):
        b1 = H.Batch(P, capacity=1, max_n=40, max_nslots=maxs, split_n=16, **kw)
        b1.add(0, sd, gam, dev(x0))
        b1.run()
        x1, r1 = b1.result(0, ps.n)
        b1.free()
        xm, rm = mix[q]
        assert _bitwise_equal(host(x1), host(xm)) and r1.tobytes() == rm.tobytes(), q
        xo, ro = O.track(ps, O.total_degree_start(ps), gam, 1, x0, max_steps=40)
        assert (r1["status"], r1["steps"], r1["accepted"]) == (ro.status, ro.steps, ro.accepted), q
        if ro.status == O.OK and ro.end_status == O.OK and r1["end_status"] == H.OK:
            _endpoint_close(ps, host(x1), xo, r1["res_norm"], ro.res_norm, P)


@pytest.mark.parametrize("mixed", [False, True])
def test_batch_panel_storage_bitwise(H, mixed):
    """Slots whose table entry asks for the left-looking panel MGS (grouped
    by rows per lane: 20, 40 and 70 rows at 8, 16 and 32 lanes) track to
    bitwise the endpoints and step counts of the global-memory form at the
    same lane-group width."""
    P = 2
    cases = []
    for q, n in enumerate((20, 40, 70)):
        rng = S.rng_for(3, 950 + q)
        ps = S.random_system(rng, n, n, (2, 4), (1, 2), (1, 2), P, const_term=True)
        cases.append((ps, S.random_unit_gamma(rng, P), S.start_solution(rng, S.degrees(ps), P)))
    cases.append(_batch_cases(P)[0])
    systems = [H.System(ps) for ps, _, _ in cases]
    maxs = max(sd.info().nslots for sd in systems)
    Ps = 1 if mixed else P
    Ns = sorted({ps.N for ps, _, _ in cases})
    out = {}
    with _tune_restored(H, Ps, *Ns):
        for grp in (8, 16, 32):
            for mode in (0, 3):
                for N in Ns:
                    H.tune_set(Ps, N, grp, mode)
                bt = H.Batch(P, capacity=5, max_n=70, max_nslots=maxs, mixed=mixed, max_steps=30)
                for slot, ((ps, gam, x0), sd) in enumerate(zip(cases, systems)):
                    bt.add(slot, sd, gam, dev(x0))
                bt.run()
                out[(grp, mode)] = [(host(x), r.tobytes())
                                    for x, r in (bt.result(slot, ps.n)
                                                 for slot, (ps, _, _) in enumerate(cases))]
                bt.free()
    for grp in (8, 16, 32):
        for q, ((x0, r0), (x1, r1)) in enumerate(zip(out[(grp, 0)], out[(grp, 3)])):
            assert r0 == r1 and _bitwise_equal(x0, x1), (grp, q)


@pytest.mark.parametrize("P", [2, 4])
def test_batch_mixed_precision_tracking(H, P):
    """The mixed-precision corrector (FP64 Jacobian and MGS, DD/QD residual
    and update) tracks to the same endpoints as the plain one, refined to
    the DD/QD tolerance, and the endpoints are roots at 320 bits."""
    cases = _batch_cases(P)
    systems = {}
    for ps, _, _ in cases:
        if id(ps) not in systems:
            systems[id(ps)] = H.System(ps)
    maxs = max(systems[id(ps)].info().nslots for ps, _, _ in cases)
    out = {}
    for mixed in (False, True):
        bt = H.Batch(P, capacity=len(cases), max_n=8, max_nslots=maxs, mixed=mixed)
        for slot, (ps, gam, x0) in enumerate(cases):
            bt.add(slot, systems[id(ps)], gam, dev(x0))
        bt.run()
        out[mixed] = [bt.result(slot, ps.n) for slot, (ps, _, _) in enumerate(cases)]
        bt.free()
    ok = 0
    for q, (ps, gam, x0) in enumerate(cases):
        (xp, rp), (xm, rm) = out[False][q], out[True][q]
        if rp["status"] != H.OK or rp["end_status"] != H.OK:
            continue
        assert rm["status"] == H.OK and rm["end_status"] == H.OK, (q, rm)
        xp, xm = host(xp), host(xm)
        scale = max(1.0, np.abs(lead_complex(xp)).max())
        _endpoint_close(ps, xm, xp, rm["res_norm"], rp["res_norm"], P)
        fv, _ = M.eval_system(ps, M.vec(xm))
        assert max(abs(v) for v in fv) <= 100 * GATE[P] * scale ** 6
        ok += 1
    assert ok >= 3


# ---------------------------------------------------------------------------
# serving: continuous batching
# ---------------------------------------------------------------------------

def test_server_results_equal_alone(H):
    """Requests of several systems and both precisions, admitted while others
    run (more requests than slots), give bitwise the results of tracking each
    path alone; a one-at-a-time server gives the same."""
    cases = [(P, c) for P in (2, 4) for c in _batch_cases(P)]
    systems = {}
    for P, (ps, _, _) in cases:
        if id(ps) not in systems:
            systems[id(ps)] = H.System(ps)
    alone = []
    for P, (ps, gam, x0) in cases:
        xo, res = H.track_paths(systems[id(ps)], gam, dev(x0[None]))
        alone.append((host(xo)[0], res[0]))
    maxs = max(s.info().nslots for s in systems.values())
    for serial in (False, True):
        # a budget for about three slots per precision: requests must queue
        probe = H.Batch(2, 1, 8, maxs)
        per = probe.device_bytes()
        probe.free()
        srv = H.Server(int(per * 3 / 0.5 * 1.5), max_n=8, max_nslots=maxs, qd_share=0.5,
                       steps_per_round=3, serial=serial)
        cap = srv.capacity()
        assert cap[0] >= 1 and cap[1] >= 1
        for rid, (P, (ps, gam, x0)) in enumerate(cases):
            srv.submit(rid, systems[id(ps)], gam, x0, srv.now())
        got = {}
        deadline = time.time() + 100
        while len(got) < len(cases) and time.time() < deadline:
            srv.pump()
            while True:
                r = srv.fetch()
                if r is None:
                    break
                got[r[0]] = r
        assert len(got) == len(cases)
        for rid in range(len(cases)):
            _, xo, res, ta, tb, tc = got[rid]
            assert _bitwise_equal(xo, alone[rid][0]), rid
            assert res.tobytes() == alone[rid][1].tobytes()
            assert ta <= tb <= tc
        srv.free()
