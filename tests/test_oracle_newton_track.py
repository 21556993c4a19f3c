"""Pins of the oracle's Newton corrector (Fig. 2) and tracker (Fig. 3).

* f_i = x_i^d - c_i decouples: one Newton iteration must equal the scalar
  map x - (x^d - c) / (d x^(d-1)) per coordinate (320-bit mpmath);
* from near a planted regular root the update norms shrink quadratically
  and the iterates reach the root to within 1e-28 (DD) / 1e-58 (QD);
* every branch of Fig. 2 and Fig. 3 is forced through its parameters;
* tracking x_i^d = c_i from g_i = x_i^d - 1 ends on the branch given by the
  closed form x(t)^d = (gamma (1-t) + t c) / (gamma (1-t) + t), followed in
  mpmath on a fine t grid.
"""
import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from oracle import mpref as M
from paper_1501_06625_amd import systems as S

TOL = {2: 1e-28, 4: 1e-58}


@pytest.mark.parametrize("P", [2, 4])
def test_newton_map_decoupled_powers(P):
    rng = S.rng_for(5, P)
    n, d = 4, 3
    cs = S.unit_complex(rng.uniform(0, 6.28, n), P)
    f = S.diagonal_power_system(cs, d, P)
    x = S.unit_complex(rng.uniform(0, 6.28, n), P)
    rc, x1, norms = O.newton_step(f, None, None, 1, 1.0, x)
    assert rc == 0
    for i in range(n):
        xi, ci = M.mp_complex(x[i]), M.mp_complex(cs[i])
        ref = xi - (xi ** d - ci) / (d * xi ** (d - 1))
        assert abs(M.mp_complex(x1[i]) - ref) <= TOL[P] * 0.01


@pytest.mark.parametrize("P", [2, 4])
def test_quadratic_convergence_planted_root(P):
    rng = S.rng_for(5, 10 + P)
    base = S.random_system(rng, 6, 6, 6, (2, 4), (1, 2), P)
    root = S.random_unit_point(rng, 6, P)
    f = M.planted_constant_terms(base, root)
    x = root.copy()
    x[:, 0, 0] += 1e-6 * rng.standard_normal(6)
    x[:, 1, 0] += 1e-6 * rng.standard_normal(6)
    dxs = []
    for _ in range(5 if P == 2 else 6):
        rc, x, norms = O.newton_step(f, None, None, 1, 1.0, x)
        assert rc == 0
        dxs.append(norms[1])
    # quadratic decrease while above the working-precision floor
    for a, b in zip(dxs, dxs[1:]):
        if b > (1e-29 if P == 2 else 1e-60):
            assert b <= 1e3 * a * a
    err = max(abs(M.mp_complex(x[i]) - M.mp_complex(root[i])) for i in range(6))
    assert err <= TOL[P]


def _small(P=2):
    rng = S.rng_for(5, 40)
    return S.random_system(rng, 5, 5, 5, (2, 3), (1, 2), P, const_term=True)


def test_fig2_branches():
    f = _small()
    x = S.random_unit_point(S.rng_for(5, 41), 5, 2)
    # residual above max_eq_val: fail at the first evaluation, x unchanged
    x1, r = O.newton(f, None, None, 1, 1.0, x, max_eq_val=1e-30)
    assert r.status == O.DIVERGED and r.iters == 1 and np.array_equal(x1, x)
    # residual below the tolerance: success without an update
    x1, r = O.newton(f, None, None, 1, 1.0, x, tol_res=1e30, max_eq_val=1e300)
    assert r.status == O.OK and r.iters == 1 and np.array_equal(x1, x)
    # iterations run out
    x1, r = O.newton(f, None, None, 1, 1.0, x, max_iter=1, tol_res=1e-300, tol_dx=1e-300,
                     max_eq_val=1e300)
    assert r.status == O.NOT_CONVERGED and r.iters == 1 and not np.array_equal(x1, x)
    # a NaN coefficient
    g = _small()
    g.coef = g.coef.copy()
    g.coef[3, 0, 0] = np.nan
    _, r = O.newton(g, None, None, 1, 1.0, x, max_eq_val=1e300)
    assert r.status == O.NAN
    # a variable that occurs nowhere: zero column, singular
    h = _small()
    h.var = np.where(h.var == 2, 1, h.var).astype(np.int32)
    _, r = O.newton(h, None, None, 1, 1.0, x, max_eq_val=1e300, tol_res=1e-300)
    assert r.status == O.ESINGULAR


@pytest.mark.parametrize("P", [2, 4])
def test_track_closed_form_powers(P):
    rng = S.rng_for(6, P)
    n, d = 3, 3
    cs = S.unit_complex(rng.uniform(0, 6.28, n), P)
    f = S.diagonal_power_system(cs, d, P)
    g = O.total_degree_start(f)
    gam = S.random_unit_gamma(rng, P)
    x0 = S.start_solution(rng, np.full(n, d), P)
    xo, r = O.track(f, g, gam, 1, x0)
    assert r.status == O.OK and r.t == 1.0
    for i in range(n):
        ref = M.closed_form_endpoint(M.mp_complex(gam), M.mp_complex(cs[i]), d,
                                     M.mp_complex(x0[i]), steps=2000)
        assert abs(M.mp_complex(xo[i]) - ref) <= TOL[P]


def test_fig3_branches():
    P = 2
    f = S.small_track_system(0, P)
    g = O.total_degree_start(f)
    rng = S.rng_for(0, 100)
    gam = S.random_unit_gamma(rng, P)
    x0 = S.ones_point(f.n, P)
    # too many steps
    _, r = O.track(f, g, gam, 1, x0, max_steps=2)
    assert r.status == O.MAX_STEPS and r.steps == 3
    # every corrector fails and the first halving falls below min_dt
    _, r = O.track(f, g, gam, 1, x0, max_eq_val=1e-300, min_dt=2.0 ** -4)
    assert r.status == O.STEP_TOO_SMALL and r.steps == 1 and r.t == 0.0
    # a NaN coefficient ends the path
    h = S.small_track_system(0, P)
    h.coef = h.coef.copy()
    h.coef[0, 0, 0] = np.nan
    _, r = O.track(h, O.total_degree_start(h), gam, 1, x0)
    assert r.status == O.NAN
    # the step limit counts rejected steps too (the schedule itself is
    # pinned on the linear paths below)
    _, r = O.track(f, g, gam, 1, x0, max_dt=0.5, max_steps=3)
    assert r.status == O.MAX_STEPS and r.steps == 4


def test_track_small_system_roots_verified():
    P = 2
    ok = 0
    for seed in (3, 5, 6):
        f = S.small_track_system(seed, P)
        g = O.total_degree_start(f)
        rng = S.rng_for(0, 100 + seed)
        gam = S.random_unit_gamma(rng, P)
        x0 = S.ones_point(f.n, P)
        xo, r = O.track(f, g, gam, 1, x0)
        xo2, r2 = O.track(f, g, gam, 1, x0)
        assert np.array_equal(xo, xo2) and r.steps == r2.steps
        assert r.status in (O.OK, O.MAX_STEPS, O.STEP_TOO_SMALL)
        if r.status == O.OK and r.end_status == O.OK:
            fv, _ = M.eval_system(f, M.vec(xo))
            assert max(abs(v) for v in fv) <= 1e-27
            ok += 1
    assert ok >= 2


# ---------------------------------------------------------------------------
# The step-size schedule of Fig. 3 on paths whose course is known exactly.
#
# With gamma = 1, g_i = x_i - 1 and f_i = x_i - c_i the homotopy
# h = (1 - t)(x - 1) + t (x - c) is x - (1 + t (c - 1)): every path is the
# straight line x(t) = 1 + t (c - 1) and J = 1.  Consequences used below:
#  * the constant prediction of the first step has residual t |1 - c|
#    (infinity norm of the leading limbs), and one Newton iteration from any
#    point lands on the line (up to DD rounding, ~1e-32);
#  * from the second accepted point on, extrapolation of any degree >= 1
#    through accepted points reproduces the line, so each later corrector
#    succeeds at its first evaluation.
# c = -1 + 2i gives |1 - c|_inf = 2.  The expected rows are written out by
# hand from the rules of Fig. 3: halve dt on a failure, count successes and
# double dt (up to max_dt) at every success once more than two are counted,
# t = min(1, t + dt).
# ---------------------------------------------------------------------------

def _line_homotopy(P, n=2):
    cs = np.zeros((n, 2, P))
    cs[:, 0, 0] = -1.0
    cs[:, 1, 0] = 2.0
    f = S.diagonal_power_system(cs, 1, P)
    g = O.total_degree_start(f)
    gam = np.zeros((2, P))
    gam[0, 0] = 1.0
    return f, g, gam, S.ones_point(n, P), cs


@pytest.mark.parametrize("order", [1, 2, 4])
def test_schedule_line_all_accepted(order):
    """Every step succeeds: 16 steps of max_dt = 1/16; 2 evaluations at the
    first (constant prediction, one solve, then a residual at rounding
    level), 1 at each later one (exact extrapolation)."""
    f, g, gam, x0, cs = _line_homotopy(2)
    xo, r, rows = O.track(f, g, gam, 1, x0, trace=True, predictor_order=order)
    assert r.status == O.OK and r.t == 1.0
    assert r.steps == 16 and r.accepted == 16 and r.newton_iters == 17
    assert [tuple(row) for row in rows] == \
        [(k / 16, 1 / 16, 1.0, 2.0 if k == 1 else 1.0) for k in range(1, 17)]
    for i in range(2):
        assert abs(M.mp_complex(xo[i]) - M.mp_complex(cs[i])) <= 1e-30


EXPECTED_FORCED = (
    # trial t, dt, accepted, evaluations
    [(1 / 16, 1 / 16, 0, 1),      # residual 1/8 > max_eq_val = 1/64: diverged
     (1 / 32, 1 / 32, 0, 1),      # 1/16 > 1/64
     (1 / 64, 1 / 64, 0, 1),      # 1/32 > 1/64
     (1 / 128, 1 / 128, 1, 2),    # 1/64 is not above it: solve, then converged
     (2 / 128, 1 / 128, 1, 1),    # second success, dt unchanged
     (3 / 128, 1 / 128, 1, 1),    # third success: dt doubles after it
     (5 / 128, 2 / 128, 1, 1),
     (9 / 128, 4 / 128, 1, 1),
     (17 / 128, 8 / 128, 1, 1)]   # dt reaches max_dt = 1/16 and stays
    + [((17 + 8 * q) / 128, 8 / 128, 1, 1) for q in range(1, 14)]
    + [(1.0, 8 / 128, 1, 1)])     # 129/128 clipped to 1


@pytest.mark.parametrize("order", [1, 3])
def test_schedule_line_forced_failures(order):
    """max_eq_val = 1/64 rejects the first three trials (halving dt each
    time); then the success count doubles dt from the fourth success on,
    capped at max_dt, and the last trial is clipped at t = 1."""
    f, g, gam, x0, cs = _line_homotopy(2)
    xo, r, rows = O.track(f, g, gam, 1, x0, trace=True, predictor_order=order,
                          max_eq_val=1.0 / 64)
    got = [tuple(float(v) for v in row) for row in rows]
    assert got == [tuple(float(v) for v in e) for e in EXPECTED_FORCED]
    assert r.status == O.OK and r.steps == len(EXPECTED_FORCED)
    assert r.accepted == len(EXPECTED_FORCED) - 3
    assert r.newton_iters == sum(e[3] for e in EXPECTED_FORCED)


def test_schedule_line_step_too_small():
    """With min_dt = 1/32 the second halving (to 1/64) ends the path."""
    f, g, gam, x0, _ = _line_homotopy(2)
    _, r, rows = O.track(f, g, gam, 1, x0, trace=True, max_eq_val=1.0 / 64, min_dt=1.0 / 32)
    assert r.status == O.STEP_TOO_SMALL and r.steps == 2 and r.t == 0.0
    assert [tuple(row[:3]) for row in rows] == [(1 / 16, 1 / 16, 0.0), (1 / 32, 1 / 32, 0.0)]


def test_schedule_line_corrector_budget():
    """max_iter = 1: the first trial's prediction (x = 1, residual 2t) fails
    until 2t < tol_res; tol_res = 1/256 accepts t = 1/1024 (residual 1/512)
    after rejecting 1/16 .. 1/512, seven halvings."""
    f, g, gam, x0, _ = _line_homotopy(2)
    _, r, rows = O.track(f, g, gam, 1, x0, trace=True, max_iter=1, tol_res=1.0 / 256,
                         tol_dx=1e-300, max_steps=8)
    assert [tuple(row[:3]) for row in rows[:8]] == \
        [(2.0 ** -e, 2.0 ** -e, 0.0) for e in range(4, 10)] + [(2.0 ** -10, 2.0 ** -10, 1.0)] \
        + [(2.0 ** -9, 2.0 ** -10, 0.0)]
    assert r.status == O.MAX_STEPS


# ---------------------------------------------------------------------------
# The predictor (Section 3.1): the interpolating polynomial of degree d
# through the last d + 1 accepted points, at the trial t.
# ---------------------------------------------------------------------------

def _poly_points(rng, P, deg, ts, n=3):
    """Values at ts of n random complex polynomials of degree deg (coefficients
    rounded to P limbs), and the polynomials (mpmath coefficients)."""
    coefs = [[M.mp_complex(S.unit_complex(rng.uniform(0, 6.28, 1), P)[0]) * (j + 1)
              for j in range(deg + 1)] for _ in range(n)]
    xs = np.zeros((len(ts), n, 2, P))
    for j, t in enumerate(ts):
        for i in range(n):
            v = sum(c * mpmath.mpf(t) ** q for q, c in enumerate(coefs[i]))
            xs[j, i] = M.complex_limbs(v, P)
    return xs, coefs


@pytest.mark.parametrize("P", [2, 4])
@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_predictor_reproduces_polynomials(P, deg):
    """Interpolation of degree d is exact on polynomials of degree <= d: the
    prediction matches the polynomial at t within the rounding of the data
    and of the weights."""
    rng = S.rng_for(6, 50 + 10 * P + deg)
    ts = [0.5 - q / 16 for q in range(deg + 1)]   # newest first, dyadic
    t = 0.5 + 1 / 16
    for data_deg in range(deg + 1):
        xs, coefs = _poly_points(rng, P, data_deg, ts)
        out = O.predict(P, ts, xs, t)
        for i in range(3):
            ref = sum(c * mpmath.mpf(t) ** q for q, c in enumerate(coefs[i]))
            assert abs(M.mp_complex(out[i]) - ref) <= 1e3 * TOL[P] * max(1, abs(ref))


def test_predictor_degree_matters():
    """A quadratic path is not reproduced by the secant (degree 1) but is by
    degree 2; the secant value is the closed form x1 + (t - t1)/(t1 - t0) (x1 - x0)."""
    rng = S.rng_for(6, 90)
    ts = [0.25, 0.125, 0.0]
    xs, coefs = _poly_points(rng, 2, 2, ts)
    t = 0.375
    sec = O.predict(2, ts[:2], xs[:2], t)
    quad = O.predict(2, ts, xs, t)
    for i in range(3):
        ref = sum(c * mpmath.mpf(t) ** q for q, c in enumerate(coefs[i]))
        x1, x0 = M.mp_complex(xs[0, i]), M.mp_complex(xs[1, i])
        secant = x1 + (mpmath.mpf(t) - ts[0]) / (mpmath.mpf(ts[0]) - ts[1]) * (x1 - x0)
        assert abs(M.mp_complex(sec[i]) - secant) <= 1e-29
        assert abs(M.mp_complex(quad[i]) - ref) <= 1e-29
        assert abs(secant - ref) > 1e-6
