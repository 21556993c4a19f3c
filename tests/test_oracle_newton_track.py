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
    # halving and doubling: at least one failure and the steps add up
    xo, r = O.track(f, g, gam, 1, x0, max_dt=0.5)
    assert r.steps >= r.accepted


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
