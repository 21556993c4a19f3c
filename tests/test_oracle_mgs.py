"""Pins of the oracle's modified Gram-Schmidt solver against 320-bit mpmath.

* backward stability: ||QR - A|| / ||A|| <= c n u;
* orthogonality lost in proportion to the condition number:
  ||Q^H Q - I|| <= c kappa u (MGS, Bjorck 1967);
* R's last column is Q^H b;
* planted solutions b = A x_true (formed at 320 bits) are recovered within
  c n kappa u;
* agreement with mpmath's own QR least-squares solver (qr_solve), square
  and overdetermined;
* an exactly zero column is reported singular.
"""
import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from oracle import mpref as M
from paper_1501_06625_amd import systems as S

UNIT = {2: 2.0 ** -104, 4: 2.0 ** -209}


def _rand_matrix(rng, N, n, P):
    th = rng.uniform(0, 2 * np.pi, N * n)
    mag = rng.uniform(0.2, 1.0, N * n)
    A = S.unit_complex(th, P).reshape(n, N, 2, P)
    with mpmath.workprec(M.PREC):
        for k in range(n):
            for i in range(N):
                A[k, i] = M.complex_limbs(M.mp_complex(A[k, i]) * mpmath.mpf(float(mag[k * N + i])), P)
    return A


def _kappa(A):
    n, N = A.shape[0], A.shape[1]
    Z = A[:, :, 0, 0] + 1j * A[:, :, 1, 0]
    return float(np.linalg.cond(Z.T))


def _mat(A):
    return M.colmajor(A)


@pytest.mark.parametrize("P,N,n", [(2, 6, 6), (2, 12, 9), (4, 7, 7), (2, 20, 20)])
def test_qr_invariants(P, N, n):
    rng = np.random.default_rng(N * 100 + n + P)
    A = _rand_matrix(rng, N, n, P)
    b = _rand_matrix(rng, N, 1, P)[0]
    rc, dx, Q, R, _ = O.mgs_solve(P, A, b)
    assert rc == 0
    u = UNIT[P]
    kappa = _kappa(A)
    Am, Qm = _mat(A), _mat(Q)
    Rm = mpmath.matrix(n, n)
    for j in range(n):
        for k in range(n):
            Rm[k, j] = M.mp_complex(R[j, k]) if k <= j else 0
            if k > j:
                assert np.all(R[j, k] == 0)
    normA = mpmath.mnorm(Am, 1)
    assert mpmath.mnorm(Qm * Rm - Am, 1) / normA <= 10 * n * u
    QhQ = Qm.H * Qm
    assert mpmath.mnorm(QhQ - mpmath.eye(n), 1) <= 10 * n * kappa * u
    # y = Q^H b
    bm = mpmath.matrix([M.mp_complex(b[i]) for i in range(N)])
    y = Qm.H * bm
    for k in range(n):
        assert abs(M.mp_complex(R[n, k]) - y[k]) <= 10 * n * kappa * u * mpmath.norm(bm)


@pytest.mark.parametrize("P,n", [(2, 8), (2, 16), (4, 8)])
def test_planted_solution(P, n):
    rng = np.random.default_rng(500 + n + P)
    A = _rand_matrix(rng, n, n, P)
    xt = _rand_matrix(rng, n, 1, P)[0]
    Am = _mat(A)
    xm = mpmath.matrix([M.mp_complex(xt[i]) for i in range(n)])
    bm = Am * xm
    b = np.array([M.complex_limbs(bm[i], P) for i in range(n)])
    rc, dx, _, _, _ = O.mgs_solve(P, A, b)
    assert rc == 0
    kappa = _kappa(A)
    err = max(abs(M.mp_complex(dx[i]) - xm[i]) for i in range(n))
    assert err <= 16 * n * kappa * UNIT[P] * mpmath.norm(xm, mpmath.inf)


@pytest.mark.parametrize("P,N,n", [(2, 10, 10), (2, 14, 8), (4, 9, 6)])
def test_matches_mpmath_qr_solve(P, N, n):
    rng = np.random.default_rng(900 + N + n + P)
    A = _rand_matrix(rng, N, n, P)
    b = _rand_matrix(rng, N, 1, P)[0]
    rc, dx, _, _, _ = O.mgs_solve(P, A, b)
    assert rc == 0
    Am = _mat(A)
    bm = mpmath.matrix([M.mp_complex(b[i]) for i in range(N)])
    ref, _ = mpmath.qr_solve(Am, bm)
    kappa = _kappa(A)
    for i in range(n):
        assert abs(M.mp_complex(dx[i]) - ref[i]) <= 16 * n * kappa * UNIT[P] * (1 + abs(ref[i])) * 4


def test_zero_column_is_singular():
    P = 2
    rng = np.random.default_rng(3)
    A = _rand_matrix(rng, 5, 5, P)
    A[2] = 0.0
    b = _rand_matrix(rng, 5, 1, P)[0]
    rc, *_ = O.mgs_solve(P, A, b)
    assert rc == O.ESINGULAR
    A2 = _rand_matrix(rng, 5, 5, P)
    A2[1, 3, 0, 0] = np.nan
    rc, *_ = O.mgs_solve(P, A2, b)
    assert rc == O.ESINGULAR


def test_diagonal_matrix_exact():
    """A = diag(2^e_k), b dyadic: Q = I, R = A, dx = b / A exactly."""
    P = 2
    n = 5
    A = np.zeros((n, n, 2, P))
    b = np.zeros((n, 2, P))
    for k in range(n):
        A[k, k, 0, 0] = 2.0 ** (k - 2)
        b[k, 0, 0] = 3.0 * 2.0 ** k
        b[k, 1, 0] = -2.0 ** -k
    rc, dx, Q, R, _ = O.mgs_solve(P, A, b)
    assert rc == 0
    for k in range(n):
        assert dx[k, 0, 0] == 3.0 * 2.0 ** k / 2.0 ** (k - 2)
        assert dx[k, 1, 0] == -2.0 ** -k / 2.0 ** (k - 2)
        assert Q[k, k, 0, 0] == 1.0


def test_threaded_columns_bitwise():
    """Large problems spread the trailing columns of each step over threads;
    each column sees the serial loop's operations, so Q, R and dx are the
    serial run's bit for bit (the serial run in a child process with one
    thread)."""
    import os
    import subprocess
    import sys
    rng = S.rng_for(9, 3)
    N = n = 160
    A = S.unit_complex(rng.uniform(0, 2 * np.pi, N * n), 2).reshape(n, N, 2, 2)
    b = S.unit_complex(rng.uniform(0, 2 * np.pi, N), 2).reshape(N, 2, 2)
    rc, dx, Q, R, _ = O.mgs_solve(2, A, b)
    assert rc == 0
    code = ("import sys, numpy as np; sys.path.insert(0, %r); from oracle import oracle as O; "
            "A = np.load(sys.argv[1]); b = np.load(sys.argv[2]); rc, dx, Q, R, _ = O.mgs_solve(2, A, b); "
            "np.save(sys.argv[3], np.concatenate([dx.ravel(), Q.ravel(), R.ravel()]))")
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        pa, pb, po = (os.path.join(d, f) for f in ("A.npy", "b.npy", "o.npy"))
        np.save(pa, A)
        np.save(pb, b)
        env = dict(os.environ, OMP_NUM_THREADS="1")
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        subprocess.check_call([sys.executable, "-c", code % root, pa, pb, po], env=env)
        serial = np.load(po)
    threaded = np.concatenate([dx.ravel(), Q.ravel(), R.ravel()])
    assert np.array_equal(serial.view(np.uint64), threaded.view(np.uint64))
