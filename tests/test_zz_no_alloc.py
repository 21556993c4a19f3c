"""hcn_newton_step_static (the Newton step on the library's fixed device
workspace, which allocates nothing) against hcn_newton_step with a
workspace of its own.  Both run the same launches on the same inputs, so x,
the norms and the status must agree bit for bit.  Two calls in a row, the
second with fewer points, so that what the first left in the fixed array
cannot leak into the second; a batch whose workspace exceeds the array is
refused before any launch."""
import numpy as np
import pytest

from paper_1501_06625_amd import systems as S
from tests.gpu_util import random_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1501_06625_amd import hcn
    return hcn


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _same_bits(a, b):
    a = a.detach().cpu().numpy()
    b = b.detach().cpu().numpy()
    assert a.shape == b.shape
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def _compare(H, sysd, xs, gamma=None, t=None):
    import torch
    xa, xb = _dev(xs), _dev(xs)
    na, sa = H.newton_step(sysd, xa, gamma=gamma, t=t)
    nb, sb = H.newton_step_static(sysd, xb, gamma=gamma, t=t)
    torch.cuda.synchronize()
    _same_bits(sa, sb)
    _same_bits(na, nb)
    _same_bits(xa, xb)
    assert (sb.cpu().numpy() == 0).all()


@pytest.mark.parametrize("P", [2, 4])
def test_static_dense32(H, P):
    """dense n = 32: a batch of 40 points, then one of 7 other points"""
    ps = S.dense32_system(0, P)
    sysd = H.System(ps)
    rng = S.rng_for(9, 40 + P)
    assert H.lib().hcn_newton_ws_bytes(sysd.handle, 40) <= H.STATIC_WS_BYTES
    print(f"static dense32 P={P} B=40 then B=7", flush=True)
    _compare(H, sysd, random_points(rng, 40, ps.n, P))
    _compare(H, sysd, random_points(rng, 7, ps.n, P))


def test_static_homotopy(H):
    """the homotopy of equation (1) on the n = 8 tracking system, 64 then
    3 points at different t"""
    import torch
    P = 2
    ps = S.small_track_system(1, P)
    sysd = H.System(ps)
    rng = S.rng_for(9, 50)
    gam = S.random_unit_gamma(rng, P)
    for B in (64, 3):
        print(f"static homotopy B={B}", flush=True)
        xs = np.stack([S.start_solution(rng, S.degrees(ps), P) for _ in range(B)])
        t = torch.from_numpy(rng.uniform(0.0, 0.3, B)).cuda()
        _compare(H, sysd, xs, gamma=gam, t=t)


def test_static_sparse512(H):
    """n = 512: the solve across workgroups (a few points), 3 then 1"""
    P = 2
    ps = S.sparse512_system(0, P)
    sysd = H.System(ps)
    rng = S.rng_for(9, 60)
    assert H.lib().hcn_newton_ws_bytes(sysd.handle, 3) <= H.STATIC_WS_BYTES
    for B in (3, 1):
        print(f"static sparse512 B={B}", flush=True)
        _compare(H, sysd, random_points(rng, B, ps.n, P))


def test_static_refuses_oversize(H):
    """a batch whose workspace exceeds the fixed array: EINVAL, nothing launched"""
    ps = S.dense32_system(0, 2)
    sysd = H.System(ps)
    lib = H.lib()
    B = 1
    while lib.hcn_newton_ws_bytes(sysd.handle, B) <= H.STATIC_WS_BYTES:
        B *= 2
    rc = lib.hcn_newton_step_static(sysd.handle, None, 1, B, None, None, None, None, None)
    assert rc == H.EINVAL
    assert b"more than the fixed" in lib.hcn_last_error()
    # an empty batch is fine
    assert lib.hcn_newton_step_static(sysd.handle, None, 1, 0, None, None, None, None,
                                      None) == H.OK
