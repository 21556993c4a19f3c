"""The C-ABI library loads on the CPU and exports every function that
include/hcn.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hcn.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hcn_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("hcn_sys_load", "hcn_eval_jac", "hcn_mgs_solve", "hcn_newton_step",
                 "hcn_track_paths"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1501_06625_amd", "libhcn.so"))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_match_header():
    from paper_1501_06625_amd import hcn
    assert sorted(hcn.EXPORTS) == _declared()


def test_host_side_argument_errors():
    """EINVAL paths run on the host before any device work."""
    from paper_1501_06625_amd import hcn
    lib = hcn.lib()
    h = ctypes.c_void_p()
    import numpy as np
    z = np.zeros(4, dtype=np.int32)
    p = z.ctypes.data_as(ctypes.c_void_p)
    assert lib.hcn_sys_load(ctypes.byref(h), 2, 2, 3, p, p, p, p, p) == hcn.EINVAL
    assert b"P must be 1, 2 or 4" in lib.hcn_last_error()
    assert lib.hcn_sys_load(ctypes.byref(h), 1, 2, 2, p, p, p, p, p) == hcn.EINVAL
    assert lib.hcn_mgs_solve(1, 2, 3, 2, None, None, None, None, None, None, 0, None) == hcn.EINVAL
    assert lib.hcn_elementwise(99, 2, 1, None, None, None, None) == hcn.EINVAL
    assert lib.hcn_version() == 100
    assert lib.hcn_set_mgs_variant(6) == hcn.EINVAL
    # the column-resident variant is not available
    assert lib.hcn_set_mgs_variant(3) == hcn.EINVAL
    assert lib.hcn_set_mgs_variant(0) == hcn.OK
    # extrapolation beyond degree 4 is refused before any allocation
    bad = hcn.track_params(2, predictor_order=5)
    assert lib.hcn_batch_create(ctypes.byref(h), 2, 4, 8, 64, 4, ctypes.byref(bad), 1, 0) == hcn.EINVAL
    neg = hcn.track_params(2, predictor_order=-1)
    assert lib.hcn_batch_create(ctypes.byref(h), 2, 4, 8, 64, 4, ctypes.byref(neg), 1, 0) == hcn.EINVAL
    # complex double batches are not offered (DD and QD only)
    ok = hcn.track_params(2)
    assert lib.hcn_batch_create(ctypes.byref(h), 1, 4, 8, 64, 4, ctypes.byref(ok), 1, 0) == hcn.EINVAL
    assert lib.hcn_set_mgs_panel(0) == hcn.EINVAL
    assert lib.hcn_set_mgs_panel(17) == hcn.EINVAL
    assert lib.hcn_set_mgs_wait_limit(-1) == hcn.EINVAL
    assert lib.hcn_set_mgs_wait_limit(hcn.MGS_WAIT_LIMIT) == hcn.OK
    assert lib.hcn_tune_set(2, 32, 16, 5) == hcn.EINVAL
    assert lib.hcn_batch_set_persistent(None, 1) == hcn.EINVAL
    assert lib.hcn_tune_set(2, 32, 12, 0) == hcn.EINVAL
    # a repeated variable inside a monomial is rejected
    eq_ptr = np.array([0, 1, 1], dtype=np.int32)
    mon_ptr = np.array([0, 2], dtype=np.int32)
    var = np.array([0, 0], dtype=np.int32)
    ex = np.array([1, 1], dtype=np.int32)
    coef = np.zeros(4)
    q = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.hcn_sys_load(ctypes.byref(h), 2, 2, 2, q(eq_ptr), q(mon_ptr), q(var), q(ex),
                            q(coef)) == hcn.EINVAL
    assert b"repeated" in lib.hcn_last_error()
    # a monomial cannot have more factors than there are unknowns
    assert lib.hcn_sys_load(ctypes.byref(h), 1, 1, 2, q(eq_ptr), q(mon_ptr), q(var), q(ex),
                            q(coef)) == hcn.EINVAL
    assert b"pairs" in lib.hcn_last_error()
