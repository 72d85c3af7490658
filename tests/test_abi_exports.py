"""The C-ABI library loads and exports every symbol include/fmbem.h declares (no GPU needed)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fmbem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char \*)\s*\**\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_symbols_exported():
    from paper_1211_7177_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    lib = ctypes.CDLL(B.LIB)
    names = _declared()
    assert "fmm_plan" in names and "gmres_solve" in names and "fmm_matvec_adjoint" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_exposes_same_names():
    from paper_1211_7177_amd import _abi
    assert set(_declared()) <= set(_abi.EXPORTS)


def test_host_validation_without_gpu():
    """Argument errors are reported before any device work."""
    import numpy as np
    from paper_1211_7177_amd import _abi
    lib = _abi.load()
    h = ctypes.c_void_p()
    pts = np.zeros((1, 3))
    r = lib.fmm_plan(pts.ctypes.data, pts.ctypes.data, np.ones(1).ctypes.data, 1, 1.0, 0.0, 8, None, None,
                     ctypes.byref(h))
    assert r == _abi.FMB_EINVAL and b"n must be" in lib.fmb_last_error()
    pts = np.random.default_rng(0).standard_normal((10, 3))
    nrm = np.tile([0.0, 0.0, 1.0], (10, 1))
    w = np.ones(10)
    r = lib.fmm_plan(pts.ctypes.data, nrm.ctypes.data, w.ctypes.data, 10, 1.0, -0.5, 8, None, None, ctypes.byref(h))
    assert r == _abi.FMB_EINVAL and b"Im k" in lib.fmb_last_error()
    bad = nrm.copy()
    bad[3] = [0.0, 0.0, 1.1]
    r = lib.fmm_plan(pts.ctypes.data, bad.ctypes.data, w.ctypes.data, 10, 1.0, 0.0, 8, None, None, ctypes.byref(h))
    assert r == _abi.FMB_EINVAL and b"unit" in lib.fmb_last_error()
    pts2 = pts.copy()
    pts2[2, 1] = np.nan
    r = lib.fmm_plan(pts2.ctypes.data, nrm.ctypes.data, w.ctypes.data, 10, 1.0, 0.0, 8, None, None, ctypes.byref(h))
    assert r == _abi.FMB_EINVAL and b"non-finite" in lib.fmb_last_error()
    w2 = w.copy()
    w2[5] = 0.0
    r = lib.fmm_plan(pts.ctypes.data, nrm.ctypes.data, w2.ctypes.data, 10, 1.0, 0.0, 8, None, None, ctypes.byref(h))
    assert r == _abi.FMB_EINVAL and b"weights" in lib.fmb_last_error()
    r = lib.fmm_plan(pts.ctypes.data, nrm.ctypes.data, w.ctypes.data, 10, 1.0, 0.0, 99, None, None, ctypes.byref(h))
    assert r == _abi.FMB_EINVAL and b"order" in lib.fmb_last_error()
    assert lib.fmm_matvec_adjoint(None, None, None, None, 1, None) == _abi.FMB_EINVAL
    assert b"plan" in lib.fmb_last_error()
    assert lib.gmres_solve_group(None, 1, None, None, None, None, None, None) == _abi.FMB_EINVAL
    pts3 = pts.copy()
    pts3[7] = pts3[2]
    r = lib.fmm_plan(pts3.ctypes.data, nrm.ctypes.data, w.ctypes.data, 10, 1.0, 0.0, 8, None, None, ctypes.byref(h))
    assert r == _abi.FMB_EINVAL and b"duplicate points 2 and 7" in lib.fmb_last_error()

    # shape-derivative entry points: every check happens on the host
    assert lib.bem_shape_pairs(None, None, None, None, 10, 1.0, 0.0, None, None, None, None, None, None,
                               None) == _abi.FMB_EINVAL
    assert b"pointer" in lib.fmb_last_error()
    out, out2 = ctypes.c_void_p(16), ctypes.c_void_p(32)
    ids, tv10 = np.arange(10, dtype=np.int32), np.zeros((10, 3, 3))
    for n_, ntri_, mode, want in ((10, 5, 2, b"1 or 3 nodes"), (10, 10, 2, b"3 nodes per triangle"),
                                  (10, 10, 7, b"mode")):
        r = lib.bem_self_blocks(pts.ctypes.data, nrm.ctypes.data, ids.ctypes.data, tv10.ctypes.data, n_, ntri_,
                                mode, 1.0, 0.0, out, out2, None)
        assert r == _abi.FMB_EINVAL and want in lib.fmb_last_error(), lib.fmb_last_error()
    pts9, bad9, nrm9, tv3 = pts[:9].copy(), bad[:9].copy(), nrm[:9].copy(), np.zeros((3, 3, 3))
    tri9 = np.arange(9, dtype=np.int32) // 3
    r = lib.bem_self_blocks(pts9.ctypes.data, bad9.ctypes.data, tri9.ctypes.data, tv3.ctypes.data, 9, 3, 2, 1.0,
                            0.0, out, out2, None)
    assert r == _abi.FMB_EINVAL and b"unit" in lib.fmb_last_error()
    badtri = tri9.copy()
    badtri[4] = 3
    r = lib.bem_self_blocks(pts9.ctypes.data, nrm9.ctypes.data, badtri.ctypes.data, tv3.ctypes.data, 9, 3, 2, 1.0,
                            0.0, out, out2, None)
    assert r == _abi.FMB_EINVAL and b"point_tri" in lib.fmb_last_error()


def test_solver_option_mapping():
    """The Python solve options reach the C struct: mixed False/True/"nested" as 0/1/2."""
    from paper_1211_7177_amd import _abi, solver
    lib = _abi.load()
    for mixed, code in ((False, 0), (True, 1), ("nested", 2)):
        o = solver._opts(lib, 1e-6, 50, 100, True, mixed, 1e-2, 30, False)
        assert o.mixed == code and o.restart == 50 and o.inner_maxit == 30 and o.precond == 1
    for precond, code in ((False, 0), (True, 1), ("block", 1), ("gmres", 2)):
        assert solver._opts(lib, 1e-6, 50, 100, precond, False, 1e-2, 30, False).precond == code
