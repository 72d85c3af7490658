"""bem_field_noalloc (targets staged in the library's fixed device array, no
allocation in the call) against bem_field on the same problem and inputs, through
the C ABI: two calls in a row, the second with fewer targets, for the scattered
field at host points and for the far-field amplitude (needs an MI355X)."""

import ctypes

import numpy as np
import pytest

from synthetic import complex_normal, icosphere, nystrom3

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_noalloc_field_equals_bem_field():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import _abi
    from paper_1211_7177_amd.solver import BemProblem
    lib = _abi.load()
    q = nystrom3(icosphere(4))
    n = q["points"].shape[0]
    pb = BemProblem(q, 1.3, 2.25 + 0.2j, order=12, depth=3, nrhs_max=2)
    x = torch.from_numpy(complex_normal((2, n, 6), 4242)).cuda()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(77)
    for nt, kind in ((900, 0), (37, 0), (500, 1), (13, 1)):
        print("noalloc nt", nt, "kind", kind, flush=True)
        if kind == 1:
            pts = rng.standard_normal((nt, 3))
            pts /= np.linalg.norm(pts, axis=1, keepdims=True)
        else:
            pts = 2.0 + rng.random((nt, 3))
        pts = np.ascontiguousarray(pts)
        e0 = torch.full((2, nt, 3), float("nan"), dtype=torch.complex128, device="cuda")
        e1 = torch.full((2, nt, 3), float("nan"), dtype=torch.complex128, device="cuda")
        _abi.check(lib.bem_field(pb.h, ctypes.c_void_p(x.data_ptr()), 2, pts.ctypes.data, nt, 0, kind,
                                 ctypes.c_void_p(e0.data_ptr()), st))
        _abi.check(lib.bem_field_noalloc(pb.h, ctypes.c_void_p(x.data_ptr()), 2, pts.ctypes.data, nt, 0, kind,
                                         ctypes.c_void_p(e1.data_ptr()), st))
        a, b = e0.cpu().numpy(), e1.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b)
    big = np.ascontiguousarray(np.full((_abi.FIELD_NOALLOC_MAX + 1, 3), 3.0))
    out = torch.empty((1, 1, 3), dtype=torch.complex128, device="cuda")
    r = lib.bem_field_noalloc(pb.h, ctypes.c_void_p(x.data_ptr()), 1, big.ctypes.data, big.shape[0], 0, 0,
                              ctypes.c_void_p(out.data_ptr()), st)
    assert r == _abi.FMB_EINVAL and b"at most" in lib.fmb_last_error()
    pb.close()
