"""Edge cases of the FMM product on the GPU: degenerate meshes, leaves larger
than a block, and rejected arguments (needs an MI355X)."""

import numpy as np
import pytest

from oracle.corrections import self_blocks
from oracle.direct import apply_corrections
from oracle.native import point_sum_c
from synthetic import complex_normal, nystrom3, seed_for, torus
from synthetic.meshes import Mesh

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import _abi
    _abi.load()
    return _abi


def _plan(abi, q, k, order, depth, precision="fp64", nrhs_max=1, translate="fp32", corr="linear"):
    return abi.Plan(q["points"], q["normals"], q["weights"], k, order, depth=depth, precision=precision,
                    nrhs_max=nrhs_max, corr=corr, point_tri=q["point_tri"], tri_vertices=q["tri_vertices"],
                    translate=translate)


def _ref(q, k, a, b, rows=None):
    y = point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b, rows=rows)
    blk = self_blocks(q["points"], q["normals"], q["point_tri"], q["tri_vertices"], k, mode="linear")
    return y + apply_corrections(q["normals"], q["point_tri"], blk, a, b, rows=rows)


def _rel(y, ref):
    return np.linalg.norm(y - ref) / np.linalg.norm(ref)


def _tri_mesh(offsets):
    v, t = [], []
    base = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.2, 0.9, 0.0]])
    for i, o in enumerate(offsets):
        v.append(base + np.asarray(o))
        t.append([3 * i, 3 * i + 1, 3 * i + 2])
    return Mesh(np.concatenate(v), np.array(t, dtype=np.int32))


def test_depth_that_splits_a_triangle_is_refused(abi):
    """Nodes of one triangle must share the near field.  A single triangle fills
    its own bounding cube, so even depth 2 splits it: refused.  The torus and the
    sphere split at depths 7 and 5 (counted on the oracle's octree): refused when
    asked for, and an automatic depth driven deep by a tiny leaf target steps
    back to a depth that keeps every triangle together."""
    from synthetic import icosphere
    q1 = nystrom3(_tri_mesh([[0, 0, 0]]))
    with pytest.raises(abi.FmbError, match="too deep"):
        _plan(abi, q1, 1.0, 8, 0)
    qt = nystrom3(torus(1.0, 0.3, 200, 50))
    with pytest.raises(abi.FmbError, match="too deep"):
        _plan(abi, qt, 4.0, 8, 7)
    qs = nystrom3(icosphere(8))
    with pytest.raises(abi.FmbError, match="too deep"):
        _plan(abi, qs, 1.0, 8, 5)
    P = abi.Plan(qs["points"], qs["normals"], qs["weights"], 1.0, 8, depth=0, point_tri=qs["point_tri"],
                 tri_vertices=qs["tri_vertices"], leaf_target=1)
    assert P.info()["depth"] <= 4
    P.close()


@pytest.mark.parametrize("offsets", [[[0, 0, 0], [7.0, 3.0, -2.0]], [[0, 0, 0], [1.5, 0, 0], [0, 2.0, 1.0]]])
def test_few_triangles(abi, offsets):
    """Two or three isolated triangles (a handful of nodes, tiny trees with few or
    no far-field pairs), FP64 and FP32."""
    q = nystrom3(_tri_mesh(offsets))
    n = q["points"].shape[0]
    a = complex_normal((n, 3), 171)
    b = complex_normal((n, 3), 172)
    ref = _ref(q, 1.3 + 0.2j, a, b)
    # far-field boxes here sit about 0.43 of their distance apart, so order 20 (FP64)
    # truncates near 1e-7 and order 12 (FP32) near 4e-5
    for prec, order, tol in (("fp64", 20, 1e-6), ("fp32", 12, 2e-4)):
        print("triangles", len(offsets), prec, flush=True)
        P = _plan(abi, q, 1.3 + 0.2j, order, 0, precision=prec)
        dt = torch.complex128 if prec == "fp64" else torch.complex64
        y = P.matvec(torch.from_numpy(a).to(dt).cuda(), torch.from_numpy(b).to(dt).cuda()).cpu().numpy()
        assert _rel(y, ref) <= tol
        P.close()


def test_leaves_larger_than_a_block(abi):
    """The 60k-node torus at depth 2: leaves of over a thousand nodes, more than
    one block of targets and of sources; FP64 p = 16 and FP32 p = 10 with 3
    right-hand sides, on 128 sampled rows."""
    q = nystrom3(torus(1.0, 0.3, 200, 50))
    n = q["points"].shape[0]
    a = complex_normal((3, n, 3), seed_for(2, "a"))
    b = complex_normal((3, n, 3), seed_for(2, "b"))
    rows = np.sort(np.random.default_rng(seed_for(2, "rows") + 2).choice(n, 128, replace=False))
    ref = _ref(q, 4.0, a, b, rows=rows)
    for prec, order, tol in (("fp64", 16, 1e-6), ("fp32", 10, 1e-3)):
        print("torus depth 2", prec, flush=True)
        P = _plan(abi, q, 4.0, order, 2, precision=prec, nrhs_max=3)
        dt = torch.complex128 if prec == "fp64" else torch.complex64
        assert max(P.info()["nbox"]) <= 64
        y = P.matvec(torch.from_numpy(a).to(dt).cuda(), torch.from_numpy(b).to(dt).cuda()).cpu().numpy()
        for r in range(3):
            assert _rel(y[r][rows], ref[r]) <= tol
        P.close()


def test_rejected_arguments(abi):
    q = nystrom3(_tri_mesh([[0, 0, 0], [3.0, 0, 0]]))
    n = q["points"].shape[0]
    P = _plan(abi, q, 1.0, 8, 0, nrhs_max=2)
    a = torch.zeros((3, n, 3), dtype=torch.complex128, device="cuda")
    lib = P._lib
    y = torch.zeros_like(a)
    import ctypes
    pa, py = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(y.data_ptr())
    assert lib.fmm_matvec(P.h, pa, pa, py, 3, None) == abi.FMB_EINVAL          # nrhs > nrhs_max
    assert lib.fmm_matvec(P.h, pa, pa, py, 0, None) == abi.FMB_EINVAL          # nrhs = 0
    assert lib.fmm_matvec(P.h, pa, pa, pa, 1, None) == abi.FMB_EINVAL          # y aliases a
    assert lib.fmm_matvec_adjoint(P.h, pa, pa, py, 1, None) == abi.FMB_EINVAL  # a_bar aliases y
    P.close()


def test_field_entry_points_reject_bad_arguments(abi):
    """bem_field with an unknown kind or a far field of the interior, far-field
    directions that are not unit vectors (also for bem_far_field_adjoint), and an
    FMM field target that coincides with a node are errors, reported before any
    kernel reads the arguments; the problem stays usable afterwards."""
    from paper_1211_7177_amd.solver import BemProblem
    from synthetic import icosphere
    q = nystrom3(icosphere(2))
    n = q["points"].shape[0]
    pb = BemProblem(q, 1.0, 2.25, order=10, depth=2)
    x = torch.from_numpy(complex_normal((1, n, 6), 201)).cuda()
    out = torch.empty((1, 1, 3), dtype=torch.complex128, device="cuda")
    pts = np.array([[0.0, 0.0, 3.0]])
    lib = abi.load()
    import ctypes
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for kind, region in ((3, 0), (-1, 0), (1, 1), (2, 1)):
        with pytest.raises(abi.FmbError):
            abi.check(lib.bem_field(pb.h, ctypes.c_void_p(x.data_ptr()), 1, pts.ctypes.data, 1, region, kind,
                                    ctypes.c_void_p(out.data_ptr()), st))
    with pytest.raises(abi.FmbError, match="unit"):
        pb.field(x, np.array([[0.0, 0.0, 2.0]]), far=True)
    with pytest.raises(abi.FmbError, match="unit"):
        pb.far_field_adjoint(torch.zeros((1, 1, 3), dtype=torch.complex128, device="cuda"), [[0.0, 0.6, 0.6]])
    with pytest.raises(abi.FmbError):
        pb.field(x, q["points"][:2].copy(), method="fmm")
    E = pb.field(x, pts).cpu().numpy()
    Ef = pb.field(x, pts, method="fmm", order=20).cpu().numpy()
    assert np.isfinite(E).all() and _rel(Ef, E) <= 1e-6          # 3.5e-6 at p = 16 for this lone far target
    pb.close()


def test_problem_create_rejects_shared_or_mismatched_plans(abi):
    """bem_problem_create refuses one plan passed as both p0 and p1 (their products
    run concurrently on the plans' own workspaces), an interior plan whose
    wavenumber is not k0 sqrt(eps mu) (Sec. 2.1, eq. 2.13), and FP32 plans whose
    wavenumbers differ from their FP64 twins."""
    import ctypes
    from synthetic import icosphere
    q = nystrom3(icosphere(2))
    lib = abi.load()
    eps = np.array([2.25, 0.0])
    mu = np.array([1.0, 0.0])
    k0, k1 = 1.0, 1.5
    p0 = _plan(abi, q, k0, 6, 2)
    p1 = _plan(abi, q, k1, 6, 2)
    pw = _plan(abi, q, 1.4, 6, 2)                                   # not k0 sqrt(2.25)
    f0 = _plan(abi, q, k0, 5, 2, precision="fp32")
    f1 = _plan(abi, q, k1, 5, 2, precision="fp32")
    fw = _plan(abi, q, 1.4, 5, 2, precision="fp32")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def create(a, b, c=None, d=None):
        h = ctypes.c_void_p()
        code = lib.bem_problem_create(a.h, b.h, c.h if c else None, d.h if d else None, eps.ctypes.data,
                                      mu.ctypes.data, st, ctypes.byref(h))
        if code == 0:
            lib.bem_problem_destroy(h)
        return code

    assert create(p0, p0) == abi.FMB_EINVAL
    assert create(p0, pw) == abi.FMB_EINVAL
    assert create(p0, p1, f0, f0) == abi.FMB_EINVAL
    assert create(p0, p1, f0, fw) == abi.FMB_EINVAL
    assert create(p0, p1, f1, f0) == abi.FMB_EINVAL
    assert create(p0, p1) == abi.FMB_OK
    assert create(p0, p1, f0, f1) == abi.FMB_OK
    for p in (p0, p1, pw, f0, f1, fw):
        p.close()
