"""Shape gradient on the GPU: the two device entry points against the oracle
element by element, and dC/dv at every vertex against differences of solves,
the oracle's solves, the invariances C_sca has, and Mie (needs an MI355X)."""

import numpy as np
import pytest

from oracle import mie
from oracle.bem import BemProblem as OracleBem
from oracle.corrections import self_blocks as oracle_blocks
from oracle.gmres import gmres_solve as oracle_gmres
from oracle.shape import cross_section_far, cross_section_surface, pair_derivatives
from synthetic import complex_normal, icosphere, nystrom3, seed_for, torus

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

D, POL = [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import _abi
    _abi.load()
    return _abi


def _g(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t if dtype is None else t.to(dtype)


def _maxrel(got, ref):
    return np.max(np.abs(got - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("k", [1.3, 2.0 + 0.7j, complex(0.5161, 15.5034)])
def test_shape_pairs_match_oracle(abi, k):
    """dB/ds, dB/dn, dB/dw of the point sum on a 1440-node torus (11 tiles of 128
    and a ragged tail) against the oracle's direct formula, FP64 to 1e-12."""
    q = nystrom3(torus(1.0, 0.3, 24, 10))
    n = q["points"].shape[0]
    lam, a, b = (complex_normal((n, 3), seed_for(7, 0) + i) for i in range(3))
    print("shape pairs k=", k, "n", n, flush=True)
    got = abi.shape_pairs(_g(q["points"]), _g(q["normals"]), _g(q["weights"]), _g(q["point_tri"]), k,
                          _g(lam), _g(a), _g(b))
    ref = pair_derivatives(q["points"], q["normals"], q["weights"], q["point_tri"], k, lam, a, b)
    for name, g_, r in zip(("ds", "dn", "dw"), got, ref):
        err = _maxrel(g_.cpu().numpy(), r)
        print("  %s max rel %.2e" % (name, err), flush=True)
        assert err <= 1e-12


def test_shape_pairs_edge_cases(abi):
    """A single triangle has no pairs (all zero); 130 scattered nodes in pairs
    sharing a 'triangle' index (two tiles, the second holding 2 nodes)."""
    q = nystrom3(torus(1.0, 0.3, 4, 3))
    z = [_g(np.ones((3, 3), np.complex128)) for _ in range(3)]
    got = abi.shape_pairs(_g(q["points"][:3]), _g(q["normals"][:3]), _g(q["weights"][:3]),
                          _g(np.zeros(3, np.int32)), 1.0, *z)
    assert all(torch.all(t == 0).item() for t in got)
    rng = np.random.default_rng(11)
    n = 130
    pts = rng.standard_normal((n, 3))
    nrm = rng.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.5, n)
    tri = (np.arange(n) // 2).astype(np.int32)
    lam, a, b = (complex_normal((n, 3), 90 + i) for i in range(3))
    got = abi.shape_pairs(_g(pts), _g(nrm), _g(w), _g(tri), 0.8 + 0.1j, _g(lam), _g(a), _g(b))
    ref = pair_derivatives(pts, nrm, w, tri, 0.8 + 0.1j, lam, a, b)
    for g_, r in zip(got, ref):
        assert _maxrel(g_.cpu().numpy(), r) <= 1e-12


@pytest.mark.parametrize("k,mode", [(1.3, "linear"), (complex(0.5161, 15.5034), "linear"), (40.0, "linear"),
                                    (2.0 + 0.5j, "mean")])
def test_self_blocks_match_oracle(abi, k, mode):
    """The self-triangle blocks of a given geometry (Appendix B) against the
    oracle's, every entry, including |k| h beyond the series branch (k = 40)."""
    q = nystrom3(torus(1.0, 0.3, 24, 10))
    print("self blocks k=", k, mode, flush=True)
    dv, dg = abi.self_blocks(q["points"], q["normals"], q["point_tri"], q["tri_vertices"], k, mode=mode)
    _, rv, rg = oracle_blocks(q["points"], q["normals"], q["point_tri"], q["tri_vertices"], k, mode=mode)
    ev, eg = _maxrel(dv.cpu().numpy(), rv), _maxrel(dg.cpu().numpy(), rg)
    print("  dV %.2e dG %.2e" % (ev, eg), flush=True)
    assert ev <= 1e-11 and eg <= 1e-11


def test_self_blocks_reject_linear_on_one_node_triangles(abi):
    q = nystrom3(torus(1.0, 0.3, 6, 4))
    with pytest.raises(abi.FmbError, match="3 nodes per triangle"):
        abi.self_blocks(q["points"][::3], q["normals"][::3], np.arange(len(q["tri_vertices"]), dtype=np.int32),
                        q["tri_vertices"], 1.0, mode="linear")


# ---------------------------------------------------------------------------
# the vertex gradient
# ---------------------------------------------------------------------------

PLAN = dict(order=20, depth=2, tol=1e-12, restart=200)


def _product_C(V, F, k0, eps, functional):
    from paper_1211_7177_amd.gradients import _functional
    from paper_1211_7177_amd.shape import nodes_of_mesh
    from paper_1211_7177_amd.solver import BemProblem
    q = nodes_of_mesh(V, F)
    pb = BemProblem(q, k0, eps, order=20, depth=2)
    x, info = pb.solve(pb.rhs_planewave(D, POL), tol=1e-12, restart=200, maxit=4000)
    C = _functional(functional, pb, q, k0, x, D, POL).item()
    pb.close()
    return C


def _direction(V, F, seed):
    from paper_1211_7177_amd.shape import vertex_normals
    r = np.random.default_rng(seed).standard_normal(len(V))
    return r[:, None] * vertex_normals(V, F)


@pytest.fixture(scope="module")
def ring_case(abi):
    """A torus of 256 triangles (768 nodes), eps = 2.25 + 0.5i, k0 = 1.5."""
    from paper_1211_7177_amd.shape import cross_section_and_vertex_gradient
    m = torus(1.0, 0.4, 16, 8)
    V, F = m.vertices.copy(), m.triangles.copy()
    out = {}
    for fun in ("far", "surface"):
        print("vertex gradient torus", fun, flush=True)
        out[fun] = cross_section_and_vertex_gradient(V, F, 1.5, 2.25 + 0.5j, D, POL, functional=fun, **PLAN)
    return V, F, out


@pytest.mark.parametrize("functional", ["far", "surface"])
def test_vertex_gradient_matches_directional_differences(ring_case, functional):
    """dC/dv . W for two seeded normal-displacement fields W against central
    differences of C at V +- h W (h = 1e-4), each a full GPU solve to 1e-12."""
    V, F, out = ring_case
    C, gV, gN = out[functional]
    for seed in (1, 2):
        W = _direction(V, F, seed)
        an = np.sum(gV * W)
        fd = (_product_C(V + 1e-4 * W, F, 1.5, 2.25 + 0.5j, functional)
              - _product_C(V - 1e-4 * W, F, 1.5, 2.25 + 0.5j, functional)) / 2e-4
        scale = np.sum(np.abs(gV * W))
        print("%s C %.8f dir %d adjoint %.10e differences %.10e (scale %.3e)" % (functional, C, seed, an, fd, scale),
              flush=True)
        assert abs(an - fd) <= 2e-6 * scale
        # W = r N_v, so the same number from the normal-displacement gradient
        r = np.random.default_rng(seed).standard_normal(len(V))
        assert abs(np.sum(r * gN) - an) <= 1e-12 * scale


def test_vertex_gradient_translation_invariance(ring_case):
    """C_sca under a plane wave is unchanged when the scatterer is translated,
    so the vertex gradient sums to zero (its parts do not: each cancels the others)."""
    V, F, out = ring_case
    for fun in ("far", "surface"):
        gV = out[fun][1]
        tot = np.linalg.norm(gV.sum(axis=0))
        print(fun, "sum of gradients", tot, "vs", np.abs(gV).sum(), flush=True)
        assert tot <= 1e-7 * np.abs(gV).sum()


def test_vertex_gradient_scaling_identity(ring_case):
    """Scaling the mesh by s multiplies C by s^2 at wavenumber s k0 (the method is
    scale-covariant: weights ~ s^2, self blocks and orders follow), so
    sum_v v . dC/dv = 2 C + k0 dC/dk0; dC/dk0 by central differences of solves."""
    V, F, out = ring_case
    C, gV, _ = out["far"]
    h = 1e-5
    dk = (_product_C(V, F, 1.5 + h, 2.25 + 0.5j, "far") - _product_C(V, F, 1.5 - h, 2.25 + 0.5j, "far")) / (2 * h)
    lhs = np.sum(V * gV)
    rhs = 2 * C + 1.5 * dk
    print("scaling: sum v.dC/dv %.10e, 2C + k0 dC/dk0 %.10e" % (lhs, rhs), flush=True)
    assert abs(lhs - rhs) <= 1e-6 * np.abs(V * gV).sum()


@pytest.mark.parametrize("functional", ["far", "surface"])
def test_vertex_gradient_matches_oracle_differences(abi, functional):
    """On a 120-triangle torus the product's gradient along a seeded normal
    field against central differences of the oracle's C (its own point sums,
    self blocks, preconditioned fGMRES to 1e-13 and functional), h = 1e-4."""
    from paper_1211_7177_amd.shape import cross_section_and_vertex_gradient
    m = torus(1.0, 0.35, 10, 6)
    V, F = m.vertices.copy(), m.triangles.copy()
    k0, eps = 1.2, 3.0 + 0.2j
    print("oracle differences", functional, flush=True)
    C, gV, _ = cross_section_and_vertex_gradient(V, F, k0, eps, D, POL, functional=functional, **PLAN)
    W = _direction(V, F, 5)

    def oracle_C(Vx):
        from synthetic.meshes import Mesh
        q = nystrom3(Mesh(Vx, F.astype(np.int32)))
        ob = OracleBem(q, k0, eps)
        x, _ = oracle_gmres(ob.apply, ob.rhs_planewave(D, POL), ob.block_preconditioner(), tol=1e-13, restart=300)
        if functional == "far":
            return cross_section_far(q, k0, x, POL)
        return cross_section_surface(q, k0, x, D, POL)

    c0 = oracle_C(V)
    fd = (oracle_C(V + 1e-4 * W) - oracle_C(V - 1e-4 * W)) / 2e-4
    an = np.sum(gV * W)
    print("%s C product %.10f oracle %.10f; along W adjoint %.10e oracle differences %.10e" % (
        functional, C, c0, an, fd), flush=True)
    assert abs(C - c0) <= 1e-8 * abs(c0)
    assert abs(an - fd) <= 2e-6 * np.sum(np.abs(gV * W))


def test_sphere_radius_derivative_matches_mie(abi):
    """Moving every vertex of a geodesic sphere (radius 1, 1280 triangles) along
    its radius changes the radius: sum_v (v/|v|) . dC/dv against the derivative
    of Mie's C_sca = pi a^2 Q_sca(k0 a) (k0 = 1, eps = 2.25), to the mesh's error."""
    from paper_1211_7177_amd.shape import cross_section_and_vertex_gradient
    m = icosphere(8)
    V, F = m.vertices.copy(), m.triangles.copy()
    C, gV, _ = cross_section_and_vertex_gradient(V, F, 1.0, 2.25, D, POL, functional="far", order=0, plan_tol=1e-8,
                                                 tol=1e-10)
    dCda = np.sum(gV * V / np.linalg.norm(V, axis=1, keepdims=True))
    m_ = np.sqrt(2.25)

    def mieC(a):
        return mie.efficiencies(a, m_)[1] * np.pi * a * a

    ref = (mieC(1 + 1e-5) - mieC(1 - 1e-5)) / 2e-5
    print("sphere: C %.6f (Mie %.6f); dC/da adjoint %.6f Mie %.6f" % (C, mieC(1.0), dCda, ref), flush=True)
    assert abs(dCda - ref) <= 2e-2 * abs(ref)


def test_vertex_gradient_two_scatterers(abi):
    """Two scatterers (a sphere of radius 0.5, eps = 2.25 + 0.3i, and a torus,
    eps = 4 + 0.1i, 1.6 apart; Fig. 1's setting): the host rows over both, each
    interior over its own nodes.  dC/dv along a seeded normal field against
    central differences (h = 1e-4) of GPU solves to 1e-12, both functionals;
    translating both together leaves C unchanged."""
    from paper_1211_7177_amd.gradients import _functional
    from paper_1211_7177_amd.shape import cross_section_and_vertex_gradient, nodes_of_mesh
    from paper_1211_7177_amd.solver import MultiBemProblem
    from synthetic import union
    m, reg = union([icosphere(2, 0.5), torus(0.5, 0.2, 8, 5)], [[0, 0, 0], [1.6, 0.2, 0.1]])
    V, F = m.vertices.copy(), m.triangles.copy()
    eps, k0 = [2.25 + 0.3j, 4.0 + 0.1j], 1.3
    region = np.repeat(reg, 3)

    def C_of(Vx, fun):
        q = nodes_of_mesh(Vx, F)
        pb = MultiBemProblem(q, region, k0, eps, order=20, depth=2)
        x, _ = pb.solve(pb.rhs_planewave(D, POL), tol=1e-12, restart=200, maxit=4000)
        c = _functional(fun, pb, q, k0, x, D, POL).item()
        pb.close()
        return c

    W = _direction(V, F, 9)
    for fun in ("far", "surface"):
        print("two scatterers", fun, flush=True)
        C, gV, _ = cross_section_and_vertex_gradient(V, F, k0, eps, D, POL, functional=fun, tri_region=reg, **PLAN)
        an = np.sum(gV * W)
        fd = (C_of(V + 1e-4 * W, fun) - C_of(V - 1e-4 * W, fun)) / 2e-4
        scale = np.sum(np.abs(gV * W))
        print("%s C %.8f: adjoint %.10e differences %.10e (scale %.3e); |sum dC/dv| %.2e" % (
            fun, C, an, fd, scale, np.linalg.norm(gV.sum(axis=0))), flush=True)
        assert abs(an - fd) <= 2e-6 * scale
        assert np.linalg.norm(gV.sum(axis=0)) <= 1e-7 * np.abs(gV).sum()


def test_impedance_vertex_gradient(abi):
    """A good conductor under the impedance condition (eq. 2.25; Z = 0.1 - 0.2i,
    k0 = 1.2, far-field C_sca) on a 120-triangle torus: dC/dv along a seeded
    normal field against central differences (h = 1e-4) of GPU solves and of the
    oracle's own solves; it sums to zero under translation."""
    from oracle.bem import IbcProblem as OracleIbc
    from paper_1211_7177_amd.gradients import far_field_cross_section
    from paper_1211_7177_amd.shape import impedance_cross_section_and_vertex_gradient, nodes_of_mesh
    from paper_1211_7177_amd.solver import IbcProblem
    from synthetic.meshes import Mesh
    m = torus(1.0, 0.35, 10, 6)
    V, F = m.vertices.copy(), m.triangles.copy()
    k0, Z = 1.2, 0.1 - 0.2j
    print("impedance vertex gradient", flush=True)
    C, gV, _ = impedance_cross_section_and_vertex_gradient(V, F, k0, Z, D, POL, order=20, depth=2, tol=1e-12,
                                                           restart=200)
    W = _direction(V, F, 4)

    def gpu_C(Vx):
        pb = IbcProblem(nodes_of_mesh(Vx, F), k0, Z, order=20, depth=2)
        x, _ = pb.solve(pb.rhs_planewave(D, POL), tol=1e-12, restart=200, maxit=4000)
        c = far_field_cross_section(pb, x, POL).item()
        pb.close()
        return c

    def oracle_C(Vx):
        q = nystrom3(Mesh(Vx, F.astype(np.int32)))
        ob = OracleIbc(q, k0, Z)
        x, _ = oracle_gmres(ob.apply, ob.rhs_planewave(D, POL), ob.block_preconditioner(), tol=1e-13, restart=300)
        return cross_section_far(q, k0, np.concatenate([x, -ob.c * ob.nnx(x)], axis=1), POL)

    an = np.sum(gV * W)
    fd_gpu = (gpu_C(V + 1e-4 * W) - gpu_C(V - 1e-4 * W)) / 2e-4
    fd_or = (oracle_C(V + 1e-4 * W) - oracle_C(V - 1e-4 * W)) / 2e-4
    scale = np.sum(np.abs(gV * W))
    print("ibc C %.8f (oracle %.8f): adjoint %.10e, GPU differences %.10e, oracle differences %.10e" % (
        C, oracle_C(V), an, fd_gpu, fd_or), flush=True)
    assert abs(an - fd_gpu) <= 2e-6 * scale and abs(an - fd_or) <= 2e-6 * scale
    assert np.linalg.norm(gV.sum(axis=0)) <= 1e-7 * np.abs(gV).sum()
