"""GPU parity of the several-scatterer system against the oracle (needs an MI355X)."""

import numpy as np
import pytest

from oracle.bem import MultiBemProblem as OracleMulti
from oracle.gmres import gmres_solve as oracle_gmres
from synthetic import complex_normal, icosphere, nystrom3, torus, union

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import solver
    return solver


@pytest.fixture(scope="module")
def three():
    """A sphere, a smaller sphere and a torus side by side (uneven node counts),
    with a lossless, a lossy dielectric and a metal-like permittivity."""
    m, treg = union([icosphere(4), icosphere(3, 0.6), torus(0.8, 0.25, 24, 8)],
                    [[0.0, 0.0, 0.0], [2.2, 0.0, 0.0], [0.0, 2.4, 0.3]])
    q = nystrom3(m)
    reg = treg[q["point_tri"]]
    eps = [2.25, 4.0 + 0.5j, -6.0 + 1.0j]
    return q, reg, eps, OracleMulti(q, reg, 1.0, eps)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_multi_apply_and_adjoint_match_oracle(gpu, three):
    q, reg, eps, ob = three
    n = q["points"].shape[0]
    print("multi apply: %d nodes, regions %s" % (n, np.bincount(reg)), flush=True)
    pb = gpu.MultiBemProblem(q, reg, 1.0, eps, order=20, depth=4)
    x = complex_normal((n, 6), 161)
    xg = torch.from_numpy(x).cuda()
    assert _rel(pb.apply(xg).cpu().numpy(), ob.apply(x)) <= 1e-7
    assert _rel(pb.apply_adjoint(xg).cpu().numpy(), ob.apply_adjoint(x)) <= 1e-7
    assert _rel(pb.precond(xg).cpu().numpy(), ob.block_preconditioner()(x)) <= 1e-11
    pb.close()


def test_multi_solves_match_oracle(gpu, three):
    q, reg, eps, ob = three
    print("multi solves", flush=True)
    b = ob.rhs_planewave([0.0, 0.6, 0.8], [1.0, 0.0, 0.0])
    xo, io = oracle_gmres(ob.apply, b, ob.block_preconditioner(), tol=1e-10, restart=200)
    pb = gpu.MultiBemProblem(q, reg, 1.0, eps, order=22, depth=4, order32=10)
    bg = torch.from_numpy(b).cuda().unsqueeze(0)
    x, info = pb.solve(bg, tol=1e-10, restart=200, maxit=800)
    print("its gpu", info["iterations"], "oracle", io["iterations"], "err", _rel(x.cpu().numpy()[0], xo))
    assert info["residual"] <= 1e-10 and _rel(x.cpu().numpy()[0], xo) <= 1e-6
    xm, im = pb.solve(bg, tol=1e-8, mixed=True, inner_tol=1e-3)
    assert im["residual"] <= 1e-8 and _rel(xm.cpu().numpy()[0], xo) <= 1e-6
    xs, _ = pb.solve(bg, tol=1e-8, mixed=True, inner_tol=1e-3, serial=True)
    assert torch.equal(xs, xm)                          # the products' order on the streams does not change a bit
    pb.close()


def test_one_region_multi_equals_single(gpu):
    q = nystrom3(icosphere(4))
    n = q["points"].shape[0]
    pm = gpu.MultiBemProblem(q, np.zeros(n, np.int32), 1.0, [2.25], order=14, depth=3, depths=[3])
    ps = gpu.BemProblem(q, 1.0, 2.25, order=14, depth=3)
    x = torch.from_numpy(complex_normal((n, 6), 162)).cuda()
    assert torch.equal(pm.apply(x), ps.apply(x))
    pm.close()
    ps.close()


def test_gold_dimer_force_on_one_sphere(gpu):
    """Two gold spheres (radius 100 nm, surface gap 250 nm, along x; 960 nodes
    each; length unit 100 nm) at 500 nm, eps from the Drude model of Sec. 3.2,
    under a wave along +z polarised along x, with the force on each sphere from
    a stress-tensor sphere around it alone (the workload of the force comparison
    in the paper's appendix D).  The GPU solve and forces against the oracle's;
    mirror symmetry of the two forces; and the sum of the two forces against the
    force from one sphere around both (0.26% apart in the oracle too: the discrete
    field is not exactly divergence-free, so the stress tensor is not exactly
    conserved between the surfaces)."""
    from oracle import fields as of
    from oracle import materials as om
    from paper_1211_7177_amd import materials, postprocess as pp
    eps = complex(materials.gold_drude(500e-9))
    k0 = float(materials.wavenumber(500e-9, 100e-9))
    m, treg = union([icosphere(4), icosphere(4)], [[-2.25, 0.0, 0.0], [2.25, 0.0, 0.0]])
    q = nystrom3(m)
    reg = treg[q["point_tri"]]
    ob = OracleMulti(q, reg, k0, [complex(om.eps_gold(om.omega(500e-9)))] * 2)
    b = ob.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])
    xo, io = oracle_gmres(ob.apply, b, ob.block_preconditioner(), tol=1e-10, restart=200)
    pb = gpu.MultiBemProblem(q, reg, k0, [eps, eps], order=20)
    x, info = pb.solve(pb.rhs_planewave([0, 0, 1.0], [1.0, 0, 0]), tol=1e-10, restart=200)
    print("dimer its gpu", info["iterations"], "oracle", io["iterations"], flush=True)
    assert _rel(x.cpu().numpy()[0], xo) <= 1e-6
    kw = dict(nt=24, nph=48)
    Fl = pp.optical_force(pb, x, [0, 0, 1.0], [1.0, 0, 0], k0, 1.6, center=[-2.25, 0, 0], **kw)[0]
    Fr = pp.optical_force(pb, x, [0, 0, 1.0], [1.0, 0, 0], k0, 1.6, center=[2.25, 0, 0], **kw)[0]
    Fb = pp.optical_force(pb, x, [0, 0, 1.0], [1.0, 0, 0], k0, 3.8, **kw)[0]
    dirs, wts = pp.sphere_quadrature(24, 48)
    pts = np.array([-2.25, 0, 0])[None] + 1.6 * dirs
    Ei = np.exp(1j * k0 * pts[:, 2])[:, None] * np.array([1.0, 0, 0])[None, :]
    Ci = 1j * k0 * np.cross(np.broadcast_to([0, 0, 1.0], Ei.shape), Ei)
    Fo = of.stress_force(Ei + of.scattered_field(q, k0, xo, pts), Ci + of.scattered_curl(q, k0, xo, pts),
                         k0, dirs, 1.6 ** 2 * wts)
    print("F_left", Fl, "oracle", Fo, "F_right", Fr, "F_both", Fb, flush=True)
    assert np.linalg.norm(Fl - Fo) <= 1e-6 * np.linalg.norm(Fo)
    scale = np.linalg.norm(Fl)
    assert abs(Fl[0] + Fr[0]) <= 1e-6 * scale and abs(Fl[2] - Fr[2]) <= 1e-6 * scale
    assert abs(Fl[1]) <= 1e-8 * scale and abs(Fr[1]) <= 1e-8 * scale
    assert np.linalg.norm(Fl + Fr - Fb) <= 0.01 * np.linalg.norm(Fb)
    pb.close()


def test_per_scatterer_eps_gradients_match_differences(gpu):
    """Two lossy spheres side by side (960 nodes each, eps 2.25 + 0.5i and
    4 + 0.3i): dC_sca/deps_j of the far-field cross section for each scatterer
    from one forward and one adjoint solve, against h = 1e-6 central differences
    of solves to 1e-12 in both directions of each complex eps_j."""
    from paper_1211_7177_amd import gradients as gr
    m, treg = union([icosphere(4), icosphere(4)], [[-1.6, 0.0, 0.0], [1.6, 0.0, 0.0]])
    q = nystrom3(m)
    reg = treg[q["point_tri"]]
    eps = [2.25 + 0.5j, 4.0 + 0.3j]
    d, p = [0.0, 0.6, 0.8], [1.0, 0.0, 0.0]
    C, g = gr.cross_section_and_eps_gradients_multi(q, reg, 1.0, eps, d, p, order=20, depths=[3, 3], tol=1e-12,
                                                    restart=200)
    h = 1e-6
    for j in range(2):
        fd = []
        for de in (h, -h, 1j * h, -1j * h):
            e2 = list(eps)
            e2[j] = e2[j] + de
            pb = gpu.MultiBemProblem(q, reg, 1.0, e2, order=20, depths=[3, 3])
            x, _ = pb.solve(pb.rhs_planewave(d, p), tol=1e-12, restart=200, maxit=4000)
            fd.append(gr.far_field_cross_section(pb, x, p).item())
            pb.close()
        fr, fi = (fd[0] - fd[1]) / (2 * h), (fd[2] - fd[3]) / (2 * h)
        print("scatterer %d: adjoint (%.8e, %.8e) differences (%.8e, %.8e)" % (j, g[j][0], g[j][1], fr, fi),
              flush=True)
        scale = max(abs(fr), abs(fi))
        assert abs(g[j][0] - fr) <= 1e-5 * scale and abs(g[j][1] - fi) <= 1e-5 * scale
    print("C", C)


def test_separation_gradient_of_two_spheres(gpu):
    """The derivative of the far-field C_sca of two lossy spheres with respect to
    moving the second one along x (their separation), by the adjoint method
    over a shape family of the coupled system, against central differences of
    its solves."""
    from paper_1211_7177_amd import gradients as gr
    from synthetic import Mesh
    m, treg = union([icosphere(4), icosphere(4)], [[-1.6, 0.0, 0.0], [1.6, 0.0, 0.0]])
    q0 = nystrom3(m)
    reg = treg[q0["point_tri"]]
    vreg = np.zeros(len(m.vertices), dtype=int)
    vreg[m.triangles[treg == 1].ravel()] = 1
    shift = np.zeros_like(m.vertices)
    shift[vreg == 1, 0] = 1.0
    eps = [2.25 + 0.5j, 4.0 + 0.3j]
    d, p = [0.0, 0.6, 0.8], [1.0, 0.0, 0.0]

    def nodes_at(th):
        return nystrom3(Mesh(m.vertices + th[0] * shift, m.triangles))

    def make(q, dep):
        return gpu.MultiBemProblem(q, reg, 1.0, eps, order=20, depth=dep, depths=[3, 3])

    C, gs = gr.cross_section_and_shape_gradient(nodes_at, 1, 1.0, eps, d, p, depth=4, tol=1e-12, restart=200,
                                                h=1e-4, functional="far", make_problem=make)
    h = 1e-4
    v = []
    for sgn in (1.0, -1.0):
        pb = make(nodes_at(np.array([sgn * h])), 4)
        x, _ = pb.solve(pb.rhs_planewave(d, p), tol=1e-12, restart=200, maxit=4000)
        v.append(gr.far_field_cross_section(pb, x, p).item())
        pb.close()
    fd = (v[0] - v[1]) / (2 * h)
    print("C %.6f dC/dseparation adjoint %.8e differences %.8e" % (C, gs[0], fd), flush=True)
    assert abs(gs[0] - fd) <= 1e-5 * abs(fd)
