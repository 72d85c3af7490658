"""Gradient of the scattering cross section with respect to every mesh vertex,
by the adjoint method: one forward solve, one adjoint solve and one
derivative pass give dC/dv at all vertices, and from it dC/d(delta_v) for
displacements delta_v of each vertex along its normal.

Geometry.  The Nystrom nodes follow from the triangle corners: three nodes
per triangle at barycentric coordinates (2/3, 1/6, 1/6) and its permutations,
the triangle's unit normal (B - A) x (C - A) / |...| (eq. B.1) and weight
area / 3 (the rule of eq. 2.8).  A vertex normal is the area-weighted mean of
its triangles' normals.

Derivative.  With the system A x = b of eqs. 2.12-2.13 and a functional
C = f(x, geometry) (C_sca of eq. 4.2, on the surface or from the far field),
lambda = A^{-H} grad_x f gives

    dC/dv = df/dv |_x + Re d/dv [ sum conj(lambda) . (b - A x) ] |_{x, lambda}.

The rows of A x are (1/2 Phi + Op_k0(Phi, -Psi), 1/2 T Phi - Op_k1(T Phi, -gamma Psi))
with T = I + (1 - eps)/eps n n^T (eq. 2.13); with several scatterers (Fig. 1) the
host rows run over every node and scatterer j's interior rows over its own
nodes with its own k_j, T_j and gamma_j.  The geometry enters through
* the incident field E_inc(s) in b and T(n) in the interior jump term:
  torch autograd on the node positions and normals;
* T(n) Phi as the interior operator's density: its derivative is
  conj(abar_1) . d(T Phi) with abar_1 = (Op_k1^H lambda_1)_a (`fmm_matvec_adjoint`);
* the point sum of each operator (pairs of distinct triangles): the node
  position, normal and weight derivatives of its bilinear form
  (`bem_shape_pairs`, direct FP64 sums);
* the self-triangle blocks (Appendix B), which depend only on their own
  triangle's corners: central differences of `bem_self_blocks`, moving corner
  j of every triangle along axis c at once (9 slots x 2 signs x 2 wavenumbers
  block builds), each triangle's own rows summing to its own derivative;
* the functional's explicit dependence on the nodes: torch autograd (the far
  field in direction chunks).
The node derivatives are then carried to the vertices by autograd through the
node rule above.
"""

import numpy as np
import torch

from ._abi import self_blocks, shape_pairs
from .gradients import _functional
from .solver import BemProblem

_BARY = ((2.0 / 3, 1.0 / 6, 1.0 / 6), (1.0 / 6, 2.0 / 3, 1.0 / 6), (1.0 / 6, 1.0 / 6, 2.0 / 3))


def nodes_of_triangles(tv):
    """(points [3nt, 3], normals [3nt, 3], weights [3nt]) of triangles with corners
    tv [nt, 3, 3] (torch or numpy, float64; node 3t + i belongs to triangle t)."""
    if isinstance(tv, np.ndarray):
        cr = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
        a2 = np.linalg.norm(cr, axis=1)
        pts = np.einsum("qk,tkd->tqd", np.asarray(_BARY), tv).reshape(-1, 3)
        return pts, np.repeat(cr / a2[:, None], 3, axis=0), np.repeat(a2 / 6.0, 3)
    cr = torch.linalg.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    a2 = torch.linalg.norm(cr, dim=1)
    bary = torch.tensor(_BARY, dtype=tv.dtype, device=tv.device)
    pts = torch.einsum("qk,tkd->tqd", bary, tv).reshape(-1, 3)
    return pts, (cr / a2[:, None]).repeat_interleave(3, dim=0), (a2 / 6.0).repeat_interleave(3)


def nodes_of_mesh(vertices, triangles):
    """The Nystrom node set (numpy dict: points, normals, weights, point_tri,
    tri_vertices) of a triangle mesh."""
    V = np.asarray(vertices, dtype=np.float64)
    F = np.asarray(triangles, dtype=np.int64)
    tv = np.ascontiguousarray(V[F])
    pts, nrm, w = nodes_of_triangles(tv)
    return {"points": np.ascontiguousarray(pts), "normals": np.ascontiguousarray(nrm),
            "weights": np.ascontiguousarray(w), "point_tri": np.repeat(np.arange(len(F), dtype=np.int32), 3),
            "tri_vertices": tv}


def vertex_normals(vertices, triangles):
    """Unit vertex normals f64[nv, 3]: the area-weighted mean of the adjacent
    triangles' normals."""
    V = np.asarray(vertices, dtype=np.float64)
    F = np.asarray(triangles, dtype=np.int64)
    cr = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    N = np.zeros_like(V)
    for j in range(3):
        np.add.at(N, F[:, j], cr)
    return N / np.linalg.norm(N, axis=1, keepdims=True)


def apply_self_blocks(nrm, point_tri, dv, dg, a, b):
    """Rows of the self-triangle terms: y_alpha = sum_j K_beta(dV_alpha j) . a_beta + dG_alpha j b_beta,
    beta the j-th node (ascending) of alpha's triangle,
    K_beta(V) . a = n_beta (V . a) - (n_beta . V) a - V (n_beta . a).  Torch [n, 3]."""
    n, m = dg.shape
    tri = point_tri.long()
    order = torch.argsort(tri, stable=True).reshape(-1, m)          # nodes of each triangle, ascending
    nc = nrm.to(torch.complex128)
    y = torch.zeros_like(a)
    for j in range(m):
        beta = order[tri, j]
        V = dv[:, j]
        nb, ab, bb = nc[beta], a[beta], b[beta]
        y = y + (nb * torch.sum(V * ab, dim=1, keepdim=True) - torch.sum(nb * V, dim=1, keepdim=True) * ab
                 - V * torch.sum(nb * ab, dim=1, keepdim=True) + dg[:, j:j + 1] * bb)
    return y


def _per_triangle(vals, point_tri_l, ntri):
    out = torch.zeros(ntri, dtype=vals.dtype, device=vals.device)
    return out.index_add_(0, point_tri_l, vals)


def self_triangle_vertex_derivative(vertices, triangles, terms, fd_rel=1e-5):
    """d/dv Re[ sum_i c_i sum_alpha conj(lam_i,alpha) . S_{k_i}(a_i, b_i)_alpha ] for
    terms = [(k_i, c_i, lam_i, a_i, b_i), ...] (torch [n, 3], on the device the blocks are built for), S_k the
    self-triangle terms of `bem_self_blocks` (LINEAR blocks), with the densities
    held fixed: central differences in each triangle corner coordinate, step
    fd_rel times the triangle's longest edge.  Returns f64[nv, 3]."""
    V = np.asarray(vertices, dtype=np.float64)
    F = np.asarray(triangles, dtype=np.int64)
    nt = len(F)
    tv0 = V[F]
    edges = np.stack([tv0[:, 1] - tv0[:, 0], tv0[:, 2] - tv0[:, 1], tv0[:, 0] - tv0[:, 2]], axis=1)
    h = fd_rel * np.max(np.linalg.norm(edges, axis=2), axis=1)          # [nt]
    point_tri = np.repeat(np.arange(nt, dtype=np.int32), 3)
    dev = terms[0][2].device
    pt_dev = torch.from_numpy(point_tri).to(dev)
    pt_l = pt_dev.long()
    h_dev = torch.from_numpy(h).to(dev)
    out = np.zeros_like(V)
    for j in range(3):
        for c in range(3):
            vals = []
            for sg in (1.0, -1.0):
                tv = tv0.copy()
                tv[:, j, c] += sg * h
                pts, nrm, _ = nodes_of_triangles(tv)
                nrm_dev = torch.from_numpy(np.ascontiguousarray(nrm)).to(dev)
                acc = torch.zeros(nt, dtype=torch.complex128, device=dev)
                for k, coef, lam, a, b in terms:
                    dv, dg = self_blocks(pts, nrm, point_tri, tv, k, device=dev)
                    y = apply_self_blocks(nrm_dev, pt_dev, dv, dg, a, b)
                    acc = acc + coef * _per_triangle(torch.sum(torch.conj(lam) * y, dim=1), pt_l, nt)
                vals.append(acc)
            d = ((vals[0] - vals[1]) / (2.0 * h_dev)).real.cpu().numpy()
            np.add.at(out[:, c], F[:, j], d)
    return out


def _far_explicit(k0, a, b_of_n, pol, s, n, w, nt=24, nph=48, chunk_bytes=5e8):
    """d/d(s, n, w) of C = sum W |F|^2 / |E0|^2 with F the far-field amplitude of
    the densities held fixed (the same sum `bem_field` evaluates:
    F(r) = -(1/4pi) sum w e^{-ik0 r.s} [ -ik0 (n (r.a) - (n.r) a - r (n.a)) + b ], a = Phi,
    b = b_of_n(n): -Psi for dielectrics, c n x (n x Phi) under the impedance condition),
    with the Gauss-Legendre x uniform rule of `far_field_cross_section`.  Directions
    are taken in chunks whose [chunk, n, 3] complex intermediates stay near
    chunk_bytes."""
    from .postprocess import sphere_quadrature
    dirs, wts = sphere_quadrature(nt, nph)
    chunk = int(max(1, min(64, chunk_bytes // (48 * s.shape[0]))))
    e0 = float(np.sum(np.abs(np.asarray(pol)) ** 2))
    sl, nl, wl = (t.detach().clone().requires_grad_(True) for t in (s, n, w))
    gs, gn, gw = torch.zeros_like(s), torch.zeros_like(n), torch.zeros_like(w)
    k0 = complex(k0)
    for lo in range(0, len(dirs), chunk):
        r = torch.from_numpy(dirs[lo:lo + chunk]).to(s.device)
        W = torch.from_numpy(wts[lo:lo + chunk]).to(s.device)
        b = b_of_n(nl)
        # sums over the nodes as elementwise products and reductions (a product with K = n and
        # N = 3 runs far below the library GEMM's speed)
        ph = wl[None, :] * torch.exp(-1j * k0 * (r @ sl.T))                # [nd, n]
        nc = nl.to(torch.complex128)
        rc = r.to(torch.complex128)
        ra = torch.sum(rc[:, None, :] * a[None], dim=2)                      # [nd, n]  r . a
        nr = torch.sum(r[:, None, :] * nl[None], dim=2).to(torch.complex128)  # [nd, n]  n . r
        na = torch.sum(nc * a, dim=1)                                        # [n]
        s1 = torch.sum((ph * ra)[:, :, None] * nc[None], dim=1)              # [nd, 3]
        s2 = torch.sum((ph * nr)[:, :, None] * a[None], dim=1)
        s3 = torch.sum(ph * na[None], dim=1)
        s4 = torch.sum(ph[:, :, None] * b[None], dim=1)
        term = (-1j * k0) * (s1 - s2 - rc * s3[:, None]) + s4
        Fk = -(1.0 / (4.0 * np.pi)) * term
        Ck = torch.sum(W[:, None] * (Fk.real ** 2 + Fk.imag ** 2)) / e0
        g = torch.autograd.grad(Ck, (sl, nl, wl))
        gs += g[0]
        gn += g[1]
        gw += g[2]
    return gs, gn, gw


def _surface_explicit(k0, x, d, pol, s, n, w):
    """d/d(s, n, w) of the surface form of C_sca (eq. 4.2) with x [n, 6] fixed."""
    sl, nl, wl = (t.detach().clone().requires_grad_(True) for t in (s, n, w))
    k0 = complex(k0)
    dd = torch.tensor(np.asarray(d, dtype=np.float64), device=s.device)
    p = torch.tensor(np.asarray(pol, dtype=np.complex128), device=s.device)
    e = torch.exp(1j * k0 * (sl @ dd))
    E = e[:, None] * p[None, :]
    curl = (1j * k0) * torch.linalg.cross(dd.to(torch.complex128).expand_as(E), E)
    Pi = torch.linalg.cross(nl.to(torch.complex128), curl)
    e0 = float(np.sum(np.abs(np.asarray(pol)) ** 2))
    esca = x[:, 0:3] - E
    nh = (x[:, 3:6] - Pi) / (1j * k0)
    C = -torch.sum(wl * torch.real(torch.sum(esca * torch.conj(nh), dim=1))) / e0
    return torch.autograd.grad(C, (sl, nl, wl))


def cross_section_and_vertex_gradient(vertices, triangles, k0, eps, d, pol, order=16, depth=0, tol=1e-10,
                                      restart=150, mu=1.0, functional="far", order32=None, solve_kw=None,
                                      fd_rel=1e-5, plan_tol=0.0, stats=None, tri_region=None):
    """(C_sca, dC/dv f64[nv, 3], dC/d(delta_v) f64[nv]) under the plane wave
    pol exp(i k0 d . s), delta_v being the displacement of vertex v along its
    vertex normal.  One scatterer of permittivity eps (and permeability mu), or,
    with tri_region (the scatterer of every triangle, 0..J-1), J scatterers with
    eps[j] and mu[j] (scalars apply to all): the host rows use every node at k0,
    scatterer j's interior rows its own nodes at k_j (Fig. 1).  functional: "far"
    (oint |F|^2 dOmega) or "surface" (eq. 4.2 on the scatterers' surfaces).
    order / plan_tol / order32 / solve_kw as for `BemProblem` and its solve
    (plan_tol applies to one scatterer only).  stats: a dict to receive the
    seconds of each phase (device-synchronised) and the solves' iteration counts."""
    import time

    from .solver import MultiBemProblem

    def mark(key, t0):
        if stats is not None:
            torch.cuda.synchronize()
            stats[key] = time.perf_counter() - t0
        return time.perf_counter()

    t0 = time.perf_counter()
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    F = np.ascontiguousarray(triangles, dtype=np.int64)
    q = nodes_of_mesh(V, F)
    if tri_region is None:
        J, region = 1, np.zeros(len(q["points"]), dtype=np.int32)
        eps_l, mu_l = [complex(eps)], [complex(mu)]
        pb = BemProblem(q, k0, eps_l[0], mu=mu_l[0], order=order, depth=depth, order32=order32, tol=plan_tol)
    else:
        region = np.repeat(np.asarray(tri_region, dtype=np.int32), 3)
        J = int(region.max()) + 1
        eps_l = [complex(e) for e in np.broadcast_to(np.asarray(eps, dtype=np.complex128), (J,))]
        mu_l = [complex(m) for m in np.broadcast_to(np.asarray(mu, dtype=np.complex128), (J,))]
        pb = MultiBemProblem(q, region, k0, eps_l, mu=mu_l, order=order, depth=depth, order32=order32)
    plans = pb.pj if J > 1 else [pb.p1]
    kj = list(pb.kj) if J > 1 else [pb.k1]
    idx = [np.nonzero(region == j)[0] for j in range(J)]
    kw = dict(tol=tol, restart=restart, maxit=4000)
    kw.update(solve_kw or {})
    try:
        t0 = mark("setup_s", t0)
        xd, inf = pb.solve(pb.rhs_planewave(d, pol), **kw)
        t0 = mark("solve_s", t0)
        xg = xd.clone().requires_grad_(True)
        C = _functional(functional, pb, q, k0, xg, d, pol)
        g = torch.autograd.grad(C, xg)[0]
        t0 = mark("functional_s", t0)
        lam, inf_adj = pb.solve(g.contiguous(), adjoint=True, **kw)
        t0 = mark("adjoint_solve_s", t0)
        if stats is not None:
            stats["iterations"] = inf["iterations"]
            stats["adjoint_iterations"] = inf_adj["iterations"]
        x, lam = xd[0], lam[0]
        dev = x.device
        idx_t = [torch.from_numpy(i).to(dev) for i in idx]
        phi, psi = x[:, 0:3].contiguous(), x[:, 3:6].contiguous()
        lam0, lam1 = lam[:, 0:3].contiguous(), lam[:, 3:6].contiguous()
        # abar_1 = (Op_kj^H lambda_1)_a of each scatterer's plan, over its own nodes
        abar1 = torch.zeros_like(lam1)
        for j in range(J):
            abar1[idx_t[j]] = plans[j].matvec_adjoint(lam1[idx_t[j]].contiguous())[0]
    finally:
        pb.close()
    t0 = mark("adjoint_product_s", t0)
    # per-node T coefficient (1 - eps)/eps and gamma = mu of the node's scatterer
    reg_t = torch.from_numpy(region.astype(np.int64)).to(dev)
    tcoef = torch.tensor([(1.0 - e) / e for e in eps_l], dtype=torch.complex128, device=dev)[reg_t][:, None]
    gam = torch.tensor(mu_l, dtype=torch.complex128, device=dev)[reg_t][:, None]

    def tmul(nrm):
        nc = nrm.to(torch.complex128)
        return phi + tcoef * nc * torch.sum(nc * phi, dim=1, keepdim=True)

    Vt = torch.from_numpy(V).to(dev).requires_grad_(True)
    Ft = torch.from_numpy(F).to(dev)
    s, n, w = nodes_of_triangles(Vt[Ft])
    s0, n0, w0 = s.detach().contiguous(), n.detach().contiguous(), w.detach().contiguous()
    tri = torch.from_numpy(q["point_tri"]).to(dev)
    tphi = tmul(n0).contiguous()
    b0, b1 = (-psi).contiguous(), (-gam * psi).contiguous()
    # point sums: sum conj(lam) . A x holds +B_k0(lam0; Phi, -Psi) over all nodes and
    # -B_kj(lam1; T Phi, -gamma Psi) over each scatterer's own nodes
    ds, dn, dw = shape_pairs(s0, n0, w0, tri, k0, lam0, phi, b0)
    for j in range(J):
        i = idx_t[j]
        dsj, dnj, dwj = shape_pairs(s0[i].contiguous(), n0[i].contiguous(), w0[i].contiguous(), tri[i].contiguous(),
                                    kj[j], lam1[i].contiguous(), tphi[i].contiguous(), b1[i].contiguous())
        ds[i] -= dsj
        dn[i] -= dnj
        dw[i] -= dwj
    t0 = mark("pairs_s", t0)
    GS, GN, GW = -ds.real, -dn.real, -dw.real
    # explicit dependence of the functional
    if functional == "far":
        es, en, ew = _far_explicit(k0, phi, lambda nl: b0, pol, s0, n0, w0)
    else:
        es, en, ew = _surface_explicit(k0, x, d, pol, s0, n0, w0)
    GS, GN, GW = GS + es, GN + en, GW + ew
    # b(s) and the normal's local and density roles: Re sum conj(lam0) . E_inc(s)
    # - Re sum [ conj(lam1) . 1/2 T(n) Phi - conj(abar1) . T(n) Phi ]
    sl, nl = s0.clone().requires_grad_(True), n0.clone().requires_grad_(True)
    dd = torch.tensor(np.asarray(d, dtype=np.float64), device=dev)
    p = torch.tensor(np.asarray(pol, dtype=np.complex128), device=dev)
    Einc = torch.exp(1j * complex(k0) * (sl @ dd))[:, None] * p[None, :]
    tp = tmul(nl)
    L = (torch.sum(torch.conj(lam0) * Einc).real
         - torch.sum(torch.conj(lam1) * (0.5 * tp) - torch.conj(abar1) * tp).real)
    ls, ln = torch.autograd.grad(L, (sl, nl))
    GS, GN = GS + ls, GN + ln
    # carry the node derivatives to the vertices
    gV = torch.autograd.grad(torch.sum(GS * s) + torch.sum(GN * n) + torch.sum(GW * w), Vt)[0].cpu().numpy()
    t0 = mark("explicit_s", t0)
    # self-triangle blocks: -Re d/dv [ S_k0(lam0; Phi, -Psi) - S_kj(lam1; T Phi, -gamma Psi) on scatterer j ]
    terms = [(k0, 1.0, lam0, phi, b0)]
    for j in range(J):
        lj = torch.zeros_like(lam1)
        lj[idx_t[j]] = lam1[idx_t[j]]
        terms.append((kj[j], -1.0, lj, tphi, b1))
    gV -= self_triangle_vertex_derivative(V, F, terms, fd_rel)
    mark("self_blocks_s", t0)
    return float(C.item()), gV, np.sum(gV * vertex_normals(V, F), axis=1)


def impedance_cross_section_and_vertex_gradient(vertices, triangles, k0, Z, d, pol, order=16, depth=0, tol=1e-10,
                                                restart=150, order32=None, solve_kw=None, fd_rel=1e-5, plan_tol=0.0):
    """(C_sca, dC/dv f64[nv, 3], dC/d(delta_v) f64[nv]) of a good conductor under
    the impedance boundary condition (eqs. 2.24-2.25), C_sca from the far field:
    A Phi = 1/2 Phi + Op_k0(Phi, b(n)), b = c n x (n x Phi), c = i k0 / Z.  Besides
    the point sum's and the self blocks' geometry, the normal enters through b
    (its derivative is conj(bbar) . db, bbar = (Op_k0^H lambda)_b) and the far field."""
    from .gradients import far_field_cross_section
    from .solver import IbcProblem
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    F = np.ascontiguousarray(triangles, dtype=np.int64)
    q = nodes_of_mesh(V, F)
    pb = IbcProblem(q, k0, Z, order=order, depth=depth, order32=order32, tol=plan_tol)
    kw = dict(tol=tol, restart=restart, maxit=4000)
    kw.update(solve_kw or {})
    try:
        xd, _ = pb.solve(pb.rhs_planewave(d, pol), **kw)
        xg = xd.clone().requires_grad_(True)
        C = far_field_cross_section(pb, xg, pol)
        g = torch.autograd.grad(C, xg)[0]
        lam, _ = pb.solve(g.contiguous(), adjoint=True, **kw)
        phi, lam = xd[0].contiguous(), lam[0].contiguous()
        _, bbar = pb.p0.matvec_adjoint(lam)
    finally:
        pb.close()
    dev = phi.device
    c = 1j * complex(k0) / complex(Z)

    def b_of(nrm):
        nc = nrm.to(torch.complex128)
        return c * (nc * torch.sum(nc * phi, dim=1, keepdim=True) - phi)

    Vt = torch.from_numpy(V).to(dev).requires_grad_(True)
    s, n, w = nodes_of_triangles(Vt[torch.from_numpy(F).to(dev)])
    s0, n0, w0 = s.detach().contiguous(), n.detach().contiguous(), w.detach().contiguous()
    tri = torch.from_numpy(q["point_tri"]).to(dev)
    b0 = b_of(n0).contiguous()
    ds, dn, dw = shape_pairs(s0, n0, w0, tri, k0, lam, phi, b0)
    es, en, ew = _far_explicit(k0, phi, b_of, pol, s0, n0, w0)
    GS, GN, GW = es - ds.real, en - dn.real, ew - dw.real
    # Re sum conj(lam) . E_inc(s) - Re sum conj(bbar) . b(n)
    sl, nl = s0.clone().requires_grad_(True), n0.clone().requires_grad_(True)
    dd = torch.tensor(np.asarray(d, dtype=np.float64), device=dev)
    p = torch.tensor(np.asarray(pol, dtype=np.complex128), device=dev)
    Einc = torch.exp(1j * complex(k0) * (sl @ dd))[:, None] * p[None, :]
    L = torch.sum(torch.conj(lam) * Einc).real - torch.sum(torch.conj(bbar) * b_of(nl)).real
    ls, ln = torch.autograd.grad(L, (sl, nl))
    GS, GN = GS + ls, GN + ln
    gV = torch.autograd.grad(torch.sum(GS * s) + torch.sum(GN * n) + torch.sum(GW * w), Vt)[0].cpu().numpy()
    gV -= self_triangle_vertex_derivative(V, F, [(k0, 1.0, lam, phi, b0)], fd_rel)
    return float(C.item()), gV, np.sum(gV * vertex_normals(V, F), axis=1)
