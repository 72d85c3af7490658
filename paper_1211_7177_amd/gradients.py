"""Scattering cross section and its gradient in the permittivity by the adjoint method.

Two forms of the scattering cross section serve as the functional.  The
surface form is
C_sca = (Z0 / |E0|^2) oint Re(E_sca x H_sca^*) . n dA (eq. 4.2) taken over the
scatterer's own surface, where the unknowns give the scattered fields
directly: E_sca = Phi - E_inc and n x H_sca = (Psi - Psi_inc) / (i omega mu0),
with Psi = n x curl E (eq. 2.12).  In the units of this library
(eps0 = mu0 = 1, omega = k0, Z0 = 1) and with (E x H^*) . n = -E . (n x H^*),

    C_sca = -(1/|E0|^2) sum_beta w_beta Re[ E_sca,beta . conj((Psi_beta - Psi_inc,beta) / (i k0)) ].

The far-field form is C_sca = oint |F|^2 dOmega / |E0|^2 with the far-field
amplitude F = L x of `bem_field`; its gradient in x is L^H (2 w F) / |E0|^2,
taken by `bem_far_field_adjoint`.  It needs Phi and Psi only through the
radiating sum, not Psi on its own, and stays accurate where the surface form
does not (on metals with edges the discrete Psi converges slowly).

For dC/d eps: A(eps) x = b gives dx = -A^{-1} (dA/deps) x deps, so with
g = grad_x C (torch's convention: dC = Re <g, dx>) and the adjoint solution
lambda = A^{-H} g,

    dC = -Re[ <lambda, (dA/deps) x> deps ].

Only the interior rows depend on eps: through T = I + (1 - eps)/eps n n^T
(dT/deps = -n n^T / eps^2) and through k1 = k0 sqrt(eps mu) (dk1/deps = k1 / (2 eps)),
whose operator derivative is taken as the central difference of two products
at k1 +- delta (plans of the same octree and order).

For a shape family nodes(theta) (theta in R^m: vertex displacements, along the
vertex normals or any other field, applied to the mesh, with points, normals,
weights and self-triangle blocks all following from the moved triangles) both
the system and the functional move: A(theta) x = b(theta), C = f(x, theta).  Then

    dC/dtheta_i = df/dtheta_i |_x + Re < lambda, d(b - A x)/dtheta_i |_x >,

again with lambda = A^{-H} g, so one forward and one adjoint solve serve every
parameter; each parameter adds the central difference of b - A x and of f at
theta +- h e_i (two problem builds and two products on the octree depth of the
unperturbed shape, with x held fixed).
The derivative in every mesh vertex at once, with no rebuilt problem per
parameter, is `shape.cross_section_and_vertex_gradient`.
"""

import numpy as np
import torch

from ._abi import Plan
from .autograd import far_field
from .postprocess import sphere_quadrature
from .solver import BemProblem, IbcProblem, MultiBemProblem, _nodes_of


def _incident(nodes, k0, d, pol, dtype=torch.complex128):
    """E_inc and Psi_inc = n x curl E_inc at the nodes (user order), GPU tensors [n, 3]."""
    s = torch.from_numpy(np.ascontiguousarray(nodes["points"])).cuda()
    nrm = torch.from_numpy(np.ascontiguousarray(nodes["normals"])).cuda()
    d = torch.tensor(np.asarray(d, dtype=np.float64), device="cuda")
    p = torch.tensor(np.asarray(pol, dtype=np.complex128), device="cuda")
    ph = torch.exp(1j * complex(k0) * (s @ d))
    E = ph[:, None] * p[None, :]
    curl = (1j * complex(k0)) * torch.linalg.cross(d.to(torch.complex128).expand_as(E), E)
    return E.to(dtype), torch.linalg.cross(nrm.to(torch.complex128), curl).to(dtype)


def scattering_cross_section(nodes, k0, x, d, pol):
    """C_sca of the solution x [n, 6] (or [1, n, 6]) for the incident wave p exp(i k0 d . s),
    as a differentiable torch scalar."""
    if x.dim() == 3:
        x = x[0]
    E, Pi = _incident(nodes, k0, d, pol)
    w = torch.from_numpy(np.ascontiguousarray(nodes["weights"])).cuda()
    e0 = float(np.sum(np.abs(np.asarray(pol)) ** 2))
    esca = x[:, 0:3] - E
    nh = (x[:, 3:6] - Pi) / (1j * complex(k0))
    return -torch.sum(w * torch.real(torch.sum(esca * torch.conj(nh), dim=1))) / e0


def far_field_cross_section(problem, x, pol, nt=24, nph=48):
    """C_sca = oint |F|^2 dOmega / |E0|^2 from the far-field amplitudes of the
    solution x [1, n, nu] (Gauss-Legendre x uniform rule on the unit sphere),
    as a differentiable torch scalar.  Unlike the surface form of eq. 4.2 it
    does not use Psi, whose discrete values converge slowly near edges and on
    metals; it is positive by construction."""
    if x.dim() == 2:
        x = x[None]
    dirs, wts = sphere_quadrature(nt, nph)
    F = far_field(problem, x, dirs)
    e0 = float(np.sum(np.abs(np.asarray(pol)) ** 2))
    w = torch.from_numpy(wts).cuda()
    return torch.sum(w[None, :, None] * (F.real ** 2 + F.imag ** 2)) / e0


def _functional(kind, problem, nodes, k0, x, d, pol):
    if kind == "surface":
        return scattering_cross_section(nodes, k0, x, d, pol)
    if kind == "far":
        return far_field_cross_section(problem, x, pol)
    raise ValueError("functional must be 'surface' or 'far'")


def cross_section_and_eps_gradient(nodes, k0, eps, d, pol, order=16, depth=0, tol=1e-10, restart=150,
                                   dk_rel=1e-5, mu=1.0, functional="surface", order32=None, solve_kw=None):
    """(C_sca, dC/dRe eps, dC/dIm eps) for one scatterer and one plane wave, by one
    forward solve, one adjoint solve and three FMM products of the interior plan.
    functional: "surface" (eq. 4.2 on the scatterer's surface) or "far" (the
    far-field integral of `far_field_cross_section`).  order32 builds FP32 plans
    too, for solve_kw such as {"mixed": "nested"} (extra options of both solves)."""
    eps = complex(eps)
    pb = BemProblem(nodes, k0, eps, mu=mu, order=order, depth=depth, order32=order32)
    dep = pb.p0.info()["depth"]
    rhs = pb.rhs_planewave(d, pol)
    kw = dict(tol=tol, restart=restart, maxit=4000)
    kw.update(solve_kw or {})
    xd, _ = pb.solve(rhs, **kw)
    xg = xd.clone().requires_grad_(True)
    C = _functional(functional, pb, nodes, k0, xg, d, pol)
    g = torch.autograd.grad(C, xg)[0]                              # dC = Re <g, dx>
    lam, _ = pb.solve(g.contiguous(), adjoint=True, **kw)
    # (dA/deps) x: interior rows only
    nrm = torch.from_numpy(np.ascontiguousarray(nodes["normals"])).cuda().to(torch.complex128)
    phi, psi = xd[0, :, 0:3], xd[0, :, 3:6]
    nphi = torch.sum(nrm * phi, dim=1, keepdim=True)
    dT_phi = (-1.0 / eps ** 2) * nrm * nphi
    T_phi = phi + ((1.0 - eps) / eps) * nrm * nphi
    k1 = pb.k1
    delta = dk_rel * abs(k1)
    pts, nn, ww = nodes["points"], nodes["normals"], nodes["weights"]
    pk = dict(depth=dep, point_tri=nodes["point_tri"], tri_vertices=nodes["tri_vertices"])
    Pp = Plan(pts, nn, ww, k1 + delta, order, **pk)
    Pm = Plan(pts, nn, ww, k1 - delta, order, **pk)
    gamma = pb.mu
    b_int = (-gamma) * psi
    dOp = (Pp.matvec(T_phi.contiguous(), b_int.contiguous())
           - Pm.matvec(T_phi.contiguous(), b_int.contiguous())) / (2.0 * delta)
    zero = torch.zeros_like(phi)
    term = 0.5 * dT_phi - pb.p1.matvec(dT_phi.contiguous(), zero) - (k1 / (2.0 * eps)) * dOp
    u = torch.sum(torch.conj(lam[0, :, 3:6]) * term).item()
    Pp.close()
    Pm.close()
    pb.close()
    return C.item(), -u.real, u.imag


def cross_section_and_shape_gradient(nodes_at, nparams, k0, eps, d, pol, order=16, depth=0, tol=1e-10, restart=150,
                                     h=1e-3, mu=1.0, functional="surface", make_problem=None):
    """(C_sca, dC/dtheta f64[nparams]) at theta = 0 for the shape family
    nodes_at(theta) (a callable returning the Nystrom nodes of the moved mesh,
    node order unchanged), by one forward and one adjoint solve and, per
    parameter, two rebuilt problems and products.  functional as for
    `cross_section_and_eps_gradient`.  make_problem(nodes, depth), when given,
    builds the system instead of a one-scatterer BemProblem (for instance a
    MultiBemProblem with its region map); depth is the requested octree depth
    of the host plan (0 first, then the depth that build chose)."""
    eps = complex(eps) if np.isscalar(eps) else eps
    if make_problem is None:
        def make_problem(q, dep):
            return BemProblem(q, k0, eps, mu=mu, order=order, depth=dep)
    q0 = nodes_at(np.zeros(nparams))
    pb = make_problem(q0, depth)
    dep = pb.p0.info()["depth"]
    kw = dict(tol=tol, restart=restart, maxit=4000)
    xd, _ = pb.solve(pb.rhs_planewave(d, pol), **kw)
    xg = xd.clone().requires_grad_(True)
    C = _functional(functional, pb, q0, k0, xg, d, pol)
    g = torch.autograd.grad(C, xg)[0]
    lam, _ = pb.solve(g.contiguous(), adjoint=True, **kw)
    pb.close()
    grad = np.zeros(nparams)
    for i in range(nparams):
        res, fun = [], []
        for sgn in (1.0, -1.0):
            th = np.zeros(nparams)
            th[i] = sgn * h
            q = nodes_at(th)
            p = make_problem(q, dep)
            res.append(p.rhs_planewave(d, pol) - p.apply(xd))
            fun.append(_functional(functional, p, q, k0, xd, d, pol).item())
            p.close()
        dr = (res[0] - res[1]) / (2.0 * h)
        grad[i] = (fun[0] - fun[1]) / (2.0 * h) + torch.sum(torch.conj(lam) * dr).real.item()
    return C.item(), grad


def cross_section_and_eps_gradients_multi(nodes, region, k0, eps, d, pol, order=16, depth=0, depths=None, tol=1e-10,
                                          restart=150, dk_rel=1e-5, mu=None, functional="far", order32=None,
                                          solve_kw=None):
    """(C_sca, g) for J scatterers (region[alpha] = j) under one plane wave,
    g[j] = (dC/dRe eps_j, dC/dIm eps_j), from one forward and one adjoint solve
    of the several-scatterer system.  Scatterer j's permittivity enters only
    its own interior rows, through T_j and k_j, so each derivative is the
    single-scatterer expression on scatterer j's nodes with its own plan (and
    two plans at k_j +- delta for dOp/dk)."""
    region = np.asarray(region)
    J = int(region.max()) + 1
    eps = [complex(e) for e in eps]
    mu = [complex(m) for m in (mu if mu is not None else [1.0] * J)]
    pb = MultiBemProblem(nodes, region, k0, eps, mu=mu, order=order, depth=depth, depths=depths, order32=order32)
    kw = dict(tol=tol, restart=restart, maxit=4000)
    kw.update(solve_kw or {})
    xd, _ = pb.solve(pb.rhs_planewave(d, pol), **kw)
    xg = xd.clone().requires_grad_(True)
    C = _functional(functional, pb, nodes, k0, xg, d, pol)
    g = torch.autograd.grad(C, xg)[0]
    lam, _ = pb.solve(g.contiguous(), adjoint=True, **kw)
    grads = np.zeros((J, 2))
    for j in range(J):
        idx = torch.from_numpy(np.nonzero(region == j)[0]).cuda()
        sub = _nodes_of(nodes, region == j)
        nrm = torch.from_numpy(sub["normals"]).cuda().to(torch.complex128)
        phi, psi = xd[0, idx, 0:3], xd[0, idx, 3:6]
        nphi = torch.sum(nrm * phi, dim=1, keepdim=True)
        e = eps[j]
        dT_phi = (-1.0 / e ** 2) * nrm * nphi
        T_phi = phi + ((1.0 - e) / e) * nrm * nphi
        kj = pb.kj[j]
        delta = dk_rel * abs(kj)
        Pj = pb.pj[j]
        pk = dict(depth=Pj.info()["depth"], point_tri=sub["point_tri"], tri_vertices=sub["tri_vertices"])
        Pp = Plan(sub["points"], sub["normals"], sub["weights"], kj + delta, order, **pk)
        Pm = Plan(sub["points"], sub["normals"], sub["weights"], kj - delta, order, **pk)
        b_int = ((-mu[j]) * psi).contiguous()
        dOp = (Pp.matvec(T_phi.contiguous(), b_int) - Pm.matvec(T_phi.contiguous(), b_int)) / (2.0 * delta)
        term = 0.5 * dT_phi - Pj.matvec(dT_phi.contiguous(), torch.zeros_like(phi)) - (kj / (2.0 * e)) * dOp
        u = torch.sum(torch.conj(lam[0, idx, 3:6]) * term).item()
        grads[j] = (-u.real, u.imag)
        Pp.close()
        Pm.close()
    val = C.item()
    pb.close()
    return val, grads


def cross_section_and_impedance_gradient(nodes, k0, Z, d, pol, order=16, depth=0, tol=1e-10, restart=150, h=1e-6):
    """(C_sca, dC/dRe Z, dC/dIm Z) of a good conductor under the impedance
    boundary condition (eq. 2.25), with C_sca from the far field.  The system
    1/2 Phi + Op_k0(Phi, c n x (n x Phi)) = E_inc depends on Z only through
    c = i k0 / Z, so (dA/dZ) x = Op_k0(0, (dc/dZ) (n (n . Phi) - Phi)) with
    dc/dZ = -i k0 / Z^2: one product of the k0 plan beside the forward and
    adjoint solves.  The far field depends on Z through the same b term; that
    explicit part is the central difference of the functional at Z +- h and
    Z +- ih with the solution held fixed."""
    Z = complex(Z)
    pb = IbcProblem(nodes, k0, Z, order=order, depth=depth)
    dep = pb.p0.info()["depth"]
    kw = dict(tol=tol, restart=restart, maxit=4000)
    xd, _ = pb.solve(pb.rhs_planewave(d, pol), **kw)
    xg = xd.clone().requires_grad_(True)
    C = far_field_cross_section(pb, xg, pol)
    g = torch.autograd.grad(C, xg)[0]
    lam, _ = pb.solve(g.contiguous(), adjoint=True, **kw)
    nrm = torch.from_numpy(np.ascontiguousarray(nodes["normals"])).cuda().to(torch.complex128)
    phi = xd[0]
    dc = -1j * complex(k0) / Z ** 2
    bz = dc * (nrm * torch.sum(nrm * phi, dim=1, keepdim=True) - phi)
    dAx = pb.p0.matvec(torch.zeros_like(phi), bz.contiguous())
    u = torch.sum(torch.conj(lam[0]) * dAx).item()
    pb.close()
    f = []
    for dz in (h, -h, 1j * h, -1j * h):
        p = IbcProblem(nodes, k0, Z + dz, order=order, depth=dep)
        f.append(far_field_cross_section(p, xd, pol).item())
        p.close()
    return C.item(), (f[0] - f[1]) / (2 * h) - u.real, (f[2] - f[3]) / (2 * h) + u.imag
