"""The vertex-gradient assembly of `paper_1211_7177_amd.shape` on the CPU (no
GPU): its device calls (the BEM problem and solves, the point-sum derivative
passes, the self-triangle blocks, the cross-section functional) are replaced by
the oracle's own pieces, and the assembled dC/dv is checked against central
differences of the oracle's solves.  This pins the adjoint-method bookkeeping
(which terms enter, their signs, the chain rule through the node rule); the GPU
tests check the device pieces themselves."""

import numpy as np
import pytest
import torch

from oracle.adjoint import apply_corrections_adjoint, point_sum_adjoint
from oracle.bem import BemProblem as OracleBem
from oracle.corrections import self_blocks as oracle_blocks
from oracle.gmres import gmres_solve
from oracle.shape import cross_section_far, cross_section_surface, pair_derivatives, sphere_rule
from synthetic import nystrom3, torus
from synthetic.meshes import Mesh

D, POL = [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]


class _InteriorPlan:
    def __init__(self, ob):
        self.ob = ob

    def matvec_adjoint(self, y):
        nd = self.ob.nodes
        a, b = point_sum_adjoint(nd["points"], nd["normals"], nd["weights"], nd["point_tri"], self.ob.k1,
                                 y.numpy())
        ca, cb = apply_corrections_adjoint(nd["normals"], nd["point_tri"], self.ob.corr1, y.numpy())
        return torch.from_numpy(a + ca), torch.from_numpy(b + cb)


class _OracleProblem:
    def __init__(self, q, k0, eps, mu=1.0, **kw):
        self.ob = OracleBem(q, k0, eps, mu)
        self.k1, self.mu, self.p1 = self.ob.k1, self.ob.mu, _InteriorPlan(self.ob)

    def rhs_planewave(self, d, p):
        return torch.from_numpy(self.ob.rhs_planewave(d, p))[None]

    def solve(self, rhs, adjoint=False, **kw):
        A = self.ob.apply_adjoint if adjoint else self.ob.apply
        x, _ = gmres_solve(A, rhs[0].detach().numpy(), self.ob.block_preconditioner(adjoint=adjoint), tol=1e-13,
                           restart=300)
        return torch.from_numpy(x)[None], {"iterations": 0}

    def close(self):
        pass


def _functional(kind, pb, q, k0, x, d, pol):
    """Both C_sca forms in torch (differentiable in x), as the oracle defines them."""
    x = x[0] if x.dim() == 3 else x
    s, n, w = (torch.from_numpy(q[key]) for key in ("points", "normals", "weights"))
    e0 = float(np.sum(np.abs(np.asarray(pol)) ** 2))
    if kind == "far":
        dirs, wts = sphere_rule(24, 48)
        r, W = torch.from_numpy(dirs), torch.from_numpy(wts)
        a, b = x[:, 0:3], -x[:, 3:6]
        ph = w[None, :] * torch.exp(-1j * k0 * (r @ s.T))
        nc, rc = n.to(torch.complex128), r.to(torch.complex128)
        term = (-1j * k0) * ((ph * (rc @ a.T)) @ nc - (ph * (r @ n.T).to(torch.complex128)) @ a
                             - rc * (ph @ torch.sum(nc * a, 1))[:, None]) + ph @ b
        F = -term / (4.0 * np.pi)
        return torch.sum(W[:, None] * (F.real ** 2 + F.imag ** 2)) / e0
    dd, p = torch.tensor(d, dtype=torch.float64), torch.tensor(pol, dtype=torch.complex128)
    E = torch.exp(1j * k0 * (s @ dd))[:, None] * p[None]
    curl = (1j * k0) * torch.linalg.cross(dd.to(torch.complex128).expand_as(E), E)
    Pi = torch.linalg.cross(n.to(torch.complex128), curl)
    return -torch.sum(w * torch.real(torch.sum((x[:, :3] - E) * torch.conj((x[:, 3:] - Pi) / (1j * k0)), 1))) / e0


def _pairs(s, n, w, tri, k, lam, a, b):
    out = pair_derivatives(s.numpy(), n.numpy(), w.numpy(), tri.numpy(), k, lam.numpy(), a.numpy(), b.numpy())
    return tuple(torch.from_numpy(t) for t in out)


def _blocks(pts, nrm, point_tri, tv, k, device=None, mode="linear"):
    _, dv, dg = oracle_blocks(pts, nrm, point_tri, tv, k, mode=mode)
    return torch.from_numpy(dv), torch.from_numpy(dg)


@pytest.mark.parametrize("functional", ["far", "surface"])
def test_vertex_gradient_assembly_matches_oracle_differences(monkeypatch, functional):
    from paper_1211_7177_amd import shape
    monkeypatch.setattr(shape, "BemProblem", _OracleProblem)
    monkeypatch.setattr(shape, "_functional", _functional)
    monkeypatch.setattr(shape, "shape_pairs", _pairs)
    monkeypatch.setattr(shape, "self_blocks", _blocks)
    m = torus(1.0, 0.35, 8, 5)                     # 80 triangles, 240 nodes
    V, F = m.vertices.copy(), m.triangles.copy()
    k0, eps = 1.2, 3.0 + 0.2j
    C, gV, _ = shape.cross_section_and_vertex_gradient(V, F, k0, eps, D, POL, functional=functional)

    def oracle_C(Vx):
        q = nystrom3(Mesh(Vx, F.astype(np.int32)))
        ob = OracleBem(q, k0, eps)
        x, _ = gmres_solve(ob.apply, ob.rhs_planewave(D, POL), ob.block_preconditioner(), tol=1e-13, restart=300)
        return cross_section_far(q, k0, x, POL) if functional == "far" else cross_section_surface(q, k0, x, D, POL)

    W = np.random.default_rng(5).standard_normal(V.shape)
    fd = (oracle_C(V + 1e-4 * W) - oracle_C(V - 1e-4 * W)) / 2e-4
    an = np.sum(gV * W)
    assert abs(C - oracle_C(V)) <= 1e-12 * abs(C)
    assert abs(an - fd) <= 1e-6 * np.sum(np.abs(gV * W)), (an, fd)
    assert np.linalg.norm(gV.sum(axis=0)) <= 1e-9 * np.abs(gV).sum()


class _MultiPlan:
    def __init__(self, ob, j):
        self.ob, self.j = ob, j

    def matvec_adjoint(self, y):
        sub = self.ob.sub[self.j]
        a, b = point_sum_adjoint(sub["points"], sub["normals"], sub["weights"], sub["point_tri"], self.ob.k[self.j],
                                 y.numpy())
        ca, cb = apply_corrections_adjoint(sub["normals"], sub["point_tri"], self.ob.corr[self.j], y.numpy())
        return torch.from_numpy(a + ca), torch.from_numpy(b + cb)


class _OracleMulti:
    def __init__(self, q, region, k0, eps, mu=None, **kw):
        from oracle.bem import MultiBemProblem
        self.ob = MultiBemProblem(q, region, k0, eps, mu)
        self.kj, self.pj = self.ob.k, [_MultiPlan(self.ob, j) for j in range(self.ob.J)]

    def rhs_planewave(self, d, p):
        return torch.from_numpy(self.ob.rhs_planewave(d, p))[None]

    def solve(self, rhs, adjoint=False, **kw):
        A = self.ob.apply_adjoint if adjoint else self.ob.apply
        x, _ = gmres_solve(A, rhs[0].detach().numpy(), self.ob.block_preconditioner(adjoint=adjoint), tol=1e-13,
                           restart=300)
        return torch.from_numpy(x)[None], {"iterations": 0}

    def close(self):
        pass


def test_vertex_gradient_assembly_two_scatterers(monkeypatch):
    """The several-scatterer path (host rows over both scatterers, each interior
    over its own nodes) with the oracle standing in, far-field C_sca."""
    from oracle.bem import MultiBemProblem
    from paper_1211_7177_amd import shape, solver
    from synthetic import icosphere, union
    monkeypatch.setattr(shape, "_functional", _functional)
    monkeypatch.setattr(shape, "shape_pairs", _pairs)
    monkeypatch.setattr(shape, "self_blocks", _blocks)
    monkeypatch.setattr(solver, "MultiBemProblem", _OracleMulti)
    m, reg = union([icosphere(2, 0.5), torus(0.5, 0.2, 6, 4)], [[0, 0, 0], [1.6, 0.2, 0.1]])
    V, F = m.vertices.copy(), m.triangles.copy()
    eps, k0 = [2.25 + 0.3j, 4.0 + 0.1j], 1.3
    C, gV, _ = shape.cross_section_and_vertex_gradient(V, F, k0, eps, D, POL, functional="far", tri_region=reg)

    def oracle_C(Vx):
        q = nystrom3(Mesh(Vx, F.astype(np.int32)))
        ob = MultiBemProblem(q, np.repeat(reg, 3), k0, eps)
        x, _ = gmres_solve(ob.apply, ob.rhs_planewave(D, POL), ob.block_preconditioner(), tol=1e-13, restart=300)
        return cross_section_far(q, k0, x, POL)

    W = np.random.default_rng(7).standard_normal(V.shape)
    fd = (oracle_C(V + 1e-4 * W) - oracle_C(V - 1e-4 * W)) / 2e-4
    an = np.sum(gV * W)
    assert abs(an - fd) <= 1e-6 * np.sum(np.abs(gV * W)), (an, fd)
    assert np.linalg.norm(gV.sum(axis=0)) <= 1e-9 * np.abs(gV).sum()


class _IbcPlan:
    def __init__(self, ob):
        self.ob = ob

    def matvec_adjoint(self, y):
        nd = self.ob.nodes
        a, b = point_sum_adjoint(nd["points"], nd["normals"], nd["weights"], nd["point_tri"], self.ob.k0, y.numpy())
        ca, cb = apply_corrections_adjoint(nd["normals"], nd["point_tri"], self.ob.corr0, y.numpy())
        return torch.from_numpy(a + ca), torch.from_numpy(b + cb)


class _OracleIbc:
    def __init__(self, q, k0, Z, **kw):
        from oracle.bem import IbcProblem
        self.ob = IbcProblem(q, k0, Z)
        self.p0, self.q, self.k0, self.c = _IbcPlan(self.ob), q, k0, 1j * k0 / Z

    def rhs_planewave(self, d, p):
        return torch.from_numpy(self.ob.rhs_planewave(d, p))[None]

    def solve(self, rhs, adjoint=False, **kw):
        A = self.ob.apply_adjoint if adjoint else self.ob.apply
        x, _ = gmres_solve(A, rhs[0].detach().numpy(), self.ob.block_preconditioner(adjoint=adjoint), tol=1e-13,
                           restart=300)
        return torch.from_numpy(x)[None], {"iterations": 0}

    def close(self):
        pass


def _far_ibc(pb, x, pol):
    x = x[0] if x.dim() == 3 else x
    nn = torch.from_numpy(pb.q["normals"]).to(torch.complex128)
    b = pb.c * (nn * torch.sum(nn * x, 1, keepdim=True) - x)
    return _functional("far", pb, pb.q, pb.k0, torch.cat([x, -b], 1), None, pol)


def test_impedance_vertex_gradient_assembly(monkeypatch):
    """The impedance path (the density c n x (n x Phi) moves with the normals)
    with the oracle standing in, far-field C_sca."""
    from oracle.bem import IbcProblem
    from paper_1211_7177_amd import gradients, shape, solver
    monkeypatch.setattr(shape, "shape_pairs", _pairs)
    monkeypatch.setattr(shape, "self_blocks", _blocks)
    monkeypatch.setattr(solver, "IbcProblem", _OracleIbc)
    monkeypatch.setattr(gradients, "far_field_cross_section", _far_ibc)
    m = torus(1.0, 0.35, 8, 5)
    V, F = m.vertices.copy(), m.triangles.copy()
    k0, Z = 1.2, 0.1 - 0.2j
    C, gV, _ = shape.impedance_cross_section_and_vertex_gradient(V, F, k0, Z, D, POL)

    def oracle_C(Vx):
        q = nystrom3(Mesh(Vx, F.astype(np.int32)))
        ob = IbcProblem(q, k0, Z)
        x, _ = gmres_solve(ob.apply, ob.rhs_planewave(D, POL), ob.block_preconditioner(), tol=1e-13, restart=300)
        return cross_section_far(q, k0, np.concatenate([x, -ob.c * ob.nnx(x)], axis=1), POL)

    W = np.random.default_rng(3).standard_normal(V.shape)
    fd = (oracle_C(V + 1e-4 * W) - oracle_C(V - 1e-4 * W)) / 2e-4
    an = np.sum(gV * W)
    assert abs(C - oracle_C(V)) <= 1e-12 * abs(C)
    assert abs(an - fd) <= 1e-6 * np.sum(np.abs(gV * W)), (an, fd)
    assert np.linalg.norm(gV.sum(axis=0)) <= 1e-9 * np.abs(gV).sum()
