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
