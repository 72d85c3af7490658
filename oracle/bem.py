"""The 6N-unknown BEM system for one scatterer in vacuum (test infrastructure).

Unknowns per node alpha: x_alpha = (Phi_alpha, Psi_alpha) in C^6 with
Phi = E_0(s_alpha) and Psi = n x (curl E_0)(s_alpha), n the outward normal of
the scatterer (eq. 2.12).  Applying the EFIE (2.5) in the host medium
(outward normal of the host = -n, so the dyadic kernel and Psi change sign)
and inside the scatterer with the boundary conditions (2.6)-(2.7),
E_1 = T E_0 and n x curl E_1 = gamma Psi, gives two 3-vector rows per node:

    (A x)_alpha[0:3] = 1/2 Phi_alpha + Op_{k0}(Phi, -Psi)_alpha
    (A x)_alpha[3:6] = 1/2 T_alpha Phi_alpha - Op_{k1}(T Phi, -gamma Psi)_alpha
    b_alpha          = (E_inc(s_alpha), 0)

T = I + (eps_0 - eps_1)/eps_1 n n, gamma = mu_1/mu_0 (eq. 2.13), the host is
vacuum (eps_0 = mu_0 = 1) and there is no incident field inside.  The paper
prints the jump term as 1/2 I in every domain block; eq. 2.5 applies it to
E_1 = T E_0, so the interior block uses 1/2 T.  Op_k is `direct.op_direct`.

The preconditioner M = A_self keeps only the coincident-node part of the
self-triangle integrals (Sec. 3.1, eq. 3.2 and the sentence after it):
with (dV, dG) the correction block of a node with itself,

    M_alpha = [[ 1/2 I + K(dV_0),          -dG_0 I      ],
               [ 1/2 T - K(dV_1) T,  gamma dG_1 I ]]

where K(V) a = n (V . a) - (n . V) a - V (n . a).
"""

import numpy as np

from .corrections import self_blocks
from .kernel import wavenumber
from .native import point_sum_c
from .direct import apply_corrections
from .adjoint import apply_corrections_adjoint, point_sum_adjoint


class BemProblem:
    def __init__(self, nodes, k0: float, eps: complex, mu: complex = 1.0, mode="linear"):
        self.nodes = nodes
        self.k0 = complex(k0)
        self.eps = complex(eps)
        self.mu = complex(mu)
        self.k1 = wavenumber(k0, eps, mu)
        self.gamma = self.mu
        n = nodes["points"].shape[0]
        self.n = n
        self.normals = nodes["normals"]
        args = (nodes["points"], nodes["normals"], nodes["point_tri"], nodes["tri_vertices"])
        self.corr0 = self_blocks(*args, self.k0, mode=mode)
        self.corr1 = self_blocks(*args, self.k1, mode=mode)
        self.matvecs = 0

    def op(self, k, corr, a, b):
        nd = self.nodes
        y = point_sum_c(nd["points"], nd["normals"], nd["weights"], nd["point_tri"], k, a, b)
        return y + apply_corrections(nd["normals"], nd["point_tri"], corr, a, b)

    def T(self, phi):
        """T Phi = Phi + (1 - eps)/eps n (n . Phi)."""
        n = self.normals
        c = (1.0 - self.eps) / self.eps
        return phi + c * n * np.sum(n * phi, axis=-1, keepdims=True)

    def apply(self, x):
        """A x for x c128[n,6] (or [nrhs,n,6])."""
        x = np.asarray(x, dtype=np.complex128)
        phi = x[..., 0:3]
        psi = x[..., 3:6]
        tphi = self.T(phi)
        r0 = 0.5 * phi + self.op(self.k0, self.corr0, phi, -psi)
        r1 = 0.5 * tphi - self.op(self.k1, self.corr1, tphi, -self.gamma * psi)
        self.matvecs += 1
        return np.concatenate([r0, r1], axis=-1)

    def op_adjoint(self, k, corr, y):
        """(a_bar, b_bar) = Op_k^H y (point sum and self-triangle terms)."""
        nd = self.nodes
        a, b = point_sum_adjoint(nd["points"], nd["normals"], nd["weights"], nd["point_tri"], k, y)
        ca, cb = apply_corrections_adjoint(nd["normals"], nd["point_tri"], corr, y)
        return a + ca, b + cb

    def apply_adjoint(self, v):
        """A^H v for v c128[n,6].  Each row of A is a sum of terms; transposing
        them one by one, with T symmetric (T^H = conj(T)) and (a_j, b_j) = Op_kj^H v_j:
            (A^H v)[0:3] = 1/2 v0 + a0 + 1/2 T^H v1 - T^H a1
            (A^H v)[3:6] = -b0 + conj(gamma) b1."""
        v = np.asarray(v, dtype=np.complex128)
        v0, v1 = v[..., 0:3], v[..., 3:6]
        a0, b0 = self.op_adjoint(self.k0, self.corr0, v0)
        a1, b1 = self.op_adjoint(self.k1, self.corr1, v1)
        n = self.normals
        ch = np.conj((1.0 - self.eps) / self.eps)

        def TH(u):
            return u + ch * n * np.sum(n * u, axis=-1, keepdims=True)

        r0 = 0.5 * v0 + a0 + TH(0.5 * v1 - a1)
        r1 = -b0 + np.conj(self.gamma) * b1
        return np.concatenate([r0, r1], axis=-1)

    def rhs_planewave(self, d, p):
        """b = (p exp(i k0 d . s), 0) for one direction d and polarisation p."""
        s = self.nodes["points"]
        e = np.exp(1j * self.k0 * (s @ np.asarray(d, dtype=np.float64)))
        out = np.zeros((self.n, 6), dtype=np.complex128)
        out[:, 0:3] = e[:, None] * np.asarray(p)[None, :]
        return out

    def precond_blocks(self):
        """M_alpha as c128[n,6,6]."""
        n = self.normals
        N = self.n
        I3 = np.eye(3)
        nn = n[:, :, None] * n[:, None, :]
        T = I3[None] + ((1.0 - self.eps) / self.eps) * nn

        def Kmat(V):
            # K(V) a = n (V . a) - (n . V) a - V (n . a)  ->  matrix n V^T - (n.V) I - V n^T
            nV = np.sum(n * V, axis=1)
            return n[:, :, None] * V[:, None, :] - nV[:, None, None] * I3[None] - V[:, :, None] * n[:, None, :]

        V0, G0 = self._diag(self.corr0)
        V1, G1 = self._diag(self.corr1)
        M = np.zeros((N, 6, 6), dtype=np.complex128)
        M[:, 0:3, 0:3] = 0.5 * I3[None] + Kmat(V0)
        M[:, 0:3, 3:6] = -G0[:, None, None] * I3[None]
        M[:, 3:6, 0:3] = 0.5 * T - Kmat(V1) @ T
        M[:, 3:6, 3:6] = self.gamma * G1[:, None, None] * I3[None]
        return M

    def _diag(self, blocks):
        """The block of every node with itself: (dV c128[n,3], dG c128[n])."""
        nodes, dV, dG = blocks
        own = nodes[self.nodes["point_tri"]] == np.arange(self.n)[:, None]
        j = np.argmax(own, axis=1)
        return dV[np.arange(self.n), j], dG[np.arange(self.n), j]

    def block_preconditioner(self, adjoint=False):
        """v -> M^{-1} v, or M^{-H} v (the adjoint system's preconditioner)."""
        Minv = np.linalg.inv(self.precond_blocks())
        if adjoint:
            Minv = np.conj(np.transpose(Minv, (0, 2, 1)))

        def apply(v):
            return np.einsum("nij,...nj->...ni", Minv, v)

        return apply


class IbcProblem:
    """The impedance-boundary-condition system of eq. 2.25 (test infrastructure).

    With n x E = Z n x (n x H) (eq. 2.24) and n x curl E = i omega mu0 n x H,
    the tangential Psi of the dielectric system is -c n x (n x Phi) with
    c = i omega mu0 / Z = i k0 / Z (vacuum units).  Substituting into the host
    rows leaves three unknowns per node, Phi = E_0:

        (A Phi)_alpha = 1/2 Phi_alpha + Op_{k0}(Phi, c n x (n x Phi))_alpha = E_inc(s_alpha),

    n x (n x Phi) = n (n . Phi) - Phi.  The preconditioner keeps the coincident-node
    block 1/2 I + K(dV) + c dG (n n^T - I).
    """

    def __init__(self, nodes, k0: float, Z: complex, mode="linear"):
        self.nodes = nodes
        self.k0 = complex(k0)
        self.Z = complex(Z)
        self.c = 1j * self.k0 / self.Z
        self.n = nodes["points"].shape[0]
        self.normals = nodes["normals"]
        args = (nodes["points"], nodes["normals"], nodes["point_tri"], nodes["tri_vertices"])
        self.corr0 = self_blocks(*args, self.k0, mode=mode)

    def nnx(self, v):
        """n x (n x v) = n (n . v) - v."""
        n = self.normals
        return n * np.sum(n * v, axis=-1, keepdims=True) - v

    def apply(self, phi):
        nd = self.nodes
        phi = np.asarray(phi, dtype=np.complex128)
        b = self.c * self.nnx(phi)
        y = point_sum_c(nd["points"], nd["normals"], nd["weights"], nd["point_tri"], self.k0, phi, b)
        return 0.5 * phi + y + apply_corrections(nd["normals"], nd["point_tri"], self.corr0, phi, b)

    def apply_adjoint(self, v):
        """A^H v = 1/2 v + a + conj(c) n x (n x b), (a, b) = Op_{k0}^H v (n x (n x .) is real symmetric)."""
        nd = self.nodes
        v = np.asarray(v, dtype=np.complex128)
        a, b = point_sum_adjoint(nd["points"], nd["normals"], nd["weights"], nd["point_tri"], self.k0, v)
        ca, cb = apply_corrections_adjoint(nd["normals"], nd["point_tri"], self.corr0, v)
        return 0.5 * v + a + ca + np.conj(self.c) * self.nnx(b + cb)

    def rhs_planewave(self, d, p):
        s = self.nodes["points"]
        e = np.exp(1j * self.k0 * (s @ np.asarray(d, dtype=np.float64)))
        return e[:, None] * np.asarray(p)[None, :]

    def precond_blocks(self):
        n = self.normals
        I3 = np.eye(3)
        nn = n[:, :, None] * n[:, None, :]
        nodes, dV, dG = self.corr0
        own = nodes[self.nodes["point_tri"]] == np.arange(self.n)[:, None]
        j = np.argmax(own, axis=1)
        V = dV[np.arange(self.n), j]
        G = dG[np.arange(self.n), j]
        nV = np.sum(n * V, axis=1)
        K = n[:, :, None] * V[:, None, :] - nV[:, None, None] * I3[None] - V[:, :, None] * n[:, None, :]
        return 0.5 * I3[None] + K + (self.c * G)[:, None, None] * (nn - I3[None])

    def block_preconditioner(self, adjoint=False):
        Minv = np.linalg.inv(self.precond_blocks())
        if adjoint:
            Minv = np.conj(np.transpose(Minv, (0, 2, 1)))

        def apply(v):
            return np.einsum("nij,...nj->...ni", Minv, v)

        return apply


def subset_nodes(nodes, mask):
    """The nodes of one scatterer (mask over all nodes) as a node set of its own:
    points, normals, weights, triangles renumbered in order of first appearance."""
    idx = np.nonzero(mask)[0]
    tri = nodes["point_tri"][idx]
    uniq, inv = np.unique(tri, return_inverse=True)
    return {"points": nodes["points"][idx], "normals": nodes["normals"][idx], "weights": nodes["weights"][idx],
            "point_tri": inv.astype(np.int32), "tri_vertices": nodes["tri_vertices"][uniq]}


class MultiBemProblem:
    """J scatterers in vacuum (Sec. 2.1, Fig. 1): node alpha belongs to scatterer
    region[alpha] = j with permittivity eps[j] and permeability mu[j].  The host
    rows use all nodes, the interior rows of scatterer j only its own nodes:

        (A x)_alpha[0:3] = 1/2 Phi_alpha + Op_{k0}(Phi, -Psi)_alpha                       (all nodes)
        (A x)_alpha[3:6] = 1/2 T_j Phi_alpha - Op_{kj}(T_j Phi, -gamma_j Psi)|_{j}(alpha)  (scatterer j)

    with k_j = k0 sqrt(eps_j mu_j), T_j = I + (1 - eps_j)/eps_j n n, gamma_j = mu_j.
    J = 1 is BemProblem.  The preconditioner keeps each node's 6x6 self block."""

    def __init__(self, nodes, region, k0, eps, mu=None, mode="linear"):
        self.nodes = nodes
        self.region = np.asarray(region)
        self.J = int(self.region.max()) + 1
        self.k0 = complex(k0)
        self.eps = [complex(e) for e in eps]
        self.mu = [complex(m) for m in (mu if mu is not None else [1.0] * self.J)]
        self.k = [wavenumber(k0, e, m) for e, m in zip(self.eps, self.mu)]
        self.n = nodes["points"].shape[0]
        self.normals = nodes["normals"]
        args = (nodes["points"], nodes["normals"], nodes["point_tri"], nodes["tri_vertices"])
        self.corr0 = self_blocks(*args, self.k0, mode=mode)
        self.sub = [subset_nodes(nodes, self.region == j) for j in range(self.J)]
        self.idx = [np.nonzero(self.region == j)[0] for j in range(self.J)]
        self.corr = [self_blocks(s["points"], s["normals"], s["point_tri"], s["tri_vertices"], kj, mode=mode)
                     for s, kj in zip(self.sub, self.k)]

    def _op(self, nodes, k, corr, a, b):
        y = point_sum_c(nodes["points"], nodes["normals"], nodes["weights"], nodes["point_tri"], k, a, b)
        return y + apply_corrections(nodes["normals"], nodes["point_tri"], corr, a, b)

    def _T(self, j, phi, conj=False):
        n = self.normals[self.idx[j]]
        c = (1.0 - self.eps[j]) / self.eps[j]
        if conj:
            c = np.conj(c)
        return phi + c * n * np.sum(n * phi, axis=-1, keepdims=True)

    def apply(self, x):
        x = np.asarray(x, dtype=np.complex128)
        phi, psi = x[:, 0:3], x[:, 3:6]
        r = np.zeros_like(x)
        r[:, 0:3] = 0.5 * phi + self._op(self.nodes, self.k0, self.corr0, phi, -psi)
        for j in range(self.J):
            i = self.idx[j]
            tphi = self._T(j, phi[i])
            r[i, 3:6] = 0.5 * tphi - self._op(self.sub[j], self.k[j], self.corr[j], tphi, -self.mu[j] * psi[i])
        return r

    def apply_adjoint(self, v):
        """Each scatterer's interior rows transpose as in BemProblem.apply_adjoint."""
        v = np.asarray(v, dtype=np.complex128)
        nd = self.nodes
        a0, b0 = point_sum_adjoint(nd["points"], nd["normals"], nd["weights"], nd["point_tri"], self.k0, v[:, 0:3])
        ca, cb = apply_corrections_adjoint(nd["normals"], nd["point_tri"], self.corr0, v[:, 0:3])
        r = np.zeros_like(v)
        r[:, 0:3] = 0.5 * v[:, 0:3] + a0 + ca
        r[:, 3:6] = -(b0 + cb)
        for j in range(self.J):
            i = self.idx[j]
            s = self.sub[j]
            a1, b1 = point_sum_adjoint(s["points"], s["normals"], s["weights"], s["point_tri"], self.k[j], v[i, 3:6])
            c1, d1 = apply_corrections_adjoint(s["normals"], s["point_tri"], self.corr[j], v[i, 3:6])
            r[i, 0:3] += self._T(j, 0.5 * v[i, 3:6] - a1 - c1, conj=True)
            r[i, 3:6] += np.conj(self.mu[j]) * (b1 + d1)
        return r

    def rhs_planewave(self, d, p):
        s = self.nodes["points"]
        e = np.exp(1j * self.k0 * (s @ np.asarray(d, dtype=np.float64)))
        out = np.zeros((self.n, 6), dtype=np.complex128)
        out[:, 0:3] = e[:, None] * np.asarray(p)[None, :]
        return out

    def precond_blocks(self):
        I3 = np.eye(3)
        M = np.zeros((self.n, 6, 6), dtype=np.complex128)

        def diag(blocks, nodes, n_nodes):
            nd_, dV, dG = blocks
            own = nd_[nodes["point_tri"]] == np.arange(n_nodes)[:, None]
            jj = np.argmax(own, axis=1)
            return dV[np.arange(n_nodes), jj], dG[np.arange(n_nodes), jj]

        def Kmat(n, V):
            nV = np.sum(n * V, axis=1)
            return n[:, :, None] * V[:, None, :] - nV[:, None, None] * I3[None] - V[:, :, None] * n[:, None, :]

        V0, G0 = diag(self.corr0, self.nodes, self.n)
        n = self.normals
        M[:, 0:3, 0:3] = 0.5 * I3[None] + Kmat(n, V0)
        M[:, 0:3, 3:6] = -G0[:, None, None] * I3[None]
        for j in range(self.J):
            i = self.idx[j]
            nj = n[i]
            V1, G1 = diag(self.corr[j], self.sub[j], len(i))
            T = I3[None] + ((1.0 - self.eps[j]) / self.eps[j]) * nj[:, :, None] * nj[:, None, :]
            M[i, 3:6, 0:3] = 0.5 * T - Kmat(nj, V1) @ T
            M[i, 3:6, 3:6] = self.mu[j] * G1[:, None, None] * I3[None]
        return M

    def block_preconditioner(self, adjoint=False):
        Minv = np.linalg.inv(self.precond_blocks())
        if adjoint:
            Minv = np.conj(np.transpose(Minv, (0, 2, 1)))

        def apply(v):
            return np.einsum("nij,...nj->...ni", Minv, v)

        return apply
