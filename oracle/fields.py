"""Fields away from the surface from the solved unknowns (test infrastructure).

Eq. 2.5 holds with the jump term 1/2 replaced by 1 at points off the boundary.
In the row convention of the 6N system (host rows 1/2 Phi + Op_{k0}(Phi, -Psi) = E_inc,
interior rows 1/2 T Phi - Op_{k1}(T Phi, -gamma Psi) = 0) this gives

    host points:      E(r)   = E_inc(r) - Op_{k0}(Phi, -Psi)(r),  so E_sca(r) = -Op_{k0}(Phi, -Psi)(r)
    interior points:  E_1(r) = Op_{k1}(T Phi, -gamma Psi)(r)

with Op(a, b)(r) = sum_beta w_beta [ n_beta (G . a_beta) - (n_beta . G) a_beta - G (n_beta . a_beta) + g b_beta ],
g = g(s_beta, r), G = grad' g = f (s_beta - r).  Far from the scatterer,
g -> e^{ikr}/(4 pi r) e^{-ik rhat . s} and G -> -i k rhat g, so
E_sca ~ e^{ikr}/r F(rhat) with

    F(rhat) = -(1/4pi) sum_beta w_beta e^{-ik rhat . s_beta}
              [ -ik ( n (rhat . a) - (n . rhat) a - rhat (n . a) ) + b ],   a = Phi, b = -Psi.

This module writes these sums out directly: every target loops over every node.
"""

import numpy as np

from .kernel import green, green_grad_src


def op_at(nodes, k, a, b, targets):
    """Op_k(a, b) evaluated at points off the surface; a, b c128[n,3]; returns c128[nt,3]."""
    s, n, w = nodes["points"], nodes["normals"], nodes["weights"]
    t = np.asarray(targets, dtype=np.float64)[:, None, :]
    g = green(k, s[None], t)
    G = green_grad_src(k, s[None], t)
    wa = w[:, None] * a
    wb = w[:, None] * b
    Ga = np.einsum("tnd,nd->tn", G, wa)
    nG = np.einsum("nd,tnd->tn", n, G)
    wna = np.sum(n * wa, axis=1)
    return Ga @ n - np.einsum("tn,nd->td", nG, wa) - np.einsum("tnd,n->td", G, wna) + g @ wb


def scattered_field(nodes, k0, x, targets):
    """E_sca at host points from the solution x c128[n,6]."""
    return -op_at(nodes, k0, x[:, 0:3], -x[:, 3:6], targets)


def interior_field(nodes, k1, eps, gamma, x, targets):
    """E_1 at points inside the scatterer."""
    n = nodes["normals"]
    phi = x[:, 0:3]
    tphi = phi + ((1.0 - eps) / eps) * n * np.sum(n * phi, axis=1, keepdims=True)
    return op_at(nodes, k1, tphi, -gamma * x[:, 3:6], targets)


def far_field(nodes, k0, x, dirs):
    """F(rhat) for unit directions dirs f64[nd,3]; returns c128[nd,3]."""
    s, n, w = nodes["points"], nodes["normals"], nodes["weights"]
    r = np.asarray(dirs, dtype=np.float64)
    a, b = x[:, 0:3], -x[:, 3:6]
    ph = np.exp(-1j * k0 * (r @ s.T)) * w[None, :]                       # [nd, n]
    ra = a @ r.T                                                         # [n, nd] rhat . a
    nr = n @ r.T                                                         # [n, nd] n . rhat
    na = np.sum(n * a, axis=1)                                           # [n]
    term = (np.einsum("nd,nk->knd", n, ra) - np.einsum("nk,nd->knd", nr, a)
            - np.einsum("kd,n->knd", r, na))                             # [nd, n, 3]
    return -(1.0 / (4.0 * np.pi)) * np.einsum("kn,knd->kd", ph, -1j * k0 * term + b[None])
