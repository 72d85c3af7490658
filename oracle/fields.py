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


def scattered_curl(nodes, k0, x, targets):
    """curl E_sca at host points.  Writing G = grad' g = -grad_r g and c = a x n,
    the summand of Op is grad_r g x c + (n . a) grad_r g + g b, whose curl in r is
    Hess(g) c + k^2 g c + grad_r g x b (the middle term is a gradient), so
    curl E_sca = -sum_beta w_beta [ Hess(g) c + k^2 g c + grad_r g x b ],
    with grad_r g = g' u, Hess(g) = (g'' - g'/R) u u^T + (g'/R) I, u = (r - s)/R,
    g' = (ik - 1/R) g, g'' = ((ik - 1/R)^2 + 1/R^2) g."""
    s, n, w = nodes["points"], nodes["normals"], nodes["weights"]
    a, b = x[:, 0:3], -x[:, 3:6]
    c = np.cross(a, n)                                           # [n, 3]
    t = np.asarray(targets, dtype=np.float64)
    d = t[:, None, :] - s[None, :, :]                            # r - s   [nt, n, 3]
    R = np.linalg.norm(d, axis=2)
    u = d / R[..., None]
    g = np.exp(1j * k0 * R) / (4.0 * np.pi * R)
    g1 = (1j * k0 - 1.0 / R) * g
    g2 = ((1j * k0 - 1.0 / R) ** 2 + 1.0 / R ** 2) * g
    uc = np.einsum("tnd,nd->tn", u, c)
    hess_c = ((g2 - g1 / R) * uc)[..., None] * u + (g1 / R)[..., None] * c[None]
    grad = g1[..., None] * u
    gxb = np.cross(grad, np.broadcast_to(b[None], grad.shape))
    summand = hess_c + (k0 ** 2) * g[..., None] * c[None] + gxb
    return -np.einsum("n,tnd->td", w, summand)


def stress_force(E, curlE, k0, normals, weights):
    """Time-averaged force oint <T> . n dA from the total fields E, curl E c128[m,3]
    sampled on a closed surface in the host medium (outward normals f64[m,3],
    area weights f64[m]).  With eps0 = mu0 = 1 the Maxwell stress tensor is
    <T> = 1/2 Re[ E E^* + H H^* - 1/2 (|E|^2 + |H|^2) I ], H = curl E / (i k0)."""
    H = np.asarray(curlE) / (1j * k0)
    E = np.asarray(E)
    n = np.asarray(normals, dtype=np.float64)
    En = np.sum(np.conj(E) * n, axis=1)
    Hn = np.sum(np.conj(H) * n, axis=1)
    e2 = np.sum(np.abs(E) ** 2, axis=1)
    h2 = np.sum(np.abs(H) ** 2, axis=1)
    Tn = 0.5 * np.real(E * En[:, None] + H * Hn[:, None] - 0.5 * (e2 + h2)[:, None] * n)
    return np.sum(np.asarray(weights)[:, None] * Tn, axis=0)
