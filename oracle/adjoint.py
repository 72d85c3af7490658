"""Conjugate transpose of one wavenumber's discretised operator (test infrastructure).

The forward operator (direct.py) maps densities (a, b) to

    y_alpha = sum_{beta: t(beta) != t(alpha)} w_beta [ n_beta (G . a_beta) - (n_beta . G) a_beta
                                                      - G (n_beta . a_beta) + g b_beta ]
              + self-triangle terms,

with g = g(|s_beta - s_alpha|) and G = grad' g = f (s_beta - s_alpha),
f = (ikR - 1) e^{ikR} / (4 pi R^3) (eqs. 2.5, 2.8, 2.12).  Transposing each
term (the dyads n G^T, G n^T swap, the scalar terms stay) gives, per source
node beta,

    a_bar_beta = w_beta sum_alpha [ G (n_beta . y_alpha) - (n_beta . G) y_alpha - n_beta (G . y_alpha) ]
    b_bar_beta = w_beta sum_alpha g y_alpha,

and the conjugate transpose is conj(Op^T conj(y)).  This module writes that out
plainly: every source row loops over every target.  It is pinned in the tests
by the identity sum conj(y) . Op(a, b) = sum conj(a_bar) . a + conj(b_bar) . b
against the forward oracle.
"""

import numpy as np

from .kernel import green, green_grad_src


def point_sum_adjoint(points, normals, weights, point_tri, k, y, rows=None, chunk=256):
    """Op^H y of the point sum (no self-triangle terms).

    y: c128[n,3] (or [nrhs,n,3]); rows: optional source indices beta.
    Returns (a_bar, b_bar), each c128[len(rows),3] (or [nrhs,len(rows),3]).
    """
    points = np.asarray(points, dtype=np.float64)
    normals = np.asarray(normals, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    point_tri = np.asarray(point_tri)
    y = np.asarray(y, dtype=np.complex128)
    batched = y.ndim == 3
    if not batched:
        y = y[None]
    yc = np.conj(y)
    n = points.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    abar = np.zeros((y.shape[0], len(rows), 3), dtype=np.complex128)
    bbar = np.zeros_like(abar)
    for s in range(0, len(rows), chunk):
        sr = rows[s:s + chunk]
        src = points[sr][:, None, :]            # s_beta   [t, 1, 3]
        tgt = points[None, :, :]                # s_alpha  [1, n, 3]
        mask = point_tri[sr][:, None] != point_tri[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.where(mask, green(k, src, tgt), 0.0)                        # [t, n]
            G = np.where(mask[..., None], green_grad_src(k, src, tgt), 0.0)    # [t, n, 3]
        nb = normals[sr]                                                       # [t, 3]
        nG = np.einsum("td,tnd->tn", nb, G)                                    # n_beta . G
        w = weights[sr][:, None]
        for r in range(y.shape[0]):
            ny = np.einsum("td,nd->tn", nb, yc[r])                             # n_beta . y_alpha
            Gy = np.einsum("tnd,nd->tn", G, yc[r])                             # G . y_alpha
            a = (np.einsum("tnd,tn->td", G, ny)
                 - nG @ yc[r]
                 - nb * Gy.sum(axis=1)[:, None])
            abar[r, s:s + len(sr)] = np.conj(w * a)
            bbar[r, s:s + len(sr)] = np.conj(w * (g @ yc[r]))
    if not batched:
        return abar[0], bbar[0]
    return abar, bbar


def apply_corrections_adjoint(normals, point_tri, blocks, y, rows=None):
    """Op^H y of the self-triangle terms.  The forward term of target alpha,
    n_b (dV . a_b) - (n_b . dV) a_b - dV (n_b . a_b) + dG b_b with
    b = nodes[t(alpha), j], dV = dV[alpha, j], dG = dG[alpha, j], transposes for
    source beta = nodes[t, j] into the sum over the nodes alpha of t of
    dV (n_b . y_alpha) - (n_b . dV) y_alpha - n_b (dV . y_alpha)  and  dG y_alpha.

    blocks = (nodes, dV, dG) from corrections.self_blocks.  Returns (a_bar, b_bar).
    """
    nodes, dV, dG = blocks
    y = np.asarray(y, dtype=np.complex128)
    batched = y.ndim == 3
    if not batched:
        y = y[None]
    yc = np.conj(y)
    n = normals.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    abar = np.zeros((y.shape[0], len(rows), 3), dtype=np.complex128)
    bbar = np.zeros_like(abar)
    for q, be in enumerate(rows):
        t = point_tri[be]
        jb = int(np.nonzero(nodes[t] == be)[0][0])
        nb = normals[be]
        for al in nodes[t]:
            V = dV[al, jb]
            for r in range(y.shape[0]):
                Y = yc[r, al]
                abar[r, q] += V * np.dot(nb, Y) - np.dot(nb, V) * Y - nb * np.dot(V, Y)
                bbar[r, q] += dG[al, jb] * Y
    abar, bbar = np.conj(abar), np.conj(bbar)
    if not batched:
        return abar[0], bbar[0]
    return abar, bbar
