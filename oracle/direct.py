"""Direct O(N^2) sum of one wavenumber's discretised operator (test infrastructure).

The EFIE (eq. 2.5) integrates, over the boundary of a domain, the kernel

    [n' grad'g - (n'.grad'g) I - grad'g n'] . E(s')  -  g I . [n' x curl' E(s')]

and the paper replaces every integral by the Nystrom sum  sum_j w_j f(s'_j, s)
(eq. 2.8).  With a = E(s') and b standing for whatever multiplies g, one
wavenumber's operator on 3-vector densities (a, b) at the quadrature nodes is

    Op_k(a, b)_alpha = sum_{beta: t(beta) != t(alpha)} w_beta [ K(n_beta; s_beta, s_alpha) . a_beta
                                                               + g(s_beta, s_alpha) b_beta ]
                       + corrections for the nodes of alpha's own triangle,

    K . a = n (grad'g . a) - (n . grad'g) a - grad'g (n . a),

where n is the source normal (the dyads of eqs. 2.5 and 2.12 written out).
Pairs inside one triangle are singular; the paper integrates them
analytically (Appendix B) and they enter through `corrections.py`.  The
fast multipole method of Sec. 2.2 approximates exactly this sum.

This is the plain definition: every target row loops over every source.
"""

import numpy as np

from .kernel import green, green_grad_src


def point_sum(points, normals, weights, point_tri, k, a, b, rows=None, chunk=256):
    """Nystrom point sum over off-triangle pairs (no self-triangle terms).

    points, normals: f64[n,3]; weights: f64[n]; point_tri: int[n];
    a, b: c128[n,3] (or [nrhs,n,3]); rows: optional target indices.
    Returns c128[len(rows),3] (or [nrhs,len(rows),3]).
    """
    points = np.asarray(points, dtype=np.float64)
    normals = np.asarray(normals, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    point_tri = np.asarray(point_tri)
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    batched = a.ndim == 3
    if not batched:
        a = a[None]
        b = b[None]
    n = points.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.zeros((a.shape[0], len(rows), 3), dtype=np.complex128)
    wa = weights[None, :, None] * a            # [r, n, 3]
    wb = weights[None, :, None] * b
    wna = np.einsum("nd,rnd->rn", normals, wa)  # w (n . a)
    for s in range(0, len(rows), chunk):
        tr = rows[s:s + chunk]
        tgt = points[tr][:, None, :]            # [t, 1, 3]
        src = points[None, :, :]                # [1, n, 3]
        mask = point_tri[tr][:, None] != point_tri[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.where(mask, green(k, src, tgt), 0.0)              # [t, n]
            G = np.where(mask[..., None], green_grad_src(k, src, tgt), 0.0)  # [t, n, 3]
        nG = np.einsum("nd,tnd->tn", normals, G)                      # n . grad'g
        for r in range(a.shape[0]):
            Ga = np.einsum("tnd,nd->tn", G, wa[r])                    # grad'g . (w a)
            y = (np.einsum("tn,nd->td", Ga, normals)                  # n (grad'g . a)
                 - np.einsum("tn,nd->td", nG, wa[r])                  # (n . grad'g) a
                 - np.einsum("tnd,n->td", G, wna[r])                  # grad'g (n . a)
                 + g @ wb[r])                                         # g b
            out[r, s:s + len(tr)] = y
    return out if batched else out[0]


def apply_corrections(normals, point_tri, blocks, a, b, rows=None):
    """Self-triangle terms: y_alpha = sum_j [K_beta(dV_{alpha j}) . a_beta + dG_{alpha j} b_beta],
    beta = nodes[t(alpha), j], K_beta(V) . a = n_beta (V . a) - (n_beta . V) a - V (n_beta . a).

    blocks = (nodes i64[ntri,m], dV c128[n,m,3], dG c128[n,m]) from
    corrections.self_blocks.  a, b: c128[n,3] or [nrhs,n,3].
    """
    nodes, dV, dG = blocks
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    batched = a.ndim == 3
    if not batched:
        a = a[None]
        b = b[None]
    n = normals.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    t = np.asarray(point_tri)[rows]
    out = np.zeros((a.shape[0], len(rows), 3), dtype=np.complex128)
    for j in range(nodes.shape[1]):
        src = nodes[t, j]
        nb = normals[src]
        V = dV[rows, j]
        G = dG[rows, j]
        nV = np.sum(nb * V, axis=1)
        for r in range(a.shape[0]):
            A = a[r][src]
            B = b[r][src]
            Va = np.sum(V * A, axis=1)
            na = np.sum(nb * A, axis=1)
            out[r] += nb * Va[:, None] - nV[:, None] * A - V * na[:, None] + G[:, None] * B
    return out if batched else out[0]


def op_direct(mesh_pts, k, a, b, corr=None, rows=None):
    """Op_k(a, b) = point sum + self-triangle corrections (if `corr` is given).

    mesh_pts: dict with points, normals, weights, point_tri.
    corr: None or the blocks from corrections.self_blocks.
    """
    y = point_sum(mesh_pts["points"], mesh_pts["normals"], mesh_pts["weights"],
                  mesh_pts["point_tri"], k, a, b, rows=rows)
    if corr is not None:
        y = y + apply_corrections(mesh_pts["normals"], mesh_pts["point_tri"], corr, a, b, rows=rows)
    return y
