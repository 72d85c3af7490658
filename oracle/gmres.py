"""Right-preconditioned flexible GMRES, complex FP64 (test infrastructure).

The paper solves the BEM system iteratively with fGMRES and a right
preconditioner, A M^{-1} (M x) = b (Sec. 3.1, eq. 3.1), the preconditioner
being applied by an inner GMRES on M.  Flexible GMRES keeps the
preconditioned directions z_j = P(v_j) so that P may change between
iterations (Saad's flexible variant, cited there).  Parameters the paper
does not give: restart length m, zero initial guess, 2-norm, classical
Gram-Schmidt done twice, happy breakdown when the new Hessenberg entry falls
below 1e-14 |A z_j|.

Steps (one cycle):
 1. r0 = b - A x0, beta = |r0|, v1 = r0 / beta, g = beta e1.
 2. for j = 1..m: z_j = P(v_j); w = A z_j; h = V^H w; w -= V h; h2 = V^H w;
    w -= V h2; h += h2; h_{j+1,j} = |w|; v_{j+1} = w / h_{j+1,j}.
 3. previous Givens rotations on column j, a new one zeroing h_{j+1,j}:
    c = |a| / sqrt(|a|^2 + |b|^2), s = (a/|a|) conj(b) / sqrt(|a|^2 + |b|^2),
    (a = h_jj, b = h_{j+1,j}); |g_{j+1}| estimates the residual.
 4. stop at |g_{j+1}| <= tol |b| or j = m: solve H y = g, x = x0 + Z y,
    recompute the true residual, restart if needed (up to maxit iterations).
"""

import numpy as np


def gmres_solve(A, b, P=None, tol=1e-8, restart=100, maxit=1000, x0=None):
    """Returns (x, info dict: iterations, residuals (true, per cycle), estimates)."""
    b = np.asarray(b, dtype=np.complex128)
    shape = b.shape
    bv = b.reshape(-1)
    nb = np.linalg.norm(bv)
    if P is None:
        def P(v):
            return v
    x = np.zeros_like(bv) if x0 is None else np.asarray(x0, dtype=np.complex128).reshape(-1).copy()
    if nb == 0.0:
        return x.reshape(shape), {"iterations": 0, "residual": 0.0, "estimates": []}

    def Av(v):
        return np.asarray(A(v.reshape(shape))).reshape(-1)

    def Pv(v):
        return np.asarray(P(v.reshape(shape))).reshape(-1)

    its = 0
    est = []
    true_res = []
    r = bv - Av(x) if x0 is not None else bv.copy()
    while True:
        beta = np.linalg.norm(r)
        true_res.append(beta / nb)
        if beta <= tol * nb or its >= maxit:
            break
        m = restart
        V = np.zeros((m + 1, bv.size), dtype=np.complex128)
        Z = np.zeros((m, bv.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = Pv(V[j])
            w = Av(Z[j])
            nw = np.linalg.norm(w)
            h = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            breakdown = hn <= 1e-14 * nw
            if not breakdown:
                V[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            aa = H[j, j]
            bb = H[j + 1, j]
            den = np.sqrt(abs(aa) ** 2 + abs(bb) ** 2)
            if abs(aa) == 0.0:
                cs[j] = 0.0
                sn[j] = 1.0
            else:
                cs[j] = abs(aa) / den
                sn[j] = (aa / abs(aa)) * np.conj(bb) / den
            H[j, j] = cs[j] * aa + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            est.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= tol * nb or breakdown or its >= maxit:
                break
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        x = x + Z[:j_done].T @ y
        r = bv - Av(x)
    return x.reshape(shape), {"iterations": its, "residual": true_res[-1], "true_residuals": true_res,
                              "estimates": est}
