"""Self-triangle integrals of g and grad'g (test infrastructure).

The singular part of eq. 2.12 is integrated analytically over the source's
own flat triangle (Sec. 2.2 after eq. 2.13, Appendix B).  For a target node O
inside triangle T the two element integrals are

    G_O = int_T g(s', O) dA'                 (weakly singular, eq. B.2)
    V_O = CPV int_T grad'g(s', O) dA'        (strongly singular, eq. B.4)

Polar coordinates about O (Fig. B.1): every edge e of T has its foot of the
perpendicular D_e, h_e = |OD_e|, unit vectors i_e = OD_e/h_e and
j_e = n x i_e, and the edge is swept by phi in [-theta_1, theta_2] with
radius rho_m(phi) = h_e / cos(phi) and direction rho^ = cos(phi) i_e + sin(phi) j_e.

* G_O = (1/4pi) sum_e int dphi int_0^rho_m exp(i k rho) drho
      = (1/4pi) sum_e int (exp(i k rho_m) - 1)/(i k) dphi.
  The paper keeps the first two Taylor terms (eq. B.2) and evaluates the
  static part with eq. B.3; the exact radial integral is used here because
  the Taylor form fails once |k| h is not small (lossy interiors).

* grad'g dA = (1/4pi) rho^ (i k rho - 1) exp(i k rho) / rho  drho dphi.  The
  -1/rho piece is the static CPV integral -(1/4pi) CPV int r/r^3 dA, which
  eq. B.9 gives in closed form; the remainder is regular:
      V_O = -(1/4pi) [eq. B.9] + (1/4pi) sum_e int rho^(phi) H(rho_m(phi)) dphi,
      H(rho) = int_0^rho [(i k u - 1) exp(i k u) + 1] / u du.
  The paper again keeps Taylor terms (eqs. B.4, B.5); the exact remainder is
  used here.

The angular integrals are done with Gauss-Legendre rules, doubled until
they change by less than 1e-12 relative; the radial integral in H is a
series for small |k| rho_m and the exponential integral E1 otherwise.

How the element integrals are shared among a triangle's nodes (the paper
only treats the one-node centroid rule, where the node gets the whole
integral):

* MEAN: each of the triangle's m nodes gets 1/m of G_O and V_O;
* LINEAR (default for three nodes): the density on the triangle is the linear
  interpolant L_beta through its three nodes, so node beta gets
      dG_{O,beta} = L_beta(O) G_O + grad L_beta . int_T g (s' - O) dA'
      dV_{O,beta} = L_beta(O) V_O + [int_T grad'g (s' - O)^T dA'] grad L_beta
  with the regular radial integrals
      int_0^rho_m rho e^{ik rho} drho         = [(1 - i k rho_m) e^{ik rho_m} - 1] / k^2
      int_0^rho_m (i k rho - 1) e^{ik rho} drho = rho_m e^{ik rho_m} - 2 (e^{ik rho_m} - 1)/(i k).
  With three nodes per triangle MEAN leaves the zero-mean in-triangle
  patterns of the Psi unknowns almost in the null space of the system;
  LINEAR does not.
"""

import numpy as np

_GL_CACHE = {}


def _gl(n):
    if n not in _GL_CACHE:
        _GL_CACHE[n] = np.polynomial.legendre.leggauss(n)
    return _GL_CACHE[n]


def edge_frames(O, tri, normal):
    """Per edge e = (V_e, V_{e+1}) of the CCW triangle: h, i, j, phi1, phi2.

    O: f64[m,3] targets, tri: f64[m,3,3], normal: f64[m,3].
    Returns arrays of shape [m,3] (h, phi1, phi2) and [m,3,3] (i, j).
    """
    m = O.shape[0]
    h = np.zeros((m, 3))
    ie = np.zeros((m, 3, 3))
    je = np.zeros((m, 3, 3))
    p1 = np.zeros((m, 3))
    p2 = np.zeros((m, 3))
    for e in range(3):
        A = tri[:, e]
        B = tri[:, (e + 1) % 3]
        t = B - A
        L = np.linalg.norm(t, axis=1)
        tu = t / L[:, None]
        # foot of the perpendicular from O onto the line AB
        D = A + np.sum((O - A) * tu, axis=1)[:, None] * tu
        OD = D - O
        hh = np.linalg.norm(OD, axis=1)
        ii = OD / hh[:, None]
        jj = np.cross(normal, ii)
        h[:, e] = hh
        ie[:, e] = ii
        je[:, e] = jj
        p1[:, e] = np.arctan2(np.sum((A - D) * jj, axis=1), hh)
        p2[:, e] = np.arctan2(np.sum((B - D) * jj, axis=1), hh)
    return h, ie, je, p1, p2


def static_cpv_r_over_r3(h, ie, p1, p2):
    """CPV int_T r/r^3 dA by eq. B.9: sum_e i_e ln[tan(pi/4 - th2/2) / tan(pi/4 + th1/2)],
    with th1 = -phi1 and th2 = phi2 the angles to the edge's end points."""
    th1 = -p1
    th2 = p2
    lr = np.log(np.tan(np.pi / 4 - th2 / 2) / np.tan(np.pi / 4 + th1 / 2))
    return np.sum(ie * lr[..., None], axis=1)


def static_drho_dphi(h, p1, p2):
    """int_T drho dphi by eq. B.3: sum_e h_e ln[tan(pi/4 + th1/2) / tan(pi/4 - th2/2)]."""
    th1 = -p1
    th2 = p2
    return np.sum(h * np.log(np.tan(np.pi / 4 + th1 / 2) / np.tan(np.pi / 4 - th2 / 2)), axis=1)


def _H(k, rho):
    """H(rho) = int_0^rho [(i k u - 1) e^{i k u} + 1]/u du, z = i k rho.

    Substituting w = i k u gives H = int_0^z [(w - 1) e^w + 1]/w dw
    = (e^z - 1) - F(z), F(z) = int_0^z (e^w - 1)/w dw = sum_{n>=1} z^n/(n n!).
    For |z| < 2 the series H = sum_{n>=2} (n-1) z^n/(n n!) is summed term by
    term; otherwise F(z) = -E1(-z) - ln(-z) - gamma (principal branches; -z has
    Re >= 0 because Im k >= 0), with E1 the exponential integral.  A fixed
    quadrature in u cannot follow the boundary layer of width 1/|k| that the
    integrand has at u = 0 when |k| rho is large (lossy interiors).
    """
    from scipy.special import exp1
    z0 = 1j * k * np.asarray(rho, dtype=np.float64)
    small = np.abs(z0) < 2.0
    zs = np.where(small, z0, 0.0)
    ser = np.zeros(z0.shape, dtype=np.complex128)
    term = zs * zs / 2.0                  # z^n / n! at n = 2
    for nn in range(2, 40):
        ser = ser + (nn - 1) * term / nn
        term = term * zs / (nn + 1)
    zl = np.where(small, 1.0, z0)
    big = np.exp(zl) - 1.0 + exp1(-zl) + np.log(-zl) + np.euler_gamma
    return np.where(small, ser, big)


def _angular(k, h, ie, je, p1, p2, nq):
    """Angular Gauss-Legendre sums for G and the regular part of V."""
    x, w = _gl(nq)
    m = h.shape[0]
    Gs = np.zeros(m, dtype=np.complex128)
    Vs = np.zeros((m, 3), dtype=np.complex128)
    for e in range(3):
        phi = 0.5 * (p2[:, e] - p1[:, e])[:, None] * (x + 1.0) + p1[:, e][:, None]   # [m,nq]
        jac = 0.5 * (p2[:, e] - p1[:, e])[:, None] * w
        rho = h[:, e][:, None] / np.cos(phi)
        if k == 0:
            gint = rho
        else:
            z = 1j * k * rho
            gint = np.where(np.abs(z) < 1e-4, rho * (1 + z / 2 + z * z / 6), (np.exp(z) - 1.0) / (1j * k))
        Gs += np.sum(jac * gint, axis=1)
        Hv = _H(k, rho)
        rhat = np.cos(phi)[..., None] * ie[:, e][:, None, :] + np.sin(phi)[..., None] * je[:, e][:, None, :]
        Vs += np.sum((jac * Hv)[..., None] * rhat, axis=1)
    return Gs, Vs


def self_terms(points, normals, point_tri, tri_vertices, k, tol=1e-12, chunk=4096):
    """G_O and V_O for every node O (its own triangle), k complex.

    Returns (V c128[n,3], G c128[n]).
    """
    points = np.asarray(points, dtype=np.float64)
    n = points.shape[0]
    V = np.zeros((n, 3), dtype=np.complex128)
    G = np.zeros(n, dtype=np.complex128)
    for s in range(0, n, chunk):
        sl = slice(s, min(n, s + chunk))
        O = points[sl]
        tri = tri_vertices[point_tri[sl]]
        nrm = normals[sl]
        h, ie, je, p1, p2 = edge_frames(O, tri, nrm)
        stat = static_cpv_r_over_r3(h, ie, p1, p2)
        nq = 16
        Gp, Vp = _angular(k, h, ie, je, p1, p2, nq)
        while True:
            nq *= 2
            Gn, Vn = _angular(k, h, ie, je, p1, p2, nq)
            dG = np.max(np.abs(Gn - Gp) / np.maximum(np.abs(Gn), 1e-300))
            dV = np.max(np.linalg.norm(Vn - Vp, axis=1) / np.maximum(np.linalg.norm(Vn, axis=1) + np.abs(stat).max(), 1e-300))
            Gp, Vp = Gn, Vn
            if dG < tol and dV < tol:
                break
            if nq >= 512:
                raise RuntimeError("angular quadrature did not converge")
        G[sl] = Gp / (4.0 * np.pi)
        V[sl] = (-stat + Vp) / (4.0 * np.pi)
    return V, G


def _first_moments(k, h, ie, je, p1, p2, nq=64):
    """Gv = int_T g (s'-O) dA' (c128[m,3]) and W = int_T grad'g (s'-O)^T dA' (c128[m,3,3])."""
    x, w = _gl(nq)
    m = h.shape[0]
    Gv = np.zeros((m, 3), dtype=np.complex128)
    W = np.zeros((m, 3, 3), dtype=np.complex128)
    for e in range(3):
        phi = 0.5 * (p2[:, e] - p1[:, e])[:, None] * (x + 1.0) + p1[:, e][:, None]
        jac = 0.5 * (p2[:, e] - p1[:, e])[:, None] * w
        rho = h[:, e][:, None] / np.cos(phi)
        z = 1j * k * rho
        E = np.exp(z)
        small = np.abs(z) < 0.1
        kk = k if k != 0 else 1.0
        # [(1 - z) e^z - 1] / k^2 = rho^2 sum_{n>=2} (n-1) z^(n-2) / n!  (cancels for small z)
        ser = np.zeros_like(z)
        term = np.ones_like(z) / 2.0          # z^0 / 2!
        for nn in range(2, 16):
            ser = ser + (nn - 1) * term
            term = term * z / (nn + 1)
        f1 = np.where(small, rho ** 2 * ser, ((1.0 - z) * E - 1.0) / (kk * kk))
        if k == 0:
            f2 = -rho
        else:
            f2 = rho * E - 2.0 * (E - 1.0) / (1j * kk)
        rh = np.cos(phi)[..., None] * ie[:, e][:, None, :] + np.sin(phi)[..., None] * je[:, e][:, None, :]
        Gv += np.sum((jac * f1)[..., None] * rh, axis=1)
        W += np.einsum("mq,mqi,mqj->mij", jac * f2, rh, rh)
    return Gv / (4.0 * np.pi), W / (4.0 * np.pi)


def triangle_nodes(point_tri, ntri):
    """i64[ntri, m]: the node indices of every triangle (m nodes each, in index order)."""
    point_tri = np.asarray(point_tri)
    order = np.argsort(point_tri, kind="stable")
    counts = np.bincount(point_tri, minlength=ntri)
    m = int(counts[0])
    if not np.all(counts == m) or m not in (1, 3):
        raise ValueError("every triangle must carry the same number of nodes, 1 or 3")
    return order.reshape(ntri, m)


def lagrange_gradients(points, normals, nodes):
    """grad L_beta (in the triangle plane) for the linear interpolant through a
    triangle's three nodes: f64[ntri, 3(beta), 3]."""
    S = points[nodes]                       # [t, 3, 3]
    nrm = normals[nodes[:, 0]]
    A = np.zeros((nodes.shape[0], 4, 4))
    A[:, :3, 0] = 1.0
    A[:, :3, 1:] = S
    A[:, 3, 1:] = nrm
    rhs = np.zeros((nodes.shape[0], 4, 3))
    rhs[:, 0, 0] = rhs[:, 1, 1] = rhs[:, 2, 2] = 1.0
    c = np.linalg.solve(A, rhs)             # [t, 4, 3]: columns = beta
    return np.transpose(c[:, 1:, :], (0, 2, 1))


def self_blocks(points, normals, point_tri, tri_vertices, k, mode="linear"):
    """Correction blocks of every target with every node of its own triangle.

    Returns (nodes i64[ntri,m], dV c128[n,m,3], dG c128[n,m]) where block
    (alpha, j) belongs to source node nodes[t(alpha), j].
    """
    points = np.asarray(points, dtype=np.float64)
    normals = np.asarray(normals, dtype=np.float64)
    point_tri = np.asarray(point_tri)
    ntri = tri_vertices.shape[0]
    nodes = triangle_nodes(point_tri, ntri)
    m = nodes.shape[1]
    V, G = self_terms(points, normals, point_tri, tri_vertices, k)
    n = points.shape[0]
    if mode == "mean" or m == 1:
        dV = np.repeat(V[:, None, :] / m, m, axis=1)
        dG = np.repeat(G[:, None] / m, m, axis=1)
        return nodes, dV, dG
    if mode != "linear":
        raise ValueError(mode)
    tri = tri_vertices[point_tri]
    h, ie, je, p1, p2 = edge_frames(points, tri, normals)
    Gv, W = _first_moments(k, h, ie, je, p1, p2)
    grads = lagrange_gradients(points, normals, nodes)[point_tri]      # [n, 3, 3]
    dV = np.einsum("nij,nbj->nbi", W, grads)
    dG = np.einsum("nbj,nj->nb", grads, Gv)
    own = nodes[point_tri]                                              # [n, 3]
    hit = own == np.arange(n)[:, None]
    dV = dV + hit[..., None] * V[:, None, :]
    dG = dG + hit * G[:, None]
    return nodes, dV, dG
