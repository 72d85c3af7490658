"""Shape derivatives of one wavenumber's point sum, and the cross-section
functionals they feed (TEST INFRASTRUCTURE: only tests/ use this module).

For fixed densities (a, b) and adjoint weights lam, the bilinear form of the
point sum of `direct.point_sum` (eq. 2.8 applied to the dyadic kernel of
eqs. 2.5 and 2.12, with g of eq. 2.4) is

    B = sum_alpha conj(lam_alpha) . PS(a, b)_alpha
      = sum_{alpha, beta: t(beta) != t(alpha)} w_beta [ grad'g . c + g e ],

    u = conj(lam_alpha),
    c = (u . n_beta) a_beta - (u . a_beta) n_beta - (n_beta . a_beta) u,
    e = u . b_beta,

since u . K(n) a = (u . n)(G . a) - (n . G)(u . a) - (u . G)(n . a) = G . c
for G = grad'g.  With d = s_beta - s_alpha, R = |d|, g = e^{ikR} / (4 pi R),
grad'g = f(R) d with f = (ikR - 1) g / R^2 and f'(R) / R = (3 - 3ikR - k^2 R^2) g / R^4:

    dB/ds_beta  = sum_alpha w_beta [ f c + ((f'/R)(d . c) + f e) d ]
    dB/ds_alpha = -sum_beta (the same summand)
    dB/dn_beta  = sum_alpha w_beta f [ (d . a_beta) u - (u . a_beta) d - (d . u) a_beta ]
    dB/dw_beta  = sum_alpha [ f (d . c) + g e ]

(holomorphic derivatives of the complex B with respect to the real
coordinates; a node is both a source and a target, so ds sums both roles).
Pinned by central differences of `direct.point_sum`.

The scattering cross section C_sca (eq. 4.2) is taken in two forms: on the
scatterer's surface from the unknowns, and as oint |F|^2 dOmega over the
far-field amplitude of `fields.far_field`.
"""

import numpy as np

from .fields import far_field
from .kernel import green


def pair_derivatives(points, normals, weights, point_tri, k, lam, a, b, chunk=64):
    """(dB/ds c128[n,3], dB/dn c128[n,3], dB/dw c128[n]) of the bilinear form above."""
    s = np.asarray(points, dtype=np.float64)
    nv = np.asarray(normals, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    tri = np.asarray(point_tri)
    lam = np.asarray(lam, dtype=np.complex128)
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    k = complex(k)
    n = s.shape[0]
    ds = np.zeros((n, 3), dtype=np.complex128)
    dn = np.zeros((n, 3), dtype=np.complex128)
    dw = np.zeros(n, dtype=np.complex128)
    na = np.sum(nv * a, axis=1)                                   # n_beta . a_beta   [n]
    for lo in range(0, n, chunk):
        rows = np.arange(lo, min(n, lo + chunk))
        u = np.conj(lam[rows])                                    # [t, 3]
        d = s[None, :, :] - s[rows][:, None, :]                   # s_beta - s_alpha  [t, n, 3]
        mask = tri[rows][:, None] != tri[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.where(mask, green(k, s[None, :, :], s[rows][:, None, :]), 0.0)
            R = np.sqrt(np.sum(d * d, axis=2))
            ikR = 1j * k * R
            f = np.where(mask, (ikR - 1.0) * g / R ** 2, 0.0)
            fp = np.where(mask, (3.0 - 3.0 * ikR + ikR * ikR) * g / R ** 4, 0.0)
        un = u @ nv.T                                             # u . n_beta   [t, n]
        ua = u @ a.T                                              # u . a_beta
        e = u @ b.T                                               # u . b_beta
        c = (un[..., None] * a[None] - ua[..., None] * nv[None]
             - na[None, :, None] * u[:, None, :])                 # [t, n, 3]
        dc = np.sum(d * c, axis=2)
        summand = w[None, :, None] * (f[..., None] * c + (fp * dc + f * e)[..., None] * d)
        ds += np.sum(summand, axis=0)
        ds[rows] -= np.sum(summand, axis=1)
        da = np.einsum("tnd,nd->tn", d, a)
        du = np.einsum("tnd,td->tn", d, u)
        dn += w[:, None] * np.sum(f[..., None] * (da[..., None] * u[:, None, :] - ua[..., None] * d
                                                  - du[..., None] * a[None]), axis=0)
        dw += np.sum(f * dc + g * e, axis=0)
    return ds, dn, dw


def bilinear_point_sum(points, normals, weights, point_tri, k, lam, a, b):
    """B = sum conj(lam) . PS(a, b) by the plain point sum (the definition the
    derivatives above are pinned against)."""
    from .direct import point_sum
    y = point_sum(points, normals, weights, point_tri, k, a, b)
    return np.sum(np.conj(lam) * y)


def incident(points, normals, k0, d, pol):
    """E_inc = p e^{i k0 d . s} and Psi_inc = n x curl E_inc at the nodes."""
    d = np.asarray(d, dtype=np.float64)
    p = np.asarray(pol, dtype=np.complex128)
    e = np.exp(1j * k0 * (points @ d))
    E = e[:, None] * p[None, :]
    curl = 1j * k0 * np.cross(d[None, :], E)
    return E, np.cross(normals, curl)


def cross_section_surface(nodes, k0, x, d, pol):
    """C_sca of eq. 4.2 on the scatterer's surface, from the unknowns x c128[n,6]:
    E_sca = Phi - E_inc, n x H_sca = (Psi - Psi_inc) / (i k0) (eps0 = mu0 = 1, Z0 = 1), so
    C = -(1/|E0|^2) sum w Re[ E_sca . conj(n x H_sca) ]."""
    s, n, w = nodes["points"], nodes["normals"], nodes["weights"]
    E, Pi = incident(s, n, k0, d, pol)
    esca = x[:, 0:3] - E
    nh = (x[:, 3:6] - Pi) / (1j * k0)
    e0 = np.sum(np.abs(np.asarray(pol)) ** 2)
    return -np.sum(w * np.real(np.sum(esca * np.conj(nh), axis=1))) / e0


def sphere_rule(nt, nph):
    """Directions and weights of the product rule on the unit sphere: Gauss-Legendre
    in cos(theta) (nt nodes) times the uniform rule in phi (nph nodes)."""
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = 2.0 * np.pi * np.arange(nph) / nph
    st = np.sqrt(1.0 - ct ** 2)
    dirs = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)),
                     np.outer(ct, np.ones(nph))], axis=-1).reshape(-1, 3)
    wts = np.outer(wt, np.full(nph, 2.0 * np.pi / nph)).reshape(-1)
    return dirs, wts


def cross_section_far(nodes, k0, x, pol, nt=24, nph=48):
    """C_sca = oint |F|^2 dOmega / |E0|^2 with F of `fields.far_field`."""
    dirs, wts = sphere_rule(nt, nph)
    F = far_field(nodes, k0, x, dirs)
    e0 = np.sum(np.abs(np.asarray(pol)) ** 2)
    return np.sum(wts * np.sum(np.abs(F) ** 2, axis=1)) / e0
