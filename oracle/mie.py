"""Mie series for a homogeneous sphere (test infrastructure; an external check).

The paper benchmarks its solver against Mie theory (Sec. 3.2) without
stating it; this module writes it from Bohren & Huffman's vector spherical
harmonic expansions (the book the paper cites for its mode analysis), for an
x-polarised plane wave exp(i k z) in vacuum hitting a sphere of radius a,
relative permittivity eps and mu = 1, time factor exp(-i omega t):

  E_inc = sum_n E_n (M_o1n^(1) - i N_e1n^(1)),          E_n = i^n (2n+1)/(n(n+1))
  E_sca = sum_n E_n (i a_n N_e1n^(3) - b_n M_o1n^(3))
  E_in  = sum_n E_n (c_n M_o1n^(1) - i d_n N_e1n^(1))    (wavenumber m k)

with the coefficients of B&H eqs. 4.52-4.53 (mu_1 = mu), curl M = k N and
curl N = k M, and the series cut at n_max = x + 4 x^(1/3) + 2 (Wiscombe).
Spherical Bessel functions come from scipy.special.
"""

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def _jn(n, z, d=False):
    return spherical_jn(n, z, derivative=d)


def _hn(n, z, d=False):
    return spherical_jn(n, z, derivative=d) + 1j * spherical_yn(n, z, derivative=d)


def _cj(n, z, d=False):
    """Spherical j_n for complex arguments via scipy (complex supported)."""
    return spherical_jn(n, z, derivative=d)


def coefficients(x: float, m: complex, nmax=None):
    """a_n, b_n, c_n, d_n for n = 1..nmax; x = k a, m = sqrt(eps)."""
    if nmax is None:
        nmax = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    n = np.arange(1, nmax + 1)
    mx = m * x
    jx = _jn(n, x)
    djx = _jn(n, x, True)
    hx = _hn(n, x)
    dhx = _hn(n, x, True)
    jmx = _cj(n, mx)
    djmx = _cj(n, mx, True)
    psi_x = x * jx
    dpsi_x = jx + x * djx
    xi_x = x * hx
    dxi_x = hx + x * dhx
    psi_mx = mx * jmx
    dpsi_mx = jmx + mx * djmx
    a = (m * psi_mx * dpsi_x - psi_x * dpsi_mx) / (m * psi_mx * dxi_x - xi_x * dpsi_mx)
    b = (psi_mx * dpsi_x - m * psi_x * dpsi_mx) / (psi_mx * dxi_x - m * xi_x * dpsi_mx)
    # [x h(x)]' = dxi_x, [x j(x)]' = dpsi_x, [mx j(mx)]' = dpsi_mx
    c = (jx * dxi_x - hx * dpsi_x) / (jmx * dxi_x - hx * dpsi_mx)
    d = m * (jx * dxi_x - hx * dpsi_x) / (m * m * jmx * dxi_x - hx * dpsi_mx)
    return n, a, b, c, d


def _pi_tau(nmax, mu):
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros((nmax + 1,) + mu.shape)
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def _vsh(n, k, r, theta, phi, kind):
    """M_o1n, M_e1n, N_o1n, N_e1n in Cartesian components at points; kind 1 (j) or 3 (h)."""
    rho = k * r
    f = _cj if kind == 1 else _hn
    z = np.array([f(nn, rho) for nn in n])                  # [nmax, npts]
    dz = np.array([f(nn, rho, True) for nn in n])
    drz = (z + rho * dz) / rho                               # [rho z]'/rho
    mu = np.cos(theta)
    pi, tau = _pi_tau(len(n), mu)
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    er = np.stack([st * cp, st * sp, ct], -1)
    et = np.stack([ct * cp, ct * sp, -st], -1)
    ep = np.stack([-sp, cp, np.zeros_like(sp)], -1)
    nn1 = (n * (n + 1))[:, None]
    Mo = (cp * pi * z)[..., None] * et - (sp * tau * z)[..., None] * ep
    Me = (-sp * pi * z)[..., None] * et - (cp * tau * z)[..., None] * ep
    No = (sp * nn1 * st * pi * z / rho)[..., None] * er + (sp * tau * drz)[..., None] * et \
        + (cp * pi * drz)[..., None] * ep
    Ne = (cp * nn1 * st * pi * z / rho)[..., None] * er + (cp * tau * drz)[..., None] * et \
        - (sp * pi * drz)[..., None] * ep
    return Mo, Me, No, Ne


def impedance_coefficients(x: float, Z: complex, nmax=None):
    """a_n, b_n of a sphere whose surface obeys n x E = Z n x (n x H) (eq. 2.24,
    Z relative to the vacuum impedance).  They are the dielectric coefficients
    above in the limit of a large lossy index m = 1/Z, where
    psi_n'(mx)/psi_n(mx) -> -i:
        a_n = (psi_n'(x) + i Z psi_n(x)) / (xi_n'(x) + i Z xi_n(x)),
        b_n = (psi_n(x) - i Z psi_n'(x)) / (xi_n(x) - i Z xi_n'(x))."""
    if nmax is None:
        nmax = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    n = np.arange(1, nmax + 1)
    jx, djx = _jn(n, x), _jn(n, x, True)
    hx, dhx = _hn(n, x), _hn(n, x, True)
    psi, dpsi = x * jx, jx + x * djx
    xi, dxi = x * hx, hx + x * dhx
    Z = complex(Z)
    a = (dpsi + 1j * Z * psi) / (dxi + 1j * Z * xi)
    b = (psi - 1j * Z * dpsi) / (xi - 1j * Z * dxi)
    return n, a, b


def impedance_fields(points, k: float, a: float, Z: complex, nmax=None):
    """(E, curl E) of the total host field around the impedance sphere."""
    n, an, bn = impedance_coefficients(k * a, Z, nmax)
    return fields(points, k, a, None, "outside", coeffs=(n, an, bn))


def fields(points, k: float, a: float, eps: complex, region="outside", nmax=None, coeffs=None):
    """(E, curl E) at points for E_inc = x^ exp(i k z).  region 'outside'
    gives the total host field E_inc + E_sca, 'scattered' E_sca alone, 'inside'
    the interior field.
    coeffs = (n, a_n, b_n) replaces the dielectric scattering coefficients."""
    p = np.asarray(points, dtype=np.float64)
    r = np.linalg.norm(p, axis=1)
    theta = np.arccos(np.clip(p[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(p[:, 1], p[:, 0])
    if coeffs is not None:
        n, an, bn = coeffs
        m = None
    else:
        m = np.sqrt(complex(eps))
        n, an, bn, cn, dn = coefficients(k * a, m, nmax)
    En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
    if region == "scattered":
        Mo3, Me3, No3, Ne3 = _vsh(n, k, r, theta, phi, 3)
        E = np.einsum("n,npd->pd", En * 1j * an, Ne3) - np.einsum("n,npd->pd", En * bn, Mo3)
        C = k * (np.einsum("n,npd->pd", En * 1j * an, Me3) - np.einsum("n,npd->pd", En * bn, No3))
    elif region == "outside":
        Mo1, Me1, No1, Ne1 = _vsh(n, k, r, theta, phi, 1)
        Mo3, Me3, No3, Ne3 = _vsh(n, k, r, theta, phi, 3)
        E = np.einsum("n,npd->pd", En, Mo1 - 1j * Ne1) + np.einsum("n,npd->pd", En * 1j * an, Ne3) \
            - np.einsum("n,npd->pd", En * bn, Mo3)
        C = k * (np.einsum("n,npd->pd", En, No1 - 1j * Me1) + np.einsum("n,npd->pd", En * 1j * an, Me3)
                 - np.einsum("n,npd->pd", En * bn, No3))
    else:
        k1 = m * k
        Mo1, Me1, No1, Ne1 = _vsh(n, k1, r, theta, phi, 1)
        E = np.einsum("n,npd->pd", En * cn, Mo1) - np.einsum("n,npd->pd", En * 1j * dn, Ne1)
        C = k1 * (np.einsum("n,npd->pd", En * cn, No1) - np.einsum("n,npd->pd", En * 1j * dn, Me1))
    return E, C


def efficiencies(x: float, m: complex, nmax=None):
    """Q_ext and Q_sca (B&H eqs. 4.61-4.62)."""
    n, a, b, _, _ = coefficients(x, m, nmax)
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (abs(a) ** 2 + abs(b) ** 2))
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    return qext, qsca


def radiation_pressure(x: float, m: complex, nmax=None, coeffs=None):
    """Q_pr = Q_ext - g Q_sca, with the asymmetry term of Bohren & Huffman's Mie theory (Sec. 4.5)
    g Q_sca = 4/x^2 [ sum_n n(n+2)/(n+1) Re(a_n a_{n+1}^* + b_n b_{n+1}^*)
                      + sum_n (2n+1)/(n(n+1)) Re(a_n b_n^*) ].
    The time-averaged force on the sphere in a plane wave of irradiance I is
    Q_pr pi a^2 I / c along the propagation direction."""
    if coeffs is None:
        n, a, b, _, _ = coefficients(x, m, nmax)
    else:
        n, a, b = coeffs
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (abs(a) ** 2 + abs(b) ** 2))
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    nn = n[:-1]
    gq = 4.0 / x ** 2 * (np.sum(nn * (nn + 2) / (nn + 1) * np.real(a[:-1] * np.conj(a[1:]) + b[:-1] * np.conj(b[1:])))
                         + np.sum((2 * n + 1) / (n * (n + 1)) * np.real(a * np.conj(b))))
    return qext - gq


def surface_unknowns(nodes, k: float, a: float, eps: complex, nmax=None):
    """Mie (Phi, Psi) at the radially projected nodes a s/|s|, with Psi formed with
    the mesh's face normal: Psi = n x curl E_0.  Returns c128[n,6]."""
    s = nodes["points"]
    proj = a * s / np.linalg.norm(s, axis=1, keepdims=True)
    E, C = fields(proj, k, a, eps, "outside", nmax)
    psi = np.cross(nodes["normals"], C)
    return np.concatenate([E, psi], axis=1)
