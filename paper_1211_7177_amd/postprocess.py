"""Cross sections and far-field multipole coefficients from a solved problem.

With the far-field amplitude F of `bem_field` (E_sca ~ e^{ik0 r} / r F(rhat)),
for an incident wave p exp(i k0 d . r):

* C_sca = oint |F|^2 dOmega / |p|^2 (eq. 4.2 taken on a sphere in the far zone),
* C_ext = (4 pi / k0) Im(conj(p) . F(d)) / |p|^2 (the optical theorem),
* C_abs = C_ext - C_sca (eq. 4.2's C_ext = C_abs + C_sca).

The time-averaged optical force on the scatterers follows from the total host
fields on a closed sphere around them: F = oint <T> . n dA with the Maxwell
stress tensor <T> = 1/2 Re[ E E^* + H H^* - 1/2 (|E|^2 + |H|^2) I ] (eps0 = mu0 = 1)
and H = curl E / (i k0), where E_sca and curl E_sca come from `bem_field`.

The expansion of eq. 4.4, E_sca = sum_n (a_n N_n + b_n M_n), is read off the
far field for an x-polarised wave along +z (the convention of the Mie
coefficients): far away r e^{-ikr} N_e1n -> (-i)^n n_n / k and
r e^{-ikr} M_o1n -> (-i)^{n+1} m_n / k with the angular functions
n_n = cos(phi) tau_n theta^ - sin(phi) pi_n phi^ and
m_n = cos(phi) pi_n theta^ - sin(phi) tau_n phi^, which are orthogonal over the
sphere with squared norm 2 pi n^2 (n+1)^2 / (2n+1).  Writing E_sca = sum_n E_n
(i a_n N_e1n - b_n M_o1n), E_n = i^n (2n+1) / (n (n+1)), the projections of
eq. 4.5 give a_n and b_n (the weighted form of the eq. 4.5 coefficients).
"""

import numpy as np


def sphere_quadrature(nt=32, nph=64):
    """Gauss-Legendre in cos(theta) times the uniform rule in phi: directions f64[m,3], weights f64[m]."""
    x, w = np.polynomial.legendre.leggauss(nt)
    ph = np.linspace(0.0, 2.0 * np.pi, nph, endpoint=False)
    ct, pp = np.meshgrid(x, ph, indexing="ij")
    st = np.sqrt(1.0 - ct ** 2)
    dirs = np.stack([st * np.cos(pp), st * np.sin(pp), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(nph, 2.0 * np.pi / nph)[None, :]).reshape(-1)
    return dirs, wts


def _far(problem, x, dirs):
    return problem.field(x, dirs, far=True).cpu().numpy()


def scattering_from_far(F, wts, pol):
    """C_sca from far-field samples F c128[m,3] with quadrature weights wts."""
    e0 = float(np.sum(np.abs(np.asarray(pol)) ** 2))
    return float(np.sum(wts * np.sum(np.abs(F) ** 2, axis=1))) / e0


def extinction_from_forward(F_fwd, pol, k0):
    """C_ext by the optical theorem from the far field F c128[3] in the incident direction."""
    p = np.asarray(pol, dtype=np.complex128)
    e0 = float(np.sum(np.abs(p) ** 2))
    return float(4.0 * np.pi / np.real(k0) * np.imag(np.sum(np.conj(p) * F_fwd))) / e0


def differential_cross_section(F, pol):
    """dC_sca/dOmega = |F(rhat)|^2 / |E0|^2 from far-field samples F c128[m,3]
    (the quantity plotted against angle in the paper's dimer comparison)."""
    e0 = float(np.sum(np.abs(np.asarray(pol)) ** 2))
    return np.sum(np.abs(np.asarray(F)) ** 2, axis=-1) / e0


def radar_cross_section(F, pol):
    """Bistatic radar cross section sigma = 4 pi |F(rhat)|^2 / |E0|^2 (monostatic
    when rhat = -d)."""
    return 4.0 * np.pi * differential_cross_section(F, pol)


def cross_sections(problem, x, d, pol, k0, nt=32, nph=64):
    """(C_ext, C_sca, C_abs) of the solution x [1, n, nu] for the wave pol exp(i k0 d . r)."""
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    dirs, wts = sphere_quadrature(nt, nph)
    F = _far(problem, x, np.vstack([dirs, d[None, :]]))[0]
    csca = scattering_from_far(F[:-1], wts, pol)
    cext = extinction_from_forward(F[-1], pol, k0)
    return cext, csca, cext - csca


def stress_tensor_force(E, curlE, k0, normals, weights):
    """oint <T> . n dA from total fields E, curl E c128[m,3] on a closed surface in
    the host medium with outward normals f64[m,3] and area weights f64[m]."""
    H = np.asarray(curlE) / (1j * k0)
    E = np.asarray(E)
    nrm = np.asarray(normals, dtype=np.float64)
    sE = np.einsum("md,md->m", np.conj(E), nrm)
    sH = np.einsum("md,md->m", np.conj(H), nrm)
    u = 0.5 * (np.einsum("md,md->m", E, np.conj(E)).real + np.einsum("md,md->m", H, np.conj(H)).real)
    t = 0.5 * np.real(E * sE[:, None] + H * sH[:, None] - u[:, None] * nrm)
    return np.einsum("m,md->d", np.asarray(weights, dtype=np.float64), t)


def optical_force(problem, x, d, pol, k0, radius, center=(0.0, 0.0, 0.0), nt=32, nph=64):
    """Time-averaged force f64[nrhs, 3] on the scatterers inside the sphere of
    the given radius and center, for the solutions x [nrhs, n, nu] of the plane
    waves pol exp(i k0 d . r) (d, pol: [3] or [nrhs, 3]).  The sphere lies in
    the host medium: it encloses the scatterers whose force is wanted, and no
    surface crosses it (around one scatterer of several, it gives the force on
    that one).  The fields are the discrete representation's, whose accuracy
    falls within about a mesh edge of a surface; keep the sphere farther off."""
    dirs, wts = sphere_quadrature(nt, nph)
    pts = np.asarray(center, dtype=np.float64)[None, :] + radius * dirs
    Es = problem.field(x, pts).cpu().numpy()
    Cs = problem.field(x, pts, curl=True).cpu().numpy()
    nr = Es.shape[0]
    D = np.broadcast_to(np.atleast_2d(np.asarray(d, dtype=np.float64)), (nr, 3))
    P = np.broadcast_to(np.atleast_2d(np.asarray(pol, dtype=np.complex128)), (nr, 3))
    out = np.zeros((nr, 3))
    for r in range(nr):
        dr = D[r] / np.linalg.norm(D[r])
        Ei = np.exp(1j * k0 * (pts @ dr))[:, None] * P[r][None, :]
        Ci = 1j * k0 * np.cross(np.broadcast_to(dr, Ei.shape), Ei)
        out[r] = stress_tensor_force(Ei + Es[r], Ci + Cs[r], k0, dirs, wts * radius ** 2)
    return out


def _pi_tau(nmax, mu):
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros((nmax + 1,) + mu.shape)
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def multipole_coefficients(F, dirs, wts, k0, nmax):
    """a_n, b_n (n = 1..nmax) of an x-polarised incidence along +z from far-field
    samples F c128[m,3] at directions dirs with quadrature weights wts."""
    ct = np.clip(dirs[:, 2], -1.0, 1.0)
    st = np.sqrt(np.maximum(1.0 - ct ** 2, 0.0))
    ph = np.arctan2(dirs[:, 1], dirs[:, 0])
    et = np.stack([ct * np.cos(ph), ct * np.sin(ph), -st], -1)
    ep = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], -1)
    Ft = np.sum(F * et, axis=1)
    Fp = np.sum(F * ep, axis=1)
    pi, tau = _pi_tau(nmax, ct)
    n = np.arange(1, nmax + 1)
    En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
    norm = 2.0 * np.pi * n ** 2 * (n + 1) ** 2 / (2 * n + 1)
    cp, sp = np.cos(ph), np.sin(ph)
    pn = np.sum(wts * (cp * tau * Ft - sp * pi * Fp), axis=1) / norm          # <n_n, F> / |n_n|^2
    pm = np.sum(wts * (cp * pi * Ft - sp * tau * Fp), axis=1) / norm          # <m_n, F> / |m_n|^2
    k = np.real(k0)
    a = pn * k / (En * 1j * (-1j) ** n)
    b = -pm * k / (En * (-1j) ** (n + 1))
    return a, b
