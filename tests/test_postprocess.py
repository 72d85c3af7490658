"""Pins of the cross-section and multipole post-processing against Mie (CPU only)."""

import numpy as np

from oracle import mie
from paper_1211_7177_amd import postprocess as pp


def _mie_far(eps, dirs, r=2e4):
    """r e^{-ikr} E_sca(r rhat) of the Mie sphere (k a = 1) at large r (the
    oracle's numerical vector spherical harmonics, scattered part only)."""
    E, _ = mie.fields(r * dirs, 1.0, 1.0, eps, "scattered")
    return E * r * np.exp(-1j * r)


def test_projection_recovers_known_coefficients():
    """A far field built from chosen a_n, b_n with the far-zone forms of N_e1n and
    M_o1n is projected back to the same coefficients."""
    rng = np.random.default_rng(3)
    nmax = 5
    a = rng.standard_normal(nmax) + 1j * rng.standard_normal(nmax)
    b = rng.standard_normal(nmax) + 1j * rng.standard_normal(nmax)
    dirs, wts = pp.sphere_quadrature(24, 48)
    ct = dirs[:, 2]
    st = np.sqrt(1 - ct ** 2)
    ph = np.arctan2(dirs[:, 1], dirs[:, 0])
    et = np.stack([ct * np.cos(ph), ct * np.sin(ph), -st], -1)
    ep = np.stack([-np.sin(ph), np.cos(ph), 0 * ph], -1)
    pi, tau = pp._pi_tau(nmax, ct)
    F = np.zeros((len(ct), 3), complex)
    k = 1.7
    for i, n in enumerate(range(1, nmax + 1)):
        En = 1j ** n * (2 * n + 1) / (n * (n + 1))
        nn = np.cos(ph)[:, None] * tau[i][:, None] * et - np.sin(ph)[:, None] * pi[i][:, None] * ep
        mm = np.cos(ph)[:, None] * pi[i][:, None] * et - np.sin(ph)[:, None] * tau[i][:, None] * ep
        F += En * (1j * a[i] * (-1j) ** n * nn - b[i] * (-1j) ** (n + 1) * mm) / k
    ra, rb = pp.multipole_coefficients(F, dirs, wts, k, nmax)
    assert np.abs(ra - a).max() <= 1e-12 and np.abs(rb - b).max() <= 1e-12


def test_mie_far_field_gives_mie_coefficients_and_cross_sections():
    for eps in (2.25, 2.25 + 0.5j):
        dirs, wts = pp.sphere_quadrature(24, 48)
        F = _mie_far(eps, dirs)
        n, a, b, _, _ = mie.coefficients(1.0, np.sqrt(eps), 4)
        ra, rb = pp.multipole_coefficients(F, dirs, wts, 1.0, 4)
        assert np.abs(ra - a).max() <= 1e-3 * np.abs(a).max() and np.abs(rb - b).max() <= 1e-3 * np.abs(a).max()
        qext, qsca = mie.efficiencies(1.0, np.sqrt(eps))
        csca = pp.scattering_from_far(F, wts, [1.0, 0, 0])
        cext = pp.extinction_from_forward(_mie_far(eps, np.array([[0.0, 0.0, 1.0]]))[0], [1.0, 0, 0], 1.0)
        assert abs(csca - qsca * np.pi) <= 1e-3 * qsca * np.pi
        assert abs(cext - qext * np.pi) <= 1e-3 * qext * np.pi


def test_stress_tensor_force_of_mie_fields():
    """The package's stress-tensor integral of the Mie total fields on the sphere
    r = 2a equals Q_pr pi a^2 / 2 (B&H Sec. 4.5) and the oracle's own integral of
    the same samples (two implementations written apart)."""
    from oracle import fields as of
    dirs, wts = pp.sphere_quadrature(32, 64)
    for eps in (2.25, 2.25 + 0.5j):
        E, C = mie.fields(2.0 * dirs, 1.0, 1.0, eps, "outside")
        F = pp.stress_tensor_force(E, C, 1.0, dirs, 4.0 * wts)
        ref = mie.radiation_pressure(1.0, np.sqrt(eps)) * np.pi / 2.0
        assert abs(F[2] - ref) <= 1e-9 * ref and np.abs(F[:2]).max() <= 1e-12
        assert np.abs(F - of.stress_force(E, C, 1.0, dirs, 4.0 * wts)).max() <= 1e-13 * ref


def test_differential_and_radar_cross_sections_of_mie_far_field():
    """On the Mie far field of an x-polarised wave along +z: dC/dOmega integrates
    to C_sca, equals (|S_2|^2 cos^2 phi + |S_1|^2 sin^2 phi) / k^2 with the
    amplitude functions S_1, S_2 of the Mie coefficients (B&H Sec. 4.4), and the
    radar cross section is 4 pi times it."""
    eps = 2.25 + 0.5j
    dirs, wts = pp.sphere_quadrature(32, 64)
    F = _mie_far(eps, dirs)
    dsc = pp.differential_cross_section(F, [1.0, 0, 0])
    qext, qsca = mie.efficiencies(1.0, np.sqrt(eps))
    assert abs(np.sum(wts * dsc) - qsca * np.pi) <= 1e-3 * qsca * np.pi
    n, a, b, _, _ = mie.coefficients(1.0, np.sqrt(eps))
    mu = np.clip(dirs[:, 2], -1, 1)
    ph = np.arctan2(dirs[:, 1], dirs[:, 0])
    pi_n = np.zeros((len(n), len(mu)))
    tau_n = np.zeros_like(pi_n)
    pi_n[0], tau_n[0] = 1.0, mu
    for i in range(1, len(n)):
        nn = i + 1
        pi_n[i] = (2 * nn - 1) / (nn - 1) * mu * pi_n[i - 1] - (nn / (nn - 1) * pi_n[i - 2] if i >= 2 else 0.0)
        tau_n[i] = nn * mu * pi_n[i] - (nn + 1) * pi_n[i - 1]
    c = (2 * n + 1) / (n * (n + 1))
    S1 = np.sum(c[:, None] * (a[:, None] * pi_n + b[:, None] * tau_n), axis=0)
    S2 = np.sum(c[:, None] * (a[:, None] * tau_n + b[:, None] * pi_n), axis=0)
    ref = (np.abs(S2) ** 2 * np.cos(ph) ** 2 + np.abs(S1) ** 2 * np.sin(ph) ** 2) / 1.0
    assert np.max(np.abs(dsc - ref)) <= 1e-3 * np.max(ref)
    assert np.allclose(pp.radar_cross_section(F, [1.0, 0, 0]), 4 * np.pi * dsc)
