"""Pins of the oracle's off-surface field, interior field and far-field formulas (CPU only)."""

import numpy as np
import pytest

from oracle import fields, mie
from synthetic import icosphere, nystrom3

TH = np.linspace(0.2, np.pi - 0.2, 12)


def _sphere_quadrature(nt=24, nph=48):
    x, w = np.polynomial.legendre.leggauss(nt)
    ph = np.linspace(0, 2 * np.pi, nph, endpoint=False)
    ct, pp = np.meshgrid(x, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    D = np.stack([st * np.cos(pp), st * np.sin(pp), ct], -1).reshape(-1, 3)
    W = (w[:, None] * np.full(nph, 2 * np.pi / nph)[None, :]).reshape(-1)
    return D, W


@pytest.mark.parametrize("eps", [2.25, 2.25 + 0.5j])
def test_representation_of_exact_surface_fields_reproduces_mie(eps):
    """The exact Mie surface fields, put through the host and interior
    representations and the far-field sum, give Mie's scattered field at
    r = 2a, its interior field at r = a/2 and its C_sca, converging under refinement."""
    out = 2.0 * np.stack([np.sin(TH), 0 * TH, np.cos(TH)], 1)
    inn = 0.5 * np.stack([0.7 * np.sin(TH), 0.7 * np.sin(TH), np.cos(TH)], 1)
    Em, _ = mie.fields(out, 1.0, 1.0, eps, "outside")
    Esm = Em - np.exp(1j * out[:, 2])[:, None] * np.array([1.0, 0, 0])
    Eim, _ = mie.fields(inn, 1.0, 1.0, eps, "inside")
    D, W = _sphere_quadrature()
    cref = mie.efficiencies(1.0, np.sqrt(eps))[1] * np.pi
    e_out, e_in, e_c = [], [], []
    for nu in (2, 4):
        q = nystrom3(icosphere(nu))
        xm = mie.surface_unknowns(q, 1.0, 1.0, eps)
        e_out.append(np.linalg.norm(fields.scattered_field(q, 1.0, xm, out) - Esm) / np.linalg.norm(Esm))
        e_in.append(np.linalg.norm(fields.interior_field(q, np.sqrt(eps), eps, 1.0, xm, inn) - Eim)
                    / np.linalg.norm(Eim))
        C = np.sum(W * np.sum(np.abs(fields.far_field(q, 1.0, xm, D)) ** 2, 1))
        e_c.append(abs(C - cref) / cref)
    print(e_out, e_in, e_c)
    assert e_out[1] < 0.35 * e_out[0] and e_out[1] < 0.03
    assert e_in[1] < 0.35 * e_in[0] and e_in[1] < 0.02
    assert e_c[1] < 0.35 * e_c[0] and e_c[1] < 0.03


def test_far_field_is_the_limit_of_the_near_sum(sphere_nodes):
    """r e^{-ikr} E_sca(r rhat) -> F(rhat) as r grows (error ~ 1/r)."""
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    rng = np.random.default_rng(5)
    x = (rng.standard_normal((n, 6)) + 1j * rng.standard_normal((n, 6))) / np.sqrt(2)
    d = rng.standard_normal((6, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    F = fields.far_field(q, 1.3, x, d)
    gaps = []
    for r in (1e2, 1e3, 1e4):
        E = fields.scattered_field(q, 1.3, x, r * d) * r * np.exp(-1.3j * r)
        gaps.append(np.linalg.norm(E - F) / np.linalg.norm(F))
    assert gaps[1] < 0.2 * gaps[0] and gaps[2] < 0.2 * gaps[1] and gaps[2] < 1e-3


def test_scattered_curl_matches_finite_differences_of_the_field(sphere_nodes):
    """curl E_sca from the closed-form Hessian sum equals the central-difference
    curl of the scattered-field sum (step 1e-5, error ~ h^2)."""
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    rng = np.random.default_rng(11)
    x = (rng.standard_normal((n, 6)) + 1j * rng.standard_normal((n, 6))) / np.sqrt(2)
    t = 1.6 * rng.standard_normal((5, 3))
    t *= (1.5 + rng.random((5, 1))) / np.linalg.norm(t, axis=1, keepdims=True)
    k0, h = 1.3 + 0.05j, 1e-5
    J = np.zeros((5, 3, 3), dtype=np.complex128)                   # J[:, i, j] = dE_i / dx_j
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, :, j] = (fields.scattered_field(q, k0, x, t + e) - fields.scattered_field(q, k0, x, t - e)) / (2 * h)
    fd = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], 1)
    cu = fields.scattered_curl(q, k0, x, t)
    assert np.linalg.norm(cu - fd) / np.linalg.norm(cu) < 1e-8


def test_scattered_curl_of_exact_surface_fields_reproduces_mie():
    """The exact Mie surface fields give Mie's curl E_sca at r = 2a, converging
    under refinement."""
    eps = 2.25 + 0.5j
    out = 2.0 * np.stack([np.sin(TH), 0.3 * np.sin(TH), np.cos(TH)], 1)
    _, Cm = mie.fields(out, 1.0, 1.0, eps, "scattered")
    err = []
    for nu in (2, 4):
        q = nystrom3(icosphere(nu))
        xm = mie.surface_unknowns(q, 1.0, 1.0, eps)
        err.append(np.linalg.norm(fields.scattered_curl(q, 1.0, xm, out) - Cm) / np.linalg.norm(Cm))
    print(err)
    assert err[1] < 0.35 * err[0] and err[1] < 0.03


@pytest.mark.parametrize("eps", [2.25, 2.25 + 0.5j, 4.0 + 0.1j])
def test_stress_tensor_force_equals_mie_radiation_pressure(eps):
    """The Maxwell-stress integral of the Mie total fields over spheres of radius
    1.5a and 3a equals Q_pr pi a^2 I (B&H Sec. 4.5 for g Q_sca, I = 1/2 for a unit
    amplitude): two independent routes to the same force; the transverse
    components vanish."""
    D, W = _sphere_quadrature(40, 80)
    ref = mie.radiation_pressure(1.0, np.sqrt(eps)) * np.pi / 2.0
    for R in (1.5, 3.0):
        E, C = mie.fields(R * D, 1.0, 1.0, eps, "outside")
        F = fields.stress_force(E, C, 1.0, D, W * R * R)
        assert abs(F[2] - ref) <= 1e-9 * ref
        assert np.max(np.abs(F[:2])) <= 1e-12


def test_radiation_pressure_reduces_to_extinction_without_asymmetry():
    """A lossless small sphere scatters almost symmetrically (g -> 0): Q_pr -> Q_ext,
    with g Q_sca of order x^2 Q_sca (the dipole-quadrupole cross terms)."""
    qext, qsca = mie.efficiencies(0.05, 1.5)
    qpr = mie.radiation_pressure(0.05, 1.5)
    assert abs(qpr - qext) <= 1e-2 * qsca
    assert abs(qpr - qext) > 0.0
