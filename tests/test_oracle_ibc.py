"""Pins of the impedance-boundary-condition oracle (eqs. 2.24-2.25) and its Mie solution (CPU only)."""

import numpy as np
import pytest

from oracle import mie
from oracle.bem import BemProblem, IbcProblem
from oracle.gmres import gmres_solve
from synthetic import complex_normal, icosphere, nystrom3


def test_impedance_mie_satisfies_the_boundary_condition():
    """n x E = Z n x (n x H) on r = a for the total field, H = curl E / (i k) (eq. 2.24);
    Z = 0 gives a perfect conductor (n x E = 0)."""
    rng = np.random.default_rng(1)
    v = rng.standard_normal((300, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for k, Z in ((1.0, 0.3 - 0.2j), (2.5, 0.05 + 0.05j)):
        E, C = mie.impedance_fields(v, k, 1.0, Z)
        lhs = np.cross(v, E)
        rhs = Z * np.cross(v, np.cross(v, C / (1j * k)))
        assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()
    E, _ = mie.impedance_fields(v, 1.0, 1.0, 0.0)
    assert np.abs(np.cross(v, E)).max() <= 1e-12 * np.abs(E).max()


def test_impedance_coefficients_are_the_large_index_limit():
    """The dielectric Mie coefficients with m = s (1 + i) approach the impedance ones
    with Z = 1/m, the gap falling like 1/|m|^2."""
    gaps = []
    for s in (10, 30, 100):
        m = s * (1 + 1j)
        _, a, b, _, _ = mie.coefficients(1.0, m)
        _, ai, bi = mie.impedance_coefficients(1.0, 1.0 / m)
        gaps.append(max(np.abs(a - ai).max(), np.abs(b - bi).max()))
    assert gaps[0] < 1e-3 and gaps[1] < gaps[0] / 5 and gaps[2] < gaps[1] / 5


def test_ibc_rows_are_the_host_rows_with_psi_substituted(sphere_nodes):
    """A_ibc Phi equals rows 0:3 of the dielectric system at Psi = -c n x (n x Phi)."""
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    Z = 0.2 - 0.1j
    ib = IbcProblem(q, 1.3, Z)
    bem = BemProblem(q, 1.3, 2.25)
    phi = complex_normal((n, 3), 121)
    psi = -ib.c * ib.nnx(phi)
    ref = bem.apply(np.concatenate([phi, psi], axis=1))[:, 0:3]
    assert np.abs(ib.apply(phi) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_ibc_adjoint_identity(sphere_nodes):
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    ib = IbcProblem(q, 1.3, 0.2 - 0.1j)
    x, v = complex_normal((n, 3), 122), complex_normal((n, 3), 123)
    lhs = np.sum(np.conj(v) * ib.apply(x))
    assert abs(lhs - np.sum(np.conj(ib.apply_adjoint(v)) * x)) <= 1e-12 * abs(lhs)
    P, PH = ib.block_preconditioner(), ib.block_preconditioner(adjoint=True)
    assert abs(np.sum(np.conj(v) * P(x)) - np.sum(np.conj(PH(v)) * x)) <= 1e-12 * abs(np.sum(np.conj(v) * P(x)))


def test_ibc_system_against_impedance_mie():
    """The exact impedance-sphere field (k0 a = 1, Z = 0.2 - 0.1i) leaves a residual
    in the discrete system that shrinks under refinement (the point-rule
    consistency error), while a flipped sign of c or a conjugated Z leaves O(1);
    the solved field approaches the Mie field."""
    Z = 0.2 - 0.1j
    res, errs = [], []
    for nu in (2, 4):
        q = nystrom3(icosphere(nu))
        s = q["points"]
        E, _ = mie.impedance_fields(s / np.linalg.norm(s, axis=1, keepdims=True), 1.0, 1.0, Z)
        ib = IbcProblem(q, 1.0, Z)
        b = ib.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])
        res.append(np.linalg.norm(ib.apply(E) - b) / np.linalg.norm(b))
        x, info = gmres_solve(ib.apply, b, ib.block_preconditioner(), tol=1e-10, restart=200)
        errs.append(np.linalg.norm(x - E) / np.linalg.norm(E))
        if nu == 4:
            for bad in (IbcProblem(q, 1.0, np.conj(Z)), IbcProblem(q, 1.0, -Z)):
                assert np.linalg.norm(bad.apply(E) - b) / np.linalg.norm(b) > 0.5
    print(res, errs)
    assert res[1] < 0.6 * res[0] and res[1] < 0.1
    assert errs[1] < 0.6 * errs[0] and errs[1] < 0.12
