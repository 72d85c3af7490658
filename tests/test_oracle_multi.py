"""Pins of the oracle's several-scatterer system (CPU only)."""

import numpy as np

from oracle.bem import BemProblem, MultiBemProblem
from oracle.gmres import gmres_solve
from synthetic import complex_normal, icosphere, nystrom3, union


def _two_spheres(d, nu=2):
    m, treg = union([icosphere(nu), icosphere(nu, 0.7)], [[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    q = nystrom3(m)
    return q, treg[q["point_tri"]]


def test_one_scatterer_is_the_single_system(sphere_nodes):
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    m = MultiBemProblem(q, np.zeros(n, int), 1.0, [2.25 + 0.3j])
    b = BemProblem(q, 1.0, 2.25 + 0.3j)
    x = complex_normal((n, 6), 151)
    assert np.abs(m.apply(x) - b.apply(x)).max() <= 1e-13 * np.abs(b.apply(x)).max()
    assert np.abs(m.precond_blocks() - b.precond_blocks()).max() <= 1e-13


def test_two_scatterers_adjoint_identity():
    q, reg = _two_spheres(2.5)
    n = q["points"].shape[0]
    m = MultiBemProblem(q, reg, 1.0, [2.25, -15 + 1j])
    x, v = complex_normal((n, 6), 152), complex_normal((n, 6), 153)
    lhs = np.sum(np.conj(v) * m.apply(x))
    assert abs(lhs - np.sum(np.conj(m.apply_adjoint(v)) * x)) <= 1e-12 * abs(lhs)


def test_far_apart_scatterers_decouple():
    """With the second sphere moved away, the first sphere's solution approaches
    its single-scatterer solution, the coupling falling roughly like 1/d."""
    q1 = nystrom3(icosphere(2))
    b1 = BemProblem(q1, 1.0, 2.25)
    rhs1 = b1.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])
    x1, _ = gmres_solve(b1.apply, rhs1, b1.block_preconditioner(), tol=1e-10, restart=200)
    gaps = []
    for d in (4.0, 16.0, 64.0):
        q, reg = _two_spheres(d)
        m = MultiBemProblem(q, reg, 1.0, [2.25, 2.25 + 0.2j])
        rhs = m.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])
        x, _ = gmres_solve(m.apply, rhs, m.block_preconditioner(), tol=1e-10, restart=200)
        gaps.append(np.linalg.norm(x[reg == 0] - x1) / np.linalg.norm(x1))
    print(gaps)
    assert gaps[1] < 0.5 * gaps[0] and gaps[2] < 0.5 * gaps[1]
