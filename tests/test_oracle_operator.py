"""Pins of the oracle's direct operator, BEM system, fGMRES and Mie series (CPU only)."""

import numpy as np
import pytest

from oracle import mie
from oracle.bem import BemProblem
from oracle.corrections import self_blocks
from oracle.direct import apply_corrections, point_sum
from oracle.gmres import gmres_solve
from oracle.native import point_sum_c
from synthetic import complex_normal, icosphere, nystrom3, seed_for, torus


def _op(q, k, a, b):
    blk = self_blocks(q["points"], q["normals"], q["point_tri"], q["tri_vertices"], k)
    return (point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b)
            + apply_corrections(q["normals"], q["point_tri"], blk, a, b))


def test_c_and_numpy_direct_sums_agree(sphere_nodes):
    q = sphere_nodes[4]
    n = q["points"].shape[0]
    a = complex_normal((2, n, 3), 11)
    b = complex_normal((2, n, 3), 12)
    for k in (1.0, 0.5 + 15.5j):
        y1 = point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b)
        y2 = point_sum(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b)
        assert np.abs(y1 - y2).max() <= 1e-13 * np.abs(y2).max()


def _transposed_sum(q, k, y):
    """Independent transposed kernel: (Op^T y)_beta = w_beta sum_alpha [n_beta^T ... ] written
    per source: a-part  = w [ n (G.y)^T ... ] rearranged as  w [ G (n.y) - (n.G) y - n (G.y) ]
    and b-part = w sum_alpha g y_alpha."""
    pts, nrm, w, tri = q["points"], q["normals"], q["weights"], q["point_tri"]
    n = pts.shape[0]
    abar = np.zeros((n, 3), complex)
    bbar = np.zeros((n, 3), complex)
    for be in range(n):
        d = pts[be][None, :] - pts           # s_beta - s_alpha for every target alpha
        R = np.linalg.norm(d, axis=1)
        m = tri != tri[be]
        e = np.exp(1j * k * R[m])
        g = e / (4 * np.pi * R[m])
        f = (1j * k * R[m] - 1) * e / (4 * np.pi * R[m] ** 3)
        G = f[:, None] * d[m]
        Y = y[m]
        nb = nrm[be]
        # y^T [n (G.a) - (n.G) a - G (n.a)] = (y.n)(G.a) - (n.G)(y.a) - (y.G)(n.a)
        abar[be] = w[be] * np.sum((Y @ nb)[:, None] * G - (G @ nb)[:, None] * Y
                                  - np.sum(Y * G, 1)[:, None] * nb[None, :], 0)
        bbar[be] = w[be] * np.sum(g[:, None] * Y, 0)
    return abar, bbar


@pytest.mark.parametrize("k", [1.3, 2 + 0.7j])
def test_point_sum_bilinear_identity_with_transposed_kernel(sphere_nodes, k):
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    a = complex_normal((n, 3), 1)
    b = complex_normal((n, 3), 2)
    y = complex_normal((n, 3), 3)
    Op = point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b)
    abar, bbar = _transposed_sum(q, k, y)
    lhs = np.sum(y * Op)
    rhs = np.sum(abar * a) + np.sum(bbar * b)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _plane_wave(q, k):
    s, nrm = q["points"], q["normals"]
    d = np.array([0.3, 0.4, np.sqrt(0.75)])
    p = np.cross(d, [1.0, 0, 0])
    p /= np.linalg.norm(p)
    e = np.exp(1j * k * (s @ d))
    E = e[:, None] * p
    curl = 1j * k * np.cross(d, p)[None] * e[:, None]
    return E, np.cross(nrm, curl)


def _dipole(q, k):
    """Field of a point dipole inside the surface and n x curl of it (curl by central differences)."""
    x0 = np.array([0.1, -0.2, 0.15])
    pd = np.array([0.2, 0.5, -0.3])

    def Ef(P):
        r = P - x0
        R = np.linalg.norm(r, axis=1)
        rh = r / R[:, None]
        g = np.exp(1j * k * R) / (4 * np.pi * R)
        return ((k ** 2 * g)[:, None] * np.cross(np.cross(rh, pd), rh)
                + (g * (1 / R ** 2 - 1j * k / R))[:, None] * (3 * rh * (rh @ pd)[:, None] - pd))

    s = q["points"]
    h = 1e-5
    J = np.zeros((len(s), 3, 3), complex)
    for dd in range(3):
        e = np.zeros(3)
        e[dd] = h
        J[:, :, dd] = (Ef(s + e) - Ef(s - e)) / (2 * h)
    curl = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], 1)
    return Ef(s), np.cross(q["normals"], curl)


@pytest.mark.parametrize("k", [1.5, 2 + 1.5j])
def test_interior_and_exterior_efie_identities_converge(sphere_nodes, k):
    """Eq. 2.5 for fields with no sources in the domain: a plane wave seen from the
    interior gives Op(E, -n x curl E) = E/2; a dipole field seen from the exterior
    (normal flipped) gives Op(E, -n x curl E) = -E/2.  The discrete residual must
    shrink under refinement (nu = 2, 4, 8)."""
    errs_in, errs_out = [], []
    for nu in (2, 4, 8):
        q = sphere_nodes[nu]
        E, Psi = _plane_wave(q, k)
        y = _op(q, k, E, -Psi)
        errs_in.append(np.linalg.norm(y - 0.5 * E) / np.linalg.norm(E))
        E, Psi = _dipole(q, k)
        y = _op(q, k, E, -Psi)
        errs_out.append(np.linalg.norm(y + 0.5 * E) / np.linalg.norm(E))
    assert errs_in[0] > errs_in[1] > errs_in[2] and errs_in[2] < 0.03
    assert errs_out[0] > errs_out[1] > errs_out[2] and errs_out[2] < 0.05
    # a sign slip in any dyad term or in the jump term gives O(1) residuals
    E, Psi = _plane_wave(sphere_nodes[8], k)
    assert np.linalg.norm(_op(sphere_nodes[8], k, E, Psi) - 0.5 * E) / np.linalg.norm(E) > 0.3


def test_mie_pins():
    rng = np.random.default_rng(1)
    v = rng.standard_normal((40, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for k, eps in ((1.0, 2.25), (4.0, complex(-15, 1)), (3.0, 1.33 ** 2)):
        Eo, Co = mie.fields(v, k, 1.0, eps, "outside", nmax=40)
        Ei, Ci = mie.fields(v, k, 1.0, eps, "inside", nmax=40)
        tan = lambda X: np.cross(v, X)
        assert np.abs(tan(Eo) - tan(Ei)).max() < 1e-12 * np.abs(Eo).max()     # tangential E
        assert np.abs(tan(Co) - tan(Ci)).max() < 1e-12 * np.abs(Co).max()     # tangential H
        assert np.abs(np.sum(v * Eo, 1) - eps * np.sum(v * Ei, 1)).max() < 1e-12  # normal D
    qext, qsca = mie.efficiencies(5.0, 1.33)
    assert abs(qext - qsca) < 1e-12 * qext          # optical theorem, lossless sphere
    E, _ = mie.fields(np.array([[0.1, 0.2, 0.3]]), 1e-3, 1.0, 2.25, "inside")
    assert abs(E[0, 0] - 3 / (2.25 + 2)) < 1e-3     # Rayleigh (electrostatic) limit


def _dense(P):
    N = P.n
    A = np.zeros((6 * N, 6 * N), complex)
    for j in range(6 * N):
        e = np.zeros(6 * N, complex)
        e[j] = 1
        A[:, j] = P.apply(e.reshape(N, 6)).reshape(-1)
    return A


def test_gmres_matches_dense_solve_and_preconditioner_helps():
    q = nystrom3(icosphere(2))
    P = BemProblem(q, 1.0, 2.25)
    A = _dense(P)
    b = P.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])
    xd = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    x, info = gmres_solve(P.apply, b, P.block_preconditioner(), tol=1e-12, restart=200, maxit=400)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9
    x2, info2 = gmres_solve(P.apply, b, None, tol=1e-8, restart=200, maxit=400)
    x3, info3 = gmres_solve(P.apply, b, P.block_preconditioner(), tol=1e-8, restart=200, maxit=400)
    assert info3["iterations"] < info2["iterations"]
    # restarted run with a tiny cycle still converges to the same solution
    x4, info4 = gmres_solve(P.apply, b, P.block_preconditioner(), tol=1e-10, restart=7, maxit=2000)
    assert np.linalg.norm(x4 - xd) / np.linalg.norm(xd) < 1e-7
    # the preconditioner blocks are the coincident-node part of A
    M = P.precond_blocks()
    for i in (0, 17, 101):
        assert np.allclose(M[i], A[6 * i:6 * i + 6, 6 * i:6 * i + 6], atol=1e-14)


def test_gmres_happy_breakdown_on_exactly_solvable_system():
    rng = np.random.default_rng(0)
    D = np.diag(np.array([2.0, 3.0, 2.0, 3.0]) + 0j)
    b = rng.standard_normal(4) + 0j
    x, info = gmres_solve(lambda v: D @ v, b, tol=1e-15, restart=10)
    assert info["iterations"] <= 2
    assert np.allclose(D @ x, b, atol=1e-14)


def test_solution_approaches_mie_under_refinement(sphere_nodes):
    errs = []
    for nu in (2, 4):
        q = sphere_nodes[nu]
        P = BemProblem(q, 1.0, 2.25)
        b = P.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])
        x, info = gmres_solve(P.apply, b, P.block_preconditioner(), tol=1e-8, restart=100)
        xm = mie.surface_unknowns(q, 1.0, 1.0, 2.25)
        errs.append(np.linalg.norm(x[:, :3] - xm[:, :3]) / np.linalg.norm(xm[:, :3]))
    assert errs[1] < errs[0] < 0.1
