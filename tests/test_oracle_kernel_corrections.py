"""Pins of the oracle's kernel and self-triangle integrals (CPU only)."""

import os

import numpy as np
import pytest

from oracle.kernel import green, green_grad_src, wavenumber
from oracle import corrections as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_wavenumber_principal_branch():
    # Sec. 2.1: k^2 = eps mu w^2/c^2 with exp(-i w t); the decaying branch has Im k >= 0
    assert abs(wavenumber(1.0, complex(-15, 1)) - complex(0.12903, 3.87513)) < 2e-5
    assert abs(wavenumber(1.0, complex(-1e4, 1e2)) - complex(0.49999, 100.00125)) < 2e-5
    assert wavenumber(4.0, complex(-15, 1)).imag > 0


@pytest.mark.parametrize("k", [1.0, 2 + 1.5j, 0.5 + 15.5j])
def test_green_gradient_is_source_derivative(k):
    rng = np.random.default_rng(3)
    src = rng.standard_normal((20, 3))
    tgt = rng.standard_normal((20, 3))
    G = green_grad_src(k, src, tgt)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (green(k, src + e, tgt) - green(k, src - e, tgt)) / (2 * h)
        assert np.max(np.abs(fd - G[:, d]) / np.abs(G).max()) < 1e-8
    # symmetry g(s', s) = g(s, s') and the Helmholtz radial ODE at one point
    assert np.allclose(green(k, src, tgt), green(k, tgt, src))


def _brute_polar(tri, O, f, N=400000):
    """int over the triangle of f(phi, rho_m, direction) dphi by the midpoint rule in phi."""
    ph = np.linspace(-np.pi, np.pi, N, endpoint=False) + np.pi / N
    d = np.stack([np.cos(ph), np.sin(ph), 0 * ph], 1)
    rm = np.full(N, np.inf)
    for e in range(3):
        A = tri[e]
        B = tri[(e + 1) % 3]
        M = np.stack([d[:, :2], np.broadcast_to(-(B - A)[:2], (N, 2))], 2)
        sol = np.linalg.solve(M, np.broadcast_to((A - O)[:2], (N, 2))[..., None])[..., 0]
        t, u = sol[:, 0], sol[:, 1]
        ok = (t > 0) & (u >= 0) & (u <= 1)
        rm = np.where(ok, np.minimum(rm, t), rm)
    return f(ph, rm, d).sum(0) * 2 * np.pi / N


SCALENE = np.array([[0.1, 0.2, 0.0], [1.0, 0.1, 0.0], [0.4, 0.9, 0.0]])
NZ = np.array([0.0, 0.0, 1.0])


def _frames(tri, O):
    return C.edge_frames(O[None], tri[None], NZ[None])


def test_equilateral_centroid_golden():
    rows = np.loadtxt(os.path.join(GOLDEN, "appendix_b_equilateral.txt"))
    for s, drho, cpv in rows:
        tri = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * np.sqrt(3) / 2, 0]], float)
        h, ie, je, p1, p2 = _frames(tri, tri.mean(0))
        assert abs(C.static_drho_dphi(h, p1, p2)[0] - drho) < 1e-9
        assert np.linalg.norm(C.static_cpv_r_over_r3(h, ie, p1, p2)[0]) <= cpv + 1e-13


@pytest.mark.parametrize("bary", [(2 / 3, 1 / 6, 1 / 6), (1 / 6, 2 / 3, 1 / 6), (0.2, 0.3, 0.5)])
def test_static_closed_forms_vs_brute_force(bary):
    O = np.asarray(bary) @ SCALENE
    h, ie, je, p1, p2 = _frames(SCALENE, O)
    b3 = _brute_polar(SCALENE, O, lambda ph, rm, d: rm)
    b9 = _brute_polar(SCALENE, O, lambda ph, rm, d: np.log(rm)[:, None] * d)
    assert abs(C.static_drho_dphi(h, p1, p2)[0] - b3) < 1e-9
    assert np.abs(C.static_cpv_r_over_r3(h, ie, p1, p2)[0] - b9).max() < 1e-9


@pytest.mark.parametrize("k", [1e-3, 0.5, 2 + 1j, 20 + 4000j])
def test_self_G_vs_brute_force(k):
    O = np.array([2 / 3, 1 / 6, 1 / 6]) @ SCALENE
    V, G = C.self_terms(O[None], NZ[None], np.array([0]), SCALENE[None], k)
    Gb = _brute_polar(SCALENE, O, lambda ph, rm, d: (np.exp(1j * k * rm) - 1) / (1j * k)) / (4 * np.pi)
    assert abs(G[0] - Gb) < 1e-9 * abs(Gb)


def test_small_k_limit_matches_appendix_b_taylor_forms():
    O = np.array([2 / 3, 1 / 6, 1 / 6]) @ SCALENE
    h, ie, je, p1, p2 = _frames(SCALENE, O)
    S = 0.5 * np.linalg.norm(np.cross(SCALENE[1] - SCALENE[0], SCALENE[2] - SCALENE[0]))
    B3 = C.static_drho_dphi(h, p1, p2)[0]
    B9 = C.static_cpv_r_over_r3(h, ie, p1, p2)[0]
    rr = _brute_polar(SCALENE, O, lambda ph, rm, d: 0.5 * rm[:, None] ** 2 * d)   # int r/r dA
    for k in (1e-2, 3e-2):
        V, G = C.self_terms(O[None], NZ[None], np.array([0]), SCALENE[None], k)
        # eq. B.2: two Taylor terms, error O((k h)^2)
        assert abs(G[0] - (B3 + 1j * k * S) / (4 * np.pi)) < 0.1 * k ** 2
        # eq. B.4 + B.5: -k^2/(8 pi) int r/r dA - (1/4pi) CPV int r/r^3 dA, error O(k^3)
        Vt = -k ** 2 / (8 * np.pi) * rr - B9 / (4 * np.pi)
        assert np.abs(V[0] - Vt).max() < 0.1 * k ** 3


def _nodes_one_triangle(tri):
    pts = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]]) @ tri
    return pts, np.repeat(NZ[None], 3, 0), np.zeros(3, dtype=np.int64)


@pytest.mark.parametrize("k", [0.7, 3 + 2j])
def test_linear_blocks_partition_of_unity_and_brute_force(k):
    pts, nrm, pt = _nodes_one_triangle(SCALENE)
    nodes, dV, dG = C.self_blocks(pts, nrm, pt, SCALENE[None], k, mode="linear")
    V, G = C.self_terms(pts, nrm, pt, SCALENE[None], k)
    # the linear basis sums to one, so the blocks add up to the element integrals
    assert np.allclose(dV.sum(1), V, atol=1e-13)
    assert np.allclose(dG.sum(1), G, atol=1e-13)
    # brute force: int g L_beta dA in polar coordinates about the target
    grads = C.lagrange_gradients(pts, nrm, nodes)[0]
    for a in range(3):
        O = pts[a]
        for b in range(3):
            gL = grads[b]

            def f(ph, rm, d, gL=gL, O=O, b=b, a=a):
                # int_0^rm e^{ik r}/(4 pi) [L_b(O) + r gL.d] dr
                e = np.exp(1j * k * rm)
                base = (e - 1) / (1j * k) * (1.0 if a == b else 0.0)
                mom = ((1 - 1j * k * rm) * e - 1) / k ** 2 * (d @ gL)
                return (base + mom) / (4 * np.pi)

            ref = _brute_polar(SCALENE, O, f)
            assert abs(dG[a, b] - ref) < 1e-8 * abs(G[a])


def test_mean_mode_is_equal_split():
    pts, nrm, pt = _nodes_one_triangle(SCALENE)
    nodes, dV, dG = C.self_blocks(pts, nrm, pt, SCALENE[None], 1.3, mode="mean")
    V, G = C.self_terms(pts, nrm, pt, SCALENE[None], 1.3)
    assert np.allclose(dV, V[:, None, :] / 3)
    assert np.allclose(dG, G[:, None] / 3)
