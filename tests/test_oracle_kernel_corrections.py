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


# ---------------------------------------------------------------------------
# Large |k| rho: the regular remainder H of CPV int grad'g (Appendix B, eqs.
# B.4, B.5, B.9 with the exact radial integral) on triangles whose edges lie
# many decay lengths 1/Im k from the node, and the LINEAR first moment.  The
# brute force integrates in polar coordinates about the node: Gauss-Legendre
# in phi inside each sector between two vertex directions (the edge distance
# rho_m(phi) is smooth there), and the radial integrals numerically in
# t = ln(rho), where the boundary layer of width 1/|k| at rho = 0 is resolved.
# ---------------------------------------------------------------------------


def _sectors(tri, O, f, nq=160):
    ang = np.sort(np.arctan2(tri[:, 1] - O[1], tri[:, 0] - O[0]))
    cuts = np.concatenate([ang, [ang[0] + 2 * np.pi]])
    x, w = np.polynomial.legendre.leggauss(nq)
    tot = 0.0
    for s in range(3):
        a, b = cuts[s], cuts[s + 1]
        ph = 0.5 * (b - a) * (x + 1) + a
        d = np.stack([np.cos(ph), np.sin(ph), 0 * ph], 1)
        rm = np.full(nq, np.inf)
        for e in range(3):
            A = tri[e]
            B = tri[(e + 1) % 3]
            M = np.stack([d[:, :2], np.broadcast_to(-(B - A)[:2], (nq, 2))], 2)
            sol = np.linalg.solve(M, np.broadcast_to((A - O)[:2], (nq, 2))[..., None])[..., 0]
            t, u = sol[:, 0], sol[:, 1]
            ok = (t > 0) & (u >= -1e-12) & (u <= 1 + 1e-12)
            rm = np.where(ok, np.minimum(rm, t), rm)
        tot = tot + np.tensordot(0.5 * (b - a) * w, f(ph, rm, d), axes=(0, 0))
    return tot


def _radial_log(rm, fn, span=40.0, panels=320, nq=10):
    """int_0^rm fn(u) du / u as an integral over t = ln u in [ln rm - span, ln rm]."""
    x, w = np.polynomial.legendre.leggauss(nq)
    h = span / panels
    t = np.log(rm)[:, None, None] - span + h * np.arange(panels)[None, :, None] + 0.5 * h * (x + 1)[None, None, :]
    u = np.exp(t)
    return np.sum(fn(u) * (0.5 * h * w)[None, None, :], axis=(1, 2))


def _V_static_scale(tri, O):
    return np.abs(_sectors(tri, O, lambda ph, rm, d: np.log(rm)[:, None] * d)).max() / (4 * np.pi)


@pytest.mark.parametrize("scale", [1.0, 0.01])
@pytest.mark.parametrize("k", [4.0, 0.5 + 15.5j, 20 + 4000j])
def test_self_V_vs_brute_force_large_kh(scale, k):
    """V = (1/4pi) int rho^ [int_0^rho_m ((i k u - 1) e^{iku} + 1)/u du - ln rho_m] dphi.
    The unit triangle at k = 0.5+15.5i and 20+4000i puts |k| rho_m far above 2 (the
    exponential-integral branch of H); at 20+4000i the remainder cancels the static
    part and V is zero to rounding, which a dropped or mis-signed term would break."""
    tri = SCALENE * scale
    for bary in ((2 / 3, 1 / 6, 1 / 6), (0.2, 0.3, 0.5)):
        O = np.asarray(bary) @ tri
        h, ie, je, p1, p2 = _frames(tri, O)
        rmax = np.max(h / np.cos(np.maximum(np.abs(p1), np.abs(p2))))
        V, G = C.self_terms(O[None], NZ[None], np.array([0]), tri[None], k)

        def f(ph, rm, d):
            H = _radial_log(rm, lambda u: (1j * k * u - 1) * np.exp(1j * k * u) + 1)
            return (H - np.log(rm))[:, None] * d

        Vb = _sectors(tri, O, f) / (4 * np.pi)
        ref = max(np.abs(Vb).max(), _V_static_scale(tri, O))
        assert np.abs(V[0] - Vb).max() <= 1e-10 * ref, (np.abs(V[0] - Vb).max(), ref)
        if scale == 1.0 and abs(k) > 10:
            assert abs(k) * rmax > 4.0
    if scale == 1.0 and abs(k) > 1000:
        assert np.abs(V[0]).max() <= 1e-12 * _V_static_scale(tri, O)


def _lagrange_grads_2d(pts):
    """grad L_b of the plane interpolant with L_b(pts[c]) = delta_bc (triangle in z = 0)."""
    A = np.column_stack([np.ones(3), pts[:, 0], pts[:, 1]])
    coef = np.linalg.solve(A, np.eye(3))          # column b: (c0, cx, cy) of L_b
    return np.column_stack([coef[1], coef[2], np.zeros(3)]), coef


@pytest.mark.parametrize("scale", [1.0, 0.01])
@pytest.mark.parametrize("k", [0.7, 0.5 + 15.5j, 20 + 4000j])
def test_linear_dV_blocks_vs_brute_force(scale, k):
    """LINEAR blocks of grad'g: dV_{O,b} = CPV int_T grad'g(s', O) L_b(s') dA', brute force in
    polar coordinates: (1/4pi) int rho^ [L_b(O) (H(rho_m) - ln rho_m) + (rho^ . grad L_b) R1(rho_m)] dphi
    with R1(rho_m) = int_0^rho_m (i k u - 1) e^{iku} du (the first moment W of the oracle)."""
    tri = SCALENE * scale
    pts, nrm, pt = _nodes_one_triangle(tri)
    nodes, dV, dG = C.self_blocks(pts, nrm, pt, tri[None], k, mode="linear")
    assert list(nodes[0]) == [0, 1, 2]
    grads, coef = _lagrange_grads_2d(pts)
    for a in range(3):
        O = pts[a]
        scale_v = _V_static_scale(tri, O)
        for b in range(3):
            LbO = coef[0, b] + coef[1, b] * O[0] + coef[2, b] * O[1]
            gL = grads[b]

            def f(ph, rm, d, LbO=LbO, gL=gL):
                H = _radial_log(rm, lambda u: (1j * k * u - 1) * np.exp(1j * k * u) + 1)
                R1 = _radial_log(rm, lambda u: (1j * k * u - 1) * np.exp(1j * k * u) * u)
                return (LbO * (H - np.log(rm)) + (d @ gL) * R1)[:, None] * d

            ref = _sectors(tri, O, f) / (4 * np.pi)
            assert np.abs(dV[a, b] - ref).max() <= 1e-9 * max(scale_v, np.abs(ref).max()), (a, b)
