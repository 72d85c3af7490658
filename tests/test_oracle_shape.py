"""Pins of the oracle's shape derivatives and cross-section functionals (CPU only)."""

import numpy as np
import pytest

from oracle import mie
from oracle.shape import (bilinear_point_sum, cross_section_far, cross_section_surface, pair_derivatives,
                          sphere_rule)
from synthetic import complex_normal, nystrom3, torus


def _case(q, seed):
    n = q["points"].shape[0]
    return tuple(complex_normal((n, 3), seed + i) for i in range(3))


@pytest.mark.parametrize("k", [1.3, 2.0 + 0.7j])
def test_pair_derivatives_match_differences_of_the_point_sum(k):
    """dB/ds, dB/dn and dB/dw against central differences of B = sum conj(lam) .
    PS(a, b) computed by the plain point sum: every coordinate of six nodes
    (source and target roles move together), h = 1e-6."""
    q = nystrom3(torus(1.0, 0.35, 10, 6))          # 120 triangles, 360 nodes
    lam, a, b = _case(q, 40)
    args = [q["points"].copy(), q["normals"].copy(), q["weights"].copy(), q["point_tri"]]
    ds, dn, dw = pair_derivatives(*args, k, lam, a, b)
    h = 1e-6
    nodes = np.random.default_rng(5).choice(q["points"].shape[0], 6, replace=False)
    for slot, dref in ((0, ds), (1, dn)):
        scale = np.max(np.abs(dref))
        for i in nodes:
            for c in range(3):
                vals = []
                for sg in (1.0, -1.0):
                    arr = [x.copy() if j < 3 else x for j, x in enumerate(args)]
                    arr[slot][i, c] += sg * h
                    vals.append(bilinear_point_sum(*arr, k, lam, a, b))
                fd = (vals[0] - vals[1]) / (2 * h)
                assert abs(fd - dref[i, c]) <= 1e-6 * scale, (slot, i, c, fd, dref[i, c])
    scale = np.max(np.abs(dw))
    for i in nodes:
        vals = []
        for sg in (1.0, -1.0):
            arr = [x.copy() if j < 3 else x for j, x in enumerate(args)]
            arr[2][i] += sg * h
            vals.append(bilinear_point_sum(*arr, k, lam, a, b))
        assert abs((vals[0] - vals[1]) / (2 * h) - dw[i]) <= 1e-7 * scale


def test_pair_derivatives_translation_and_exclusion():
    """B depends on node positions only through differences, so the position
    derivatives sum to zero; pairs inside one triangle carry no term, so a mesh
    of one triangle has no derivative at all."""
    q = nystrom3(torus(1.0, 0.35, 8, 5))
    lam, a, b = _case(q, 60)
    ds, dn, dw = pair_derivatives(q["points"], q["normals"], q["weights"], q["point_tri"], 1.7 + 0.2j, lam, a, b)
    assert np.linalg.norm(ds.sum(axis=0)) <= 1e-12 * np.linalg.norm(ds)
    one = {key: (v[:3] if key != "tri_vertices" else v[:1]) for key, v in q.items()}
    d1 = pair_derivatives(one["points"], one["normals"], one["weights"], one["point_tri"], 1.0, lam[:3], a[:3],
                          b[:3])
    assert all(np.all(x == 0) for x in d1)


def test_sphere_rule_integrates_spherical_polynomials():
    """The product rule holds 4 pi, integrates x^2 to 4 pi / 3 and z^4 to 4 pi / 5."""
    dirs, w = sphere_rule(24, 48)
    assert abs(w.sum() - 4 * np.pi) <= 1e-12
    assert abs(np.sum(w * dirs[:, 0] ** 2) - 4 * np.pi / 3) <= 1e-12
    assert abs(np.sum(w * dirs[:, 2] ** 4) - 4 * np.pi / 5) <= 1e-12


@pytest.mark.parametrize("eps", [2.25, 2.25 + 0.5j])
def test_cross_sections_of_exact_sphere_fields_match_mie(sphere_nodes, eps):
    """Both forms of C_sca, fed the exact (Mie) surface fields of a sphere of
    radius 1 at k0 = 1, give Mie's Q_sca pi a^2 to the surface rule's error."""
    q = sphere_nodes[8]
    xm = mie.surface_unknowns(q, 1.0, 1.0, eps)
    ref = mie.efficiencies(1.0, np.sqrt(eps))[1] * np.pi
    cs = cross_section_surface(q, 1.0, xm, [0, 0, 1.0], [1.0, 0, 0])
    cf = cross_section_far(q, 1.0, xm, [1.0, 0, 0])
    assert abs(cs - ref) <= 5e-3 * ref
    assert abs(cf - ref) <= 5e-3 * ref
