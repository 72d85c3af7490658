"""Pins of the oracle's conjugate-transpose operator (CPU only)."""

import numpy as np
import pytest

from oracle.adjoint import apply_corrections_adjoint, point_sum_adjoint
from oracle.corrections import self_blocks
from oracle.direct import apply_corrections, point_sum
from oracle.native import point_sum_c
from synthetic import complex_normal, torus, nystrom3


def _dot(u, v):
    return np.sum(np.conj(u) * v)


@pytest.mark.parametrize("k", [1.3, 2.0 + 0.7j, 0.5 + 15.5j])
def test_point_sum_adjoint_identity(sphere_nodes, k):
    """sum conj(y) . Op(a, b) = sum conj(a_bar) . a + conj(b_bar) . b against the
    forward oracle (itself pinned by the EFIE identities)."""
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    a, b, y = (complex_normal((n, 3), s) for s in (21, 22, 23))
    Op = point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b)
    ab, bb = point_sum_adjoint(q["points"], q["normals"], q["weights"], q["point_tri"], k, y)
    lhs = _dot(y, Op)
    rhs = _dot(ab, a) + _dot(bb, b)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # each part separately: b only, then a only
    Ob = point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, 0 * a, b)
    assert abs(_dot(y, Ob) - _dot(bb, b)) <= 1e-12 * abs(_dot(y, Ob))


def test_point_sum_adjoint_rows_batched_and_entrywise():
    """Sampled rows and batches equal the full single call; a unit y_alpha
    picks out one column of the operator."""
    q = nystrom3(torus(1.0, 0.3, 12, 6))
    n = q["points"].shape[0]
    k = 1.0 + 0.2j
    y = complex_normal((2, n, 3), 31)
    ab, bb = point_sum_adjoint(q["points"], q["normals"], q["weights"], q["point_tri"], k, y)
    rows = np.array([0, 5, 17, n - 1])
    ar, br = point_sum_adjoint(q["points"], q["normals"], q["weights"], q["point_tri"], k, y[1], rows=rows)
    assert np.allclose(ar, ab[1][rows], rtol=0, atol=1e-14 * np.abs(ab).max())
    assert np.allclose(br, bb[1][rows], rtol=0, atol=1e-14 * np.abs(bb).max())
    # entry (alpha, c) of Op(a, b) for unit a_beta,d is conj(a_bar_beta,d) of the unit y_alpha,c
    al, c, be, d = 3, 1, 40, 2
    e = np.zeros((n, 3), complex)
    e[al, c] = 1.0
    ua, ub = point_sum_adjoint(q["points"], q["normals"], q["weights"], q["point_tri"], k, e)
    a = np.zeros((n, 3), complex)
    a[be, d] = 1.0
    col = point_sum(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, 0 * a, rows=[al])
    assert abs(col[0, c] - np.conj(ua[be, d])) <= 1e-14 * max(1.0, abs(col[0, c]))


@pytest.mark.parametrize("mode", ["linear", "mean"])
def test_correction_adjoint_identity(sphere_nodes, mode):
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    k = 1.5 + 0.3j
    blk = self_blocks(q["points"], q["normals"], q["point_tri"], q["tri_vertices"], k, mode=mode)
    a, b, y = (complex_normal((n, 3), s) for s in (41, 42, 43))
    C = apply_corrections(q["normals"], q["point_tri"], blk, a, b)
    ab, bb = apply_corrections_adjoint(q["normals"], q["point_tri"], blk, y)
    lhs = _dot(y, C)
    assert abs(lhs - (_dot(ab, a) + _dot(bb, b))) <= 1e-12 * abs(lhs)


def test_bem_apply_adjoint_identity(sphere_nodes):
    """sum conj(v) . A x = sum conj(A^H v) . x for the 6N system (lossy interior),
    and M^{-H} is the conjugate transpose of M^{-1} in the same sense."""
    from oracle.bem import BemProblem
    q = sphere_nodes[2]
    n = q["points"].shape[0]
    ob = BemProblem(q, 1.0, -15 + 1j)
    x = complex_normal((n, 6), 81)
    v = complex_normal((n, 6), 82)
    lhs = _dot(v, ob.apply(x))
    rhs = _dot(ob.apply_adjoint(v), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    P, PH = ob.block_preconditioner(), ob.block_preconditioner(adjoint=True)
    assert abs(_dot(v, P(x)) - _dot(PH(v), x)) <= 1e-12 * abs(_dot(v, P(x)))
