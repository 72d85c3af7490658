"""Pins of the reference octree (CPU only)."""

import numpy as np
import pytest

from oracle.tree import Octree, encode, deinterleave, interleave, quantize
from synthetic import icosphere, nystrom3, torus


def test_morton_hand_example():
    # q = (1, 0, 0) -> bit 0; (0, 1, 0) -> bit 1; (0, 0, 1) -> bit 2; (3, 1, 2) -> 0b 100 011 ... computed by hand
    q = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 1, 2], [2 ** 21 - 1, 0, 0]])
    c = interleave(q)
    assert c[0] == 1 and c[1] == 2 and c[2] == 4
    # (3,1,2): bit0: x=1,y=1,z=0 -> 0b011 = 3 ; bit1: x=1,y=0,z=1 -> 0b101 << 3 = 40
    assert c[3] == 3 + 40
    assert c[4] == sum(1 << (3 * b) for b in range(21))
    for key, lvl in ((12345, 6), (7, 1), (0, 0)):
        assert encode(*deinterleave(key, lvl), lvl) == key


def test_quantisation_is_sub_then_mul_and_clamped():
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.25], [0.3, 0.7, 0.9]])
    lo, ext, inv, q = quantize(pts)
    assert ext == 1.0 and inv == 2.0 ** 21
    assert (q[1] == [2 ** 21 - 1, 2 ** 20, 2 ** 19]).all()       # the max coordinate clamps
    assert q[2, 0] == int(np.floor((0.3 - 0.0) * 2.0 ** 21))
    with pytest.raises(ValueError):
        quantize(np.zeros((4, 3)))


@pytest.mark.parametrize("shape", ["sphere", "torus"])
def test_tree_invariants_and_exact_cover(shape):
    if shape == "sphere":
        q = nystrom3(icosphere(4))
        depth = 3
    else:
        q = nystrom3(torus(1.0, 0.3, 40, 12))
        depth = 4
    pts = q["points"]
    T = Octree(pts, depth)
    n = pts.shape[0]
    sc = T.codes[T.perm]
    assert np.all(sc[1:] >= sc[:-1])
    # stable: equal codes keep index order
    eq = sc[1:] == sc[:-1]
    assert np.all(T.perm[1:][eq] > T.perm[:-1][eq])
    L = depth
    # every point in exactly one leaf; boxes are non-empty and sorted
    assert T.box_start[L][0] == 0 and T.box_start[L][-1] == n
    assert np.all(np.diff(T.box_start[L]) > 0)
    for l in range(depth + 1):
        assert np.all(np.diff(T.keys[l].astype(np.int64)) > 0)
        for i, nb in enumerate(T.nbr[l]):
            assert i in nb
            for j in nb:
                assert i in T.nbr[l][j]                          # symmetric
        if l >= 1:
            assert np.all(T.keys[l - 1][T.parent[l]] == T.keys[l] >> np.uint64(3))
    # every (target leaf, source point) pair is covered exactly once by the
    # leaf's neighbour list or by the FF list of exactly one ancestor level
    for tl in range(len(T.keys[L])):
        count = np.zeros(n, dtype=int)
        for j in T.nbr[L][tl]:
            count[T.box_start[L][j]:T.box_start[L][j + 1]] += 1
        box = tl
        for l in range(L, 1, -1):
            for j in T.ff[l][box]:
                # all sorted points inside box j of level l
                count[T.box_start[l][j]:T.box_start[l][j + 1]] += 1
            box = T.parent[l][box]
        assert np.all(count == 1)
    # far-field boxes are never adjacent and their parents are
    for l in range(2, depth + 1):
        for i, ff in enumerate(T.ff[l]):
            ci = T.coords[l][i]
            for j in ff:
                d = np.abs(T.coords[l][j] - ci)
                assert d.max() >= 2
                pd = np.abs(T.coords[l - 1][T.parent[l][j]] - T.coords[l - 1][T.parent[l][i]])
                assert pd.max() <= 1


def _split_triangle_pairs(q, depth):
    """Node pairs of one triangle whose leaves are not neighbours in the reference octree."""
    from oracle.tree import Octree
    T = Octree(q["points"], depth)
    inv = np.empty_like(T.perm)
    inv[T.perm] = np.arange(len(T.perm))
    leaf = T.point_box[depth][inv]
    tri = q["point_tri"]
    order = np.argsort(tri, kind="stable")
    bad = 0
    for t in range(int(tri.max()) + 1):
        nodes = order[np.searchsorted(tri[order], t):np.searchsorted(tri[order], t, side="right")]
        for i, a in enumerate(nodes):
            near = set(T.nbr[depth][leaf[a]].tolist())
            bad += sum(1 for b in nodes[i + 1:] if leaf[b] not in near)
    return bad


def test_deep_trees_split_triangles():
    """Why the library refuses some depths: at the configurations' depths every
    triangle's nodes share the near field, one level or two deeper they do not
    (the torus at depth 7, the 1280-triangle sphere at depth 5)."""
    from synthetic import icosphere, nystrom3, torus
    qt = nystrom3(torus(1.0, 0.3, 200, 50))
    qs = nystrom3(icosphere(8))
    assert _split_triangle_pairs(qt, 5) == 0 and _split_triangle_pairs(qt, 7) > 0
    assert _split_triangle_pairs(qs, 3) == 0 and _split_triangle_pairs(qs, 5) > 0
