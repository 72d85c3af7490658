"""The large PEC-like prolate ellipsoid (semi-axes 4:1:1, 1,003,520 triangles,
3,010,560 nodes, k0 = 40, eps = -1e4 + 1e2 i, octree depth 8) on the GPU against
the oracle: the octree bit for bit, the exterior operator (orders per level up to
~170 at level 2) and the local-only interior operator on sampled rows (needs an
MI355X)."""

import numpy as np
import pytest

from oracle.corrections import self_blocks
from oracle.direct import apply_corrections
from oracle.kernel import wavenumber
from oracle.native import point_sum_c
from oracle.tree import Octree
from synthetic import CONFIGS, complex_normal, config_mesh, nystrom3, seed_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CFG = CONFIGS[5]
K0 = CFG["k0"]
K1 = wavenumber(K0, CFG["eps"])


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import _abi
    _abi.load()
    return _abi


@pytest.fixture(scope="module")
def c5():
    return nystrom3(config_mesh(5))


def _rel(y, ref):
    return np.linalg.norm(y - ref) / np.linalg.norm(ref)


def sampled_reference(q, k, a, b, rows):
    """The oracle's operator (point sum + LINEAR self-triangle blocks) on `rows`.
    The blocks of a row depend only on its own triangle, so they are built on the
    sub-mesh of the sampled rows' triangles (nodes 3t, 3t+1, 3t+2 of triangle t)."""
    y = point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b, rows=rows)
    tris = np.unique(q["point_tri"][rows])
    sub = (3 * tris[:, None] + np.arange(3)[None, :]).reshape(-1)
    assert np.all(q["point_tri"][sub] == np.repeat(tris, 3))
    remap = np.repeat(np.arange(len(tris)), 3)
    blk = self_blocks(q["points"][sub], q["normals"][sub], remap, q["tri_vertices"][tris], k, mode="linear")
    loc = np.searchsorted(sub, rows)
    corr = apply_corrections(q["normals"][sub], remap, blk, a[..., sub, :], b[..., sub, :], rows=loc)
    return y + corr


def test_c5_tree_bit_exact(abi, c5):
    q = c5
    print("c5 tree", flush=True)
    P = abi.Plan(q["points"], q["normals"], q["weights"], K0, 4, depth=8, corr="none")
    ref = Octree(q["points"], 8)
    t = P.export_tree(8)
    assert np.array_equal(t["codes"], ref.codes)
    assert np.array_equal(t["perm"], ref.perm.astype(np.int32))
    for l in range(9):
        t = P.export_tree(l)
        assert np.array_equal(t["keys"], ref.keys[l])
        assert np.array_equal(t["start"], ref.box_start[l].astype(np.int32))
        assert np.array_equal(t["parent"], ref.parent[l].astype(np.int32))
        big = np.iinfo(np.int32).max
        nb = np.sort(np.where(t["nbr"] >= 0, t["nbr"], big), axis=1)
        for bx in range(len(ref.keys[l])):
            c = len(ref.nbr[l][bx])
            assert np.array_equal(nb[bx][:c], ref.nbr[l][bx]) and np.all(nb[bx][c:] == big)
            if l >= 2:
                ff = np.sort(t["ff_idx"][t["ff_ofs"][bx]:t["ff_ofs"][bx + 1]])
                assert np.array_equal(ff, ref.ff[l][bx])
        print("c5 tree level", l, "boxes", len(ref.keys[l]), flush=True)
    P.close()


def test_c5_exterior_and_interior_sampled_rows(abi, c5):
    """Exterior k0 = 40: FP64 orders per level for 1e-6 (16 at the leaves to ~170
    at level 2) within 1e-6 of the oracle on 1024 seeded rows; FP32 orders for 1e-4
    within 2e-4.  Interior k1 = 20 + 4000i: every level's far field is damped by
    exp(-Im k1 h_l) < 1e-16, so the plan is local only; within 1e-9 of the oracle
    (FP64) and 1e-5 (FP32)."""
    q = c5
    n = q["points"].shape[0]
    a = complex_normal((n, 3), seed_for(5, "a"))
    b = complex_normal((n, 3), seed_for(5, "b"))
    rows = np.sort(np.random.default_rng(seed_for(5, "rows")).choice(n, 1024, replace=False))
    kw = dict(depth=8, corr="linear", point_tri=q["point_tri"], tri_vertices=q["tri_vertices"])
    for k, cases in ((K0, (("fp64", 1e-6, 1e-6), ("fp32", 1e-4, 2e-4))),
                     (K1, (("fp64", 1e-6, 1e-9), ("fp32", 1e-4, 1e-5)))):
        print("c5 oracle rows k=", k, flush=True)
        ref = sampled_reference(q, k, a, b, rows)
        for prec, tol, bound in cases:
            dt = torch.complex128 if prec == "fp64" else torch.complex64
            print("c5 plan", prec, "k=", k, flush=True)
            P = abi.Plan(q["points"], q["normals"], q["weights"], k, 0, precision=prec, tol=tol, **kw)
            y = P.matvec(torch.from_numpy(a).to("cuda", dt), torch.from_numpy(b).to("cuda", dt)).cpu().numpy()
            err = _rel(y[rows], ref)
            inf = P.info()
            print("c5 k=%s %s orders %s far_lmin %d rel err %.3e device GB %.1f" % (
                k, prec, inf["order_level"], inf["far_lmin"], err, inf["device_bytes"] / 1e9), flush=True)
            assert err <= bound
            P.close()
