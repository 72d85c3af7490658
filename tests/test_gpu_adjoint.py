"""GPU parity of the adjoint FMM product Op_k^H y against the oracle (needs an MI355X)."""

import numpy as np
import pytest

from oracle.adjoint import apply_corrections_adjoint, point_sum_adjoint
from oracle.corrections import self_blocks
from synthetic import complex_normal, icosphere, nystrom3, seed_for, torus

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import _abi
    _abi.load()
    return _abi


@pytest.fixture(scope="module")
def sphere():
    return nystrom3(icosphere(8))          # 1280 triangles, 3840 nodes


def _plan(abi, q, k, order, depth, precision="fp64", corr="linear", nrhs_max=1, translate="fp32"):
    return abi.Plan(q["points"], q["normals"], q["weights"], k, order, depth=depth, precision=precision,
                    nrhs_max=nrhs_max, corr=corr, point_tri=q["point_tri"], tri_vertices=q["tri_vertices"],
                    translate=translate)


def _gpu(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _rel(y, ref):
    return np.linalg.norm(y - ref) / np.linalg.norm(ref)


def _oracle_adjoint(q, k, y, corr="linear", rows=None):
    ab, bb = point_sum_adjoint(q["points"], q["normals"], q["weights"], q["point_tri"], k, y, rows=rows)
    if corr != "none":
        blk = self_blocks(q["points"], q["normals"], q["point_tri"], q["tri_vertices"], k, mode=corr)
        ca, cb = apply_corrections_adjoint(q["normals"], q["point_tri"], blk, y, rows=rows)
        ab, bb = ab + ca, bb + cb
    return ab, bb


@pytest.mark.parametrize("k", [1.0, 1.5, 2.0 + 1.5j])
def test_fp64_adjoint_matches_oracle(abi, sphere, k):
    q = sphere
    n = q["points"].shape[0]
    y = complex_normal((n, 3), seed_for(1, "a") + 7)
    print("fp64 adjoint sphere k =", k, flush=True)
    P = _plan(abi, q, k, 16, 3)
    ab, bb = P.matvec_adjoint(_gpu(y))
    ab, bb = ab.cpu().numpy(), bb.cpu().numpy()
    ra, rb = _oracle_adjoint(q, k, y)
    ea, eb = _rel(ab, ra), _rel(bb, rb)
    print("rel err a_bar %.3e b_bar %.3e" % (ea, eb))
    assert ea <= 1e-6 and eb <= 1e-6
    P.close()


def test_adjoint_identity_batched_and_deterministic(abi, sphere):
    """sum conj(y) . Op(a, b) = sum conj(a_bar) . a + conj(b_bar) . b with both
    products from the GPU (to the FMM error); batched columns equal single
    calls bit for bit; two runs are identical."""
    q = sphere
    n = q["points"].shape[0]
    k = 1.2 + 0.4j
    P = _plan(abi, q, k, 20, 3, nrhs_max=3)
    a = complex_normal((3, n, 3), 51)
    b = complex_normal((3, n, 3), 52)
    y = complex_normal((3, n, 3), 53)
    Op = P.matvec(_gpu(a), _gpu(b)).cpu().numpy()
    ab, bb = P.matvec_adjoint(_gpu(y))
    ab2, bb2 = P.matvec_adjoint(_gpu(y))
    assert torch.equal(ab, ab2) and torch.equal(bb, bb2)
    ab, bb = ab.cpu().numpy(), bb.cpu().numpy()
    for r in range(3):
        lhs = np.sum(np.conj(y[r]) * Op[r])
        rhs = np.sum(np.conj(ab[r]) * a[r]) + np.sum(np.conj(bb[r]) * b[r])
        assert abs(lhs - rhs) <= 1e-8 * abs(lhs)
        s_a, s_b = P.matvec_adjoint(_gpu(y[r]))
        assert np.array_equal(s_a.cpu().numpy(), ab[r]) and np.array_equal(s_b.cpu().numpy(), bb[r])
    P.close()


@pytest.mark.parametrize("translate,order,tol", [("fp32", 8, 3e-4), ("bf16x3", 8, 3e-4), ("bf16x3", 5, 3e-3)])
def test_fp32_adjoint_matches_oracle(abi, sphere, translate, order, tol):
    q = sphere
    n = q["points"].shape[0]
    k = 1.5
    y = complex_normal((n, 3), 61)
    print("fp32 adjoint", translate, order, flush=True)
    P = _plan(abi, q, k, order, 3, precision="fp32", translate=translate)
    ab, bb = P.matvec_adjoint(_gpu(y, torch.complex64))
    ra, rb = _oracle_adjoint(q, k, y)
    ea, eb = _rel(ab.cpu().numpy(), ra), _rel(bb.cpu().numpy(), rb)
    print("rel err a_bar %.3e b_bar %.3e" % (ea, eb))
    assert ea <= tol and eb <= tol
    P.close()


def test_adjoint_without_corrections_ragged_leaves(abi):
    """A plan with no self-triangle terms (point sum only) on a small torus whose
    leaves hold uneven node counts; depth 4."""
    q = nystrom3(torus(1.0, 0.3, 40, 12))
    n = q["points"].shape[0]
    k = 2.0 + 0.5j
    y = complex_normal((n, 3), 71)
    P = _plan(abi, q, k, 16, 4, corr="none")
    ab, bb = P.matvec_adjoint(_gpu(y))
    ra, rb = _oracle_adjoint(q, k, y, corr="none")
    assert _rel(ab.cpu().numpy(), ra) <= 1e-6 and _rel(bb.cpu().numpy(), rb) <= 1e-6
    P.close()


@pytest.mark.parametrize("k", [4.0, complex(0.5161, 15.5034)])
def test_torus_full_size_adjoint_sampled_rows(abi, k):
    """The 60k-node torus (depth 5, FP64 p = 16) on 256 seeded source rows."""
    q = nystrom3(torus(1.0, 0.3, 200, 50))
    n = q["points"].shape[0]
    y = complex_normal((n, 3), seed_for(2, "a") + 9)
    rows = np.sort(np.random.default_rng(seed_for(2, "rows") + 1).choice(n, 256, replace=False))
    print("torus adjoint k =", k, flush=True)
    P = _plan(abi, q, k, 16, 5)
    ab, bb = P.matvec_adjoint(_gpu(y))
    ra, rb = _oracle_adjoint(q, k, y, rows=rows)
    ea, eb = _rel(ab.cpu().numpy()[rows], ra), _rel(bb.cpu().numpy()[rows], rb)
    print("rel err a_bar %.3e b_bar %.3e" % (ea, eb))
    assert ea <= 1e-6 and eb <= 1e-6
    P.close()
