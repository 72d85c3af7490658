"""GPU parity of the impedance-boundary-condition system (eq. 2.25) against the oracle."""

import numpy as np
import pytest

from oracle import mie
from oracle.bem import IbcProblem as OracleIbc
from oracle.gmres import gmres_solve as oracle_gmres
from synthetic import complex_normal, icosphere, nystrom3, torus

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

Z = 0.2 - 0.1j


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import solver
    return solver


@pytest.fixture(scope="module")
def small():
    q = nystrom3(icosphere(4))      # 320 triangles, 960 nodes
    return q, OracleIbc(q, 1.0, Z)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_ibc_apply_adjoint_precond_rhs_match_oracle(gpu, small):
    q, ob = small
    n = q["points"].shape[0]
    print("ibc apply small sphere", flush=True)
    pb = gpu.IbcProblem(q, 1.0, Z, order=20, depth=3)
    x = complex_normal((n, 3), 131)
    xg = torch.from_numpy(x).cuda()
    assert _rel(pb.apply(xg).cpu().numpy(), ob.apply(x)) <= 1e-7
    assert _rel(pb.apply_adjoint(xg).cpu().numpy(), ob.apply_adjoint(x)) <= 1e-7
    assert _rel(pb.precond(xg).cpu().numpy(), ob.block_preconditioner()(x)) <= 1e-11
    b = pb.rhs_planewave([0, 0, 1.0], [1.0, 0, 0]).cpu().numpy()[0]
    assert _rel(b, ob.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])) <= 1e-14
    pb.close()


def test_ibc_solves_match_oracle_and_mie(gpu, small):
    q, ob = small
    print("ibc solves small sphere", flush=True)
    b = ob.rhs_planewave([0, 0, 1.0], [1.0, 0, 0])
    xo, io = oracle_gmres(ob.apply, b, ob.block_preconditioner(), tol=1e-11, restart=200)
    pb = gpu.IbcProblem(q, 1.0, Z, order=22, depth=3, order32=10)
    bg = torch.from_numpy(b).cuda().unsqueeze(0)
    x, info = pb.solve(bg, tol=1e-11, restart=200, maxit=600)
    print("its gpu", info["iterations"], "oracle", io["iterations"], "err", _rel(x.cpu().numpy()[0], xo))
    assert info["residual"] <= 1e-11 and _rel(x.cpu().numpy()[0], xo) <= 1e-6
    assert abs(info["iterations"] - io["iterations"]) <= 3
    xm, im = pb.solve(bg, tol=1e-8, mixed=True, inner_tol=1e-3)
    assert im["residual"] <= 1e-8 and _rel(xm.cpu().numpy()[0], xo) <= 1e-6
    s = q["points"]
    E, _ = mie.impedance_fields(s / np.linalg.norm(s, axis=1, keepdims=True), 1.0, 1.0, Z)
    print("vs impedance-sphere Mie", _rel(xm.cpu().numpy()[0], E))
    assert _rel(xm.cpu().numpy()[0], E) <= 0.12
    # adjoint solve against the oracle's
    c = complex_normal((q["points"].shape[0], 3), 132)
    ao, _ = oracle_gmres(ob.apply_adjoint, c, ob.block_preconditioner(adjoint=True), tol=1e-11, restart=200)
    xa, ia = pb.solve(torch.from_numpy(c).cuda().unsqueeze(0), tol=1e-11, restart=200, maxit=600, adjoint=True)
    assert _rel(xa.cpu().numpy()[0], ao) <= 1e-6
    pb.close()


def test_group_with_ibc_and_dielectric_members(gpu):
    """An IBC torus and a dielectric sphere in one gmres_solve_group call, each
    bit-identical to its own solve."""
    qt = nystrom3(torus(1.0, 0.3, 24, 8))
    qs = nystrom3(icosphere(4))
    pi = gpu.IbcProblem(qt, 1.5, 0.1 + 0.1j, order=14, depth=3, order32=8)
    pd = gpu.BemProblem(qs, 1.0, 2.25, order=14, depth=3, order32=8)
    ri = pi.rhs_planewave([0.0, 0.6, 0.8], [1.0, 0.0, 0.0])
    rd = pd.rhs_planewave([0.0, 0.0, 1.0], [0.0, 1.0, 0.0])
    xs, infos = gpu.solve_group([pi, pd], [ri, rd], tol=1e-8, mixed=True, inner_tol=1e-3)
    for pb, r, x, inf in zip((pi, pd), (ri, rd), xs, infos):
        x1, i1 = pb.solve(r, tol=1e-8, mixed=True, inner_tol=1e-3)
        assert inf["residual"] <= 1e-8 and torch.equal(x, x1)
    pi.close()
    pd.close()
