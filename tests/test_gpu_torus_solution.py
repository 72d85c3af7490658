"""Solution accuracy on the 60k-node torus (R = 1, r = 0.3, 20,000 triangles,
eps = -15 + 1i, k0 = 4, depth 5): the GPU's plain FP64 solve and its mixed
FP32/FP64 solve against the oracle's own fGMRES solution of the same direct-sum
system (written by tests/golden/make_torus_oracle_solution.py to a residual of
1e-10), relative L2 over all 6N unknowns (needs an MI355X)."""

import json
import os

import numpy as np
import pytest

from synthetic import CONFIGS, config_mesh, nystrom3, plane_waves, seed_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "torus60k_oracle_solution.npy")
META = os.path.join(os.path.dirname(__file__), "golden", "torus60k_oracle_solution.json")
# FP64 operator for the solution's 1e-6: orders per level for 1e-9 (forward
# error ~ condition number x operator error)
TOL64 = 1e-9
SOLVE_TOL = 1e-9


@pytest.fixture(scope="module")
def torus_problem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLDEN):
        pytest.skip("the oracle's torus solution has not been written (tests/golden/make_torus_oracle_solution.py)")
    from paper_1211_7177_amd.solver import BemProblem
    with open(META) as f:
        meta = json.load(f)
    assert meta["true_relative_residual"] <= 1e-9
    cfg = CONFIGS[2]
    nodes = nystrom3(config_mesh(2))
    pb = BemProblem(nodes, cfg["k0"], cfg["eps"], order=0, depth=cfg["depth"], order32=5, tol=TOL64)
    d, pol = plane_waves(1, seed_for(2, "dirs"), seed_for(2, "pols"))
    yield pb, pb.rhs_planewave(d, pol), np.load(GOLDEN, allow_pickle=False)
    pb.close()


def _rel(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def test_fp64_solution_within_1e6_of_oracle_solution(torus_problem):
    pb, rhs, xo = torus_problem
    print("torus fp64 solve, orders", pb.p0.info()["order_level"], flush=True)
    x, info = pb.solve(rhs, tol=SOLVE_TOL, restart=300, maxit=3000)
    err = _rel(x[0].cpu().numpy(), xo)
    print("torus fp64: %d iterations, residual %.2e, forward error vs oracle %.3e" % (
        info["iterations"], info["residual"], err), flush=True)
    assert err <= 1e-6


def test_mixed_solution_within_1e6_of_oracle_solution(torus_problem):
    pb, rhs, xo = torus_problem
    x, info = pb.solve(rhs, tol=SOLVE_TOL, mixed=True, inner_tol=5e-3, restart=150, maxit=3000)
    err = _rel(x[0].cpu().numpy(), xo)
    print("torus mixed: %d iterations, %d refinements, residual %.2e, forward error vs oracle %.3e" % (
        info["iterations"], info["refinements"], info["residual"], err), flush=True)
    assert err <= 1e-6
