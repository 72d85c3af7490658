"""The autotuner's choices, checked against the oracle (needs an MI355X)."""

import numpy as np
import pytest

from oracle.corrections import self_blocks
from oracle.direct import apply_corrections
from oracle.native import point_sum_c
from synthetic import icosphere, nystrom3

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tune():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1211_7177_amd import autotune
    return autotune


@pytest.fixture(scope="module")
def sphere():
    return nystrom3(icosphere(8))          # 1280 triangles, 3840 nodes


def test_tune_matvec_picks_fastest_plan_within_tolerance(tune, sphere):
    q, k, tol = sphere, 1.5, 1e-3
    print("tune_matvec sphere 3840 nodes", flush=True)
    best, table = tune.tune_matvec(q, k, tol, depths=(3,), orders=(3, 5, 8), translates=("fp32", "bf16x3"),
                                   reps=5)
    for r in table:
        print(r)
    assert len(table) == 6 and best is not None
    assert best["ok"] and best["ms"] == min(r["ms"] for r in table if r["ok"])
    for tr in ("fp32", "bf16x3"):
        errs = [r["err"] for r in table if r["translate"] == tr]
        assert errs[2] < errs[0]                        # order 8 beats order 3
    # the winner's own error against the oracle's direct sum (independent of the reference plan)
    from paper_1211_7177_amd._abi import Plan
    n = q["points"].shape[0]
    rng = np.random.default_rng(3)
    a = (rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))) / np.sqrt(2)
    b = (rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))) / np.sqrt(2)
    P = Plan(q["points"], q["normals"], q["weights"], k, best["order"], depth=best["depth"], precision="fp32",
             translate=best["translate"], point_tri=q["point_tri"], tri_vertices=q["tri_vertices"])
    y = P.matvec(torch.from_numpy(a).to(torch.complex64).cuda(),
                 torch.from_numpy(b).to(torch.complex64).cuda()).cpu().numpy()
    P.close()
    rows = np.arange(0, n, 7)
    ref = point_sum_c(q["points"], q["normals"], q["weights"], q["point_tri"], k, a, b, rows=rows)
    blk = self_blocks(q["points"], q["normals"], q["point_tri"], q["tri_vertices"], k, mode="linear")
    ref = ref + apply_corrections(q["normals"], q["point_tri"], blk, a, b, rows=rows)
    err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
    print("winner vs oracle", err)
    assert err <= 2 * tol


def test_tune_solve_reaches_tolerance(tune, sphere):
    print("tune_solve sphere 3840 nodes", flush=True)
    best, table = tune.tune_solve(sphere, 1.0, 2.25, [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], tol=1e-8,
                                  orders32=(5, 8), translates=("fp32",), inner_tols=(1e-3, 1e-2), order64=20,
                                  depth=3, modes=("refine", "nested"))
    for r in table:
        print(r)
    assert len(table) == 8 and best is not None
    assert all(r["ok"] for r in table if r["mode"] == "nested")
    assert best["residual"] <= 1e-8
    assert best["s"] == min(r["s"] for r in table if r["ok"])


def test_tune_solve_over_depths(tune, sphere):
    """The depth dimension: depths 2 and 3 of the 3840-node sphere, each row
    carrying the plans' actual depth, both reaching the tolerance, the winner
    the fastest."""
    print("tune_solve over depths", flush=True)
    best, table = tune.tune_solve(sphere, 1.0, 2.25, [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], tol=1e-8, orders32=(5,),
                                  translates=("fp32",), inner_tols=(1e-2,), order64=20, depths=(2, 3))
    for r in table:
        print(r)
    assert [r["depth"] for r in table] == [2, 3]
    assert all(r["ok"] for r in table) and best["s"] == min(r["s"] for r in table)
