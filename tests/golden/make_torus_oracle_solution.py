"""Writes the oracle's solution of the 60k-node torus system (test infrastructure).

The system is the 6N BEM system of the silver-like torus (R = 1, r = 0.3,
200 x 50 x 2 triangles, 60,000 nodes, eps = -15 + 1i, k0 = 4) for the seeded
plane wave of that configuration (Sec. 2.1, eqs. 2.9-2.13), right-preconditioned
by the per-node self blocks (Sec. 3.1, eq. 3.2) and solved by the oracle's own
fGMRES on the direct-sum operator to a relative residual of 1e-10.  Only
`oracle/` and the seeded input generators run here; nothing of the GPU library.

Output: `torus60k_oracle_solution.npy` (c128[60000, 6], user node order) beside
this file and a small JSON record of the run.  The iterate is saved after every
restart cycle, so an interrupted run keeps its last cycle.

Run: python tests/golden/make_torus_oracle_solution.py [--threads T]
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "torus60k_oracle_solution.npy")
META = os.path.join(HERE, "torus60k_oracle_solution.json")
TOL = 1e-10
RESTART = 300


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    if args.threads:
        os.environ["OMP_NUM_THREADS"] = str(args.threads)
    import numpy as np
    from oracle.bem import BemProblem
    from oracle import gmres as og
    from synthetic import CONFIGS, config_mesh, nystrom3, plane_waves, seed_for

    cfg = CONFIGS[2]
    nodes = nystrom3(config_mesh(2))
    d, pol = plane_waves(1, seed_for(2, "dirs"), seed_for(2, "pols"))
    t0 = time.time()
    ob = BemProblem(nodes, cfg["k0"], cfg["eps"])
    b = ob.rhs_planewave(d[0], pol[0])
    P = ob.block_preconditioner()
    print("problem built in %.1f s, n = %d" % (time.time() - t0, ob.n), flush=True)

    state = {"applies": 0, "t0": time.time()}

    def A(x):
        state["applies"] += 1
        if state["applies"] % 10 == 0:
            print("apply %d, %.0f s" % (state["applies"], time.time() - state["t0"]), flush=True)
        return ob.apply(x)

    x = None
    its = 0
    res = None
    # restart cycles one by one so that each cycle's iterate is kept on disk
    while True:
        x, info = og.gmres_solve(A, b, P, tol=TOL, restart=RESTART, maxit=RESTART, x0=x)
        its += info["iterations"]
        res = info["residual"]
        np.save(OUT, x)
        meta = {"config": "torus_R1_r0.3_20000tri_60000nodes_eps-15+1i_k0_4", "self_blocks": "linear",
                "rhs": "plane wave, seeded direction/polarisation of configuration 2", "tol": TOL,
                "restart": RESTART, "iterations": its, "true_relative_residual": res,
                "applies": state["applies"], "seconds": time.time() - state["t0"]}
        with open(META, "w") as f:
            json.dump(meta, f, indent=1)
        print("cycle done: %d iterations, residual %.3e" % (its, res), flush=True)
        if res <= TOL or its >= 3000:
            break


if __name__ == "__main__":
    main()
