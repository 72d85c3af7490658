"""Measured choice of the FP32 operator and inner-solve schedule.

Two levels, both timing real launches on the current device through the C ABI
(no model of the hardware):

* `tune_matvec` ranks FP32 plans of one wavenumber (octree depth, expansion
  order, translation kernel) by time per product, keeping those whose product
  on a seeded density stays within `tol` (relative 2-norm) of an FP64
  reference plan of high order.
* `tune_solve` ranks whole mixed-precision solves of one scatterer (octree
  depth, FP32 order, translation kernel, inner tolerance) by time to the FP64
  residual `tol`, since a cheaper but coarser inner operator can cost
  refinement steps.

Each returns the winning candidate and the full table.
"""

import itertools
import time

import numpy as np
import torch

from ._abi import Plan
from .solver import BemProblem


def _seeded_density(n, seed, dtype):
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((2, n, 3)) + 1j * rng.standard_normal((2, n, 3))) / np.sqrt(2.0)
    t = torch.from_numpy(z).to(dtype).cuda()
    return t[0].contiguous(), t[1].contiguous()


def _time_calls(fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_matvec(nodes, k, tol, depths=(0,), orders=(4, 5, 6, 8), translates=("fp32", "bf16x3"), ref_order=16,
                ref_depth=0, reps=20, seed=12117177, corr="linear"):
    """Fastest FP32 plan within `tol` of the FP64 reference product.

    Returns (best, table): each table row is a dict with depth, order,
    translate, ms (per product), err (relative to the reference), ok."""
    kw = dict(point_tri=nodes["point_tri"], tri_vertices=nodes["tri_vertices"], corr=corr)
    pts, nrm, w = nodes["points"], nodes["normals"], nodes["weights"]
    n = pts.shape[0]
    a64, b64 = _seeded_density(n, seed, torch.complex128)
    ref = Plan(pts, nrm, w, k, ref_order, depth=ref_depth, **kw)
    y_ref = ref.matvec(a64, b64)
    ref.close()
    a32, b32 = a64.to(torch.complex64), b64.to(torch.complex64)
    table = []
    for depth, order, tr in itertools.product(depths, orders, translates):
        P = Plan(pts, nrm, w, k, order, depth=depth, precision="fp32", translate=tr, **kw)
        y = P.matvec(a32, b32).to(torch.complex128)
        err = (torch.linalg.vector_norm(y - y_ref) / torch.linalg.vector_norm(y_ref)).item()
        ms = _time_calls(lambda: P.matvec(a32, b32), reps)
        table.append({"depth": P.info()["depth"], "order": order, "translate": tr, "ms": ms, "err": err,
                      "ok": err <= tol})
        P.close()
    ok = [r for r in table if r["ok"]]
    best = min(ok, key=lambda r: r["ms"]) if ok else None
    return best, table


def tune_solve(nodes, k0, eps, rhs_dir, rhs_pol, tol=1e-6, orders32=(4, 5, 6), translates=("bf16x3", "fp32"),
               inner_tols=(5e-3,), order64=16, depth=0, restart=150, reps=1, modes=("refine",), depths=None):
    """Fastest mixed-precision solve configuration reaching the residual `tol`.
    modes: "refine" (FP32 inner solves inside FP64 refinement) and/or "nested"
    (FP64 fGMRES preconditioned by FP32 fGMRES cycles of at most 100 steps).
    depths: octree depths to try (0 picks one from the node count); default
    the single `depth`.

    Returns (best, table): each row holds depth (the plans' actual depth),
    mode, order32, translate, inner_tol, s (seconds per solve, the mean of
    `reps` solves after one untimed solve), iterations, refinements, fallback,
    residual, ok."""
    table = []
    for dep, order32, tr in itertools.product(depths if depths is not None else (depth,), orders32, translates):
        pb = BemProblem(nodes, k0, eps, order=order64, depth=dep, order32=order32, translate32=tr)
        actual = pb.p0.info()["depth"]
        rhs = pb.rhs_planewave(rhs_dir, rhs_pol)
        for mode, itol in itertools.product(modes, inner_tols):
            def run():
                if mode == "nested":
                    return pb.solve(rhs, tol=tol, mixed="nested", inner_tol=itol, inner_maxit=100, restart=restart,
                                    maxit=3000, raise_on_noconv=False)
                return pb.solve(rhs, tol=tol, mixed=True, inner_tol=itol, restart=restart, maxit=3000,
                                raise_on_noconv=False)
            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                _, info = run()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            table.append({"depth": actual, "mode": mode, "order32": order32, "translate": tr, "inner_tol": itol,
                          "s": dt,
                          "iterations": info["iterations"], "refinements": info["refinements"],
                          "fallback": info["fp64_fallback"], "residual": info["residual"],
                          "ok": info["residual"] <= tol})
        pb.close()
    ok = [r for r in table if r["ok"]]
    best = min(ok, key=lambda r: r["s"]) if ok else None
    return best, table
