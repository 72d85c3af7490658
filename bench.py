"""Benchmark: FMM matvecs/s and GMRES solves/s at 1e-6 relative error, FP32 against plain FP64,
on one MI355X.

Headline workload: the large PEC-like prolate ellipsoid (semi-axes 4:1:1, 1,003,520 triangles, 3,010,560 nodes,
18.1M unknowns, eps = -1e4 + 1e2 i, k0 = 40 along the minor semi-axis a = 1, octree depth 8).  One timed step is
the FP32 fast-multipole product of both wavenumbers on seeded complex64 densities: the exterior k0 = 40 plan
(orders per level from the leaves to level 2, rotation / coaxial translations) and the local-only interior plan
(k1 = 20 + 4000i); gather, P2M, M2M, M2L, L2L, L2P, P2P and the FP64 self-triangle corrections.  Plans are
built from host arrays and the densities are resident in HBM before timing starts.  Beside it: the FP64
products, their accuracy against the oracle on sampled rows, a full mixed-precision fGMRES solve of the
18.1M-unknown system, the roofline of the near field and the M2L translations, and the oracle's direct sum
timed on the host cores.  The 60k-node torus section compares whole solves (FP32 inner / FP64 refinement
against plain FP64) at equal accuracy.

Prints one JSON line.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp64_TF": 78.6, "fp32_TF": 157.3, "bf16_TF": 2500.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed FP32 products of the large-ellipsoid workload")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--c5-tol32", type=float, default=1e-4, help="FP32 plans: accuracy the per-level orders target")
    ap.add_argument("--c5-tol64", type=float, default=1e-6, help="FP64 plans: accuracy the per-level orders target")
    ap.add_argument("--c5-rows", type=int, default=1024, help="seeded oracle rows of the large-ellipsoid checks")
    ap.add_argument("--c5-solve-s", type=float, default=45.0,
                    help="wall-clock budget (s) of the large-ellipsoid solve (0: skip the solve)")
    ap.add_argument("--c5-solve-chunk", type=int, default=1000,
                    help="Krylov iterations per call of the large-ellipsoid solve (progress line after each)")
    ap.add_argument("--skip-torus", action="store_true", help="skip the 60k-node torus solve comparison")
    ap.add_argument("--torus-steps", type=int, default=3)
    ap.add_argument("--torus-warmup", type=int, default=1)
    ap.add_argument("--order64", type=int, default=0,
                    help="torus FP64 plans: fixed order (> 0) or orders per level for --tol64 (<= 0)")
    ap.add_argument("--tol64", type=float, default=1e-8, help="torus FP64 plans with orders per level: accuracy")
    ap.add_argument("--order32", type=int, default=5)
    ap.add_argument("--tol", type=float, default=1e-8,
                    help="torus solves: relative FP64 residual (1e-8 with the 1e-8 FP64 operator puts both timed "
                         "solutions within 1e-6 of the converged discrete solution)")
    ap.add_argument("--inner-tol", type=float, default=5e-3)
    ap.add_argument("--restart", type=int, default=150, help="Krylov basis size (inner solves and the FP64 solve)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1500, help="seeded rows of the oracle residual check")
    ap.add_argument("--cpu-sample-rows", type=int, default=0,
                    help="target rows of the timed oracle apply (0: all rows, one full BEM application)")
    ap.add_argument("--skip-fp64-solve", action="store_true")
    ap.add_argument("--skip-adjoint-solve", action="store_true")
    ap.add_argument("--dimer", action="store_true",
                    help="also time the gold-dimer optical-force workload from mesh to force")
    ap.add_argument("--c3", action="store_true", help="also run the batched three-mesh section (several minutes)")
    ap.add_argument("--c3-rhs", type=int, default=4, help="plane waves per mesh of the three-mesh section "
                    "(the configuration's 64: about 200 GB and many minutes for the sphere)")
    ap.add_argument("--c3-fp64-rhs", type=int, default=2, help="waves per mesh of the plain FP64 comparison")
    ap.add_argument("--split-ring", action=argparse.BooleanOptionalAction, default=True,
                    help="the split-ring solves, product rates and vertex gradient (49k triangles; about 30 s)")
    ap.add_argument("--translate32", choices=["fp32", "bf16x3"], default="bf16x3")
    ap.add_argument("--batch", type=int, default=8,
                    help="also time one lockstep solve of this many plane waves (0: skip)")
    ap.add_argument("--inner-reorth", action="store_true",
                    help="second (DGKS-triggered) Gram-Schmidt pass in the inner FP32 solves too")
    ap.add_argument("--serial", action="store_true",
                    help="run the k0 and k1 FMM products of each application one after the other (one stream)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the octree depth, FP32 order and translation kernel by timing whole solves first "
                         "(autotune.tune_solve)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay the two FMM products from a captured HIP graph (default: eager launches)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device-to-device copy (calibrates FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def sr_pairs(info):
    """Far-field (S|R) box pairs of one matvec, all levels."""
    return sum(info["m2l_pairs"])


def sr_flops(info, nrhs=1):
    """Algorithmic flops of one matvec's S|R translations: a complex (p^2 x p^2)
    by (p^2 x 3 nrhs) product per pair, 8 flops per complex multiply-add, i.e.
    24 p^4 per pair and right-hand side."""
    p2 = info["order"] ** 2
    return 8.0 * p2 * p2 * 3 * nrhs * sr_pairs(info)


def sr_bytes(info, csize, nrhs=1):
    """Algorithmic HBM bytes of one matvec's S|R translations: each pair reads
    its source block (3 nrhs columns of p^2 coefficients) and writes its slot
    once; the operators (per offset and level) are read once per job and are
    not counted."""
    return 2.0 * 3 * nrhs * info["order"] ** 2 * csize * sr_pairs(info)


P2P_FLOPS_PER_PAIR = 150.0   # ~45 geometry (r, 1/R, g, grad g) + ~105 per rhs; plus rsqrt, sincos, exp


def p2p_pairs(info, n):
    """Near (target, source) pairs the method must evaluate: the plan's count
    less the 3 same-triangle pairs of every target (computed as masked)."""
    return info["p2p_pairs"] - 3 * n


CSRC = os.path.join(ROOT, "paper_1211_7177_amd", "csrc")
# kernel -> (committed FETCH_SIZE / WRITE_SIZE summary, source file the kernel is built from)
TRAFFIC_FILES = {
    "k_translate_bf3 S|R": (os.path.join(ROOT, "profiles", "translate_bf3_sr_torus60k_p5_hbm_traffic.md"),
                            os.path.join(CSRC, "matvec.hip")),
    "k_p2p32": (os.path.join(ROOT, "profiles", "p2p32_torus60k_hbm_traffic.md"), os.path.join(CSRC, "matvec.hip")),
    "k_p2p32 c5": (os.path.join(ROOT, "profiles", "p2p32_ellipsoid1M_hbm_traffic.md"), os.path.join(CSRC, "matvec.hip")),
    "k_hf_m2l_w c5": (os.path.join(ROOT, "profiles", "hf_m2l_w_ellipsoid1M_level8_hbm_traffic.md"),
                      os.path.join(CSRC, "hf.hip")),
}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from its committed FETCH_SIZE /
    WRITE_SIZE summary, or None when there is none or the kernel source has
    changed since the counters were taken."""
    try:
        meta = {}
        summary, src = TRAFFIC_FILES[kernel]
        with open(summary) as f:
            for line in f:
                if ":" in line and line.startswith("    "):
                    k, v = line.strip().split(":", 1)
                    meta[k.strip()] = v.strip()
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if meta.get("kernel") != kernel or meta.get("source_sha256") != sha:
            return None
        return float(meta["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def split_ring_section(log):
    """The split-ring workload (square ring, side 1, width 0.2, thickness 0.1, gap 0.2; eps = -15 + 1i,
    k0 = pi/2, wave along +z polarised across the gap): a nested solve, a plain FP64 solve and a nested adjoint
    solve to 1e-8 (restart 400), the forward and adjoint FMM product rates of its k0 plans, and the gradient of
    the far-field C_sca at every vertex.  Runs after the timed solves of the main workload, outside their timed
    region."""
    import torch
    from synthetic import config_mesh, nystrom3
    from paper_1211_7177_amd.solver import BemProblem
    mesh = config_mesh(4)
    q = nystrom3(mesh)
    n = q["points"].shape[0]
    pb = BemProblem(q, np.pi / 2, complex(-15.0, 1.0), order=16, order32=5, translate32="bf16x3")
    b = pb.rhs_planewave([0.0, 0.0, 1.0], [0.0, 1.0, 0.0])
    nested = dict(mixed="nested", inner_tol=1e-2, inner_maxit=100)
    out = {"workload": "split_ring_%dtri_%dnodes_eps-15+1i_k0pi/2" % (len(mesh.triangles), n),
           "depth": pb.p0.info()["depth"], "tol": 1e-8, "restart": 400}
    for name, kw in (("nested_solve", nested), ("fp64_solve", {}), ("nested_adjoint_solve", dict(nested, adjoint=True))):
        pb.solve(b, tol=1e-2, restart=400, maxit=4000, raise_on_noconv=False, **kw)      # allocations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = pb.solve(b, tol=1e-8, restart=400, maxit=4000, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"s": dt, "iterations": info["iterations"], "outer": info["refinements"],
                     "residual": info["residual"]}
        log("split ring", name, out[name])
    out["speedup_nested_vs_fp64"] = out["fp64_solve"]["s"] / out["nested_solve"]["s"]
    rates = {}
    for tag, plan, cdt in (("fp64", pb.p0, torch.complex128), ("fp32", pb.p0_32, torch.complex64)):
        a = torch.randn(1, n, 3, dtype=cdt, device="cuda")
        y = plan.matvec(a, a)
        plan.matvec_adjoint(y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            plan.matvec(a, a, out=y)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(10):
            plan.matvec_adjoint(y)
        torch.cuda.synchronize()
        rates[tag] = {"matvecs_per_s": 10 / (t1 - t0), "adjoint_matvecs_per_s": 10 / (time.perf_counter() - t1)}
    out["fmm_k0_plan"] = rates
    pb.close()
    # dC_sca/dv at every vertex (far-field form): one forward and one adjoint solve (nested, 1e-12), the
    # point-sum derivative passes at k0 and k1, the explicit terms and the self-triangle block differences
    from paper_1211_7177_amd.shape import cross_section_and_vertex_gradient
    stats = {}
    t0 = time.perf_counter()
    C, gV, _ = cross_section_and_vertex_gradient(mesh.vertices, mesh.triangles, np.pi / 2, complex(-15.0, 1.0),
                                                 [0.0, 0.0, 1.0], [0.0, 1.0, 0.0], order=16, order32=5, tol=1e-12,
                                                 restart=400, functional="far", solve_kw=nested, stats=stats)
    dt = time.perf_counter() - t0
    out["vertex_gradient"] = {
        "vertices": int(len(mesh.vertices)), "C_sca_far": C, "s": dt, "phases_s": stats,
        "translation_residual": float(np.linalg.norm(gV.sum(axis=0)) / np.abs(gV).sum()),
        # two passes (target role, source role) over all n^2 node pairs at each of k0 and k1
        "pair_evaluations_per_s": 4.0 * n * n / stats["pairs_s"],
    }
    log("split ring vertex gradient", out["vertex_gradient"])
    return out


def c3_section(args, log, rows=400):
    """The batched workload of three uneven meshes: an ellipsoid (1.5, 1, 0.75) of 24,000 nodes at k0 = 2,
    eps 2.25; a torus of 90,000 nodes at k0 = 5, eps -15 + 1i; a sphere of 245,760 nodes at k0 a = 10, eps 2.25.
    args.c3_rhs plane waves per mesh (seeded directions and polarisations) are solved in lockstep through plans
    built for that many columns, the three meshes in one `gmres_solve_group` call (one host thread and stream
    each), to a relative FP64 residual of 1e-8:
      * FP32/batched: FP32 inner solves (FP32 plans at orders per level for 1e-4) inside FP64 iterative
        refinement (switching to nested mode if a refinement stalls);
      * plain FP64: FP64 fGMRES on the first args.c3_fp64_rhs waves of each mesh (its per-wave rate);
    the FP64 operator at orders per level for 1e-8 in both.  Equal accuracy: the two solutions of the shared
    waves, and the oracle's direct-sum residual of wave 0 of each mesh on `rows` seeded rows."""
    import torch
    from synthetic import CONFIGS, config_mesh, nystrom3, plane_waves, seed_for
    from paper_1211_7177_amd.solver import BemProblem, solve_group
    nrhs, n64 = args.c3_rhs, min(args.c3_fp64_rhs, args.c3_rhs)
    pbs, rhs, meshes = [], [], []
    t0 = time.perf_counter()
    for cfg in (31, 32, 33):
        c = CONFIGS[cfg]
        q = nystrom3(config_mesh(cfg))
        pb = BemProblem(q, c["k0"], c["eps"], order=0, tol=1e-8, order32=0, tol32=1e-4, nrhs_max=nrhs,
                        depth=c["depth"])
        d, pol = plane_waves(nrhs, seed_for(cfg, "dirs"), seed_for(cfg, "pols"))
        pbs.append(pb)
        rhs.append(pb.rhs_planewave(d, pol))
        meshes.append({"name": c["name"], "nodes": q["points"].shape[0], "k0": c["k0"], "eps": str(c["eps"]),
                       "depth": c["depth"], "fp64_orders": pb.p0.info()["order_level"], "q": q})
    torch.cuda.synchronize()
    log("c3: problems built in %.1f s" % (time.perf_counter() - t0))
    out = {"nrhs_per_mesh": nrhs, "fp64_nrhs_per_mesh": n64, "tol": 1e-8,
           "fp32": "orders per level for 1e-4, FP32 Krylov, restart 200",
           "why_fp32_orders": "order-8 split-BF16 plans (5.9e-4 from the FP64 operator on the sphere at k0 a = 10) "
                              "left the refinement stalling; per-level orders put the FP32 operator within 1e-6",
           "fp64_operator": "orders per level for 1e-8"}
    sols = {}
    # FP32/batched: all waves of the three meshes in one group call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos = solve_group(pbs, rhs, tol=1e-8, maxit=3000, raise_on_noconv=False, mixed=True, inner_tol=5e-3,
                            restart=200)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sols["fp32_batched"] = xs
    res = [{"iterations": i["iterations"], "refinements": i["refinements"], "residual": i["residual"],
            "fp64_fallback": i.get("fp64_fallback")} for i in infos]
    out["fp32_batched"] = {"s": dt, "rhs_solves_per_s": 3 * nrhs / dt, "meshes": res}
    log("c3 fp32_batched: %d waves per mesh in %.1f s" % (nrhs, dt), res)
    # plain FP64: mesh by mesh, in calls of 300 iterations resuming from the iterate (a progress line each)
    sols["fp64"] = []
    res, tot = [], 0.0
    for m, pb, b in zip(meshes, pbs, rhs):
        bb = b[:n64].contiguous()
        x, its = None, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            x, info = pb.solve(bb, tol=1e-8, restart=300, maxit=300, x0=x, raise_on_noconv=False)
            torch.cuda.synchronize()
            its += info["iterations"]
            log("c3 fp64 %s: %d iterations, residual %.2e, %.1f s" % (m["name"], its, info["residual"],
                                                                      time.perf_counter() - t0))
            if info["residual"] <= 1e-8 or its >= 6000:
                break
        dtm = time.perf_counter() - t0
        tot += dtm
        sols["fp64"].append(x)
        res.append({"iterations": its, "residual": info["residual"], "s": dtm})
    out["fp64"] = {"s": tot, "rhs_solves_per_s": 3 * n64 / tot, "meshes": res,
                   "note": "meshes one after the other, %d waves each in lockstep" % n64}
    # equal accuracy
    acc = []
    for m, pb, x32, x64, b in zip(meshes, pbs, sols["fp32_batched"], sols["fp64"], rhs):
        a = {"solution_rel_diff_shared_waves": float(torch.linalg.norm((x32[:n64] - x64).flatten()) /
                                                    torch.linalg.norm(x64.flatten()))}
        for name, x in (("fp32_batched", x32), ("fp64", x64)):
            a["oracle_residual_rows_" + name] = oracle_residual_rows(m["q"], float(np.real(pb.k0)), pb.eps,
                                                                      x[0].cpu().numpy(), b[0].cpu().numpy(), rows)
        acc.append(a)
    out["accuracy"] = acc
    out["meshes"] = [{k: v for k, v in m.items() if k != "q"} for m in meshes]
    out["speedup_per_rhs_fp32_batched_vs_fp64"] = out["fp32_batched"]["rhs_solves_per_s"] / out["fp64"]["rhs_solves_per_s"]
    log("c3 accuracy", acc, "speedup per wave %.1f" % out["speedup_per_rhs_fp32_batched_vs_fp64"])
    for pb in pbs:
        pb.close()
    return out


def dimer_section(log, nu=17):
    """The optical-force workload of the paper's appendix D: two gold spheres (radius 100 nm, a 250 nm gap along x,
    Drude gold at 500 nm; length unit 100 nm), icospheres of 20 nu^2 triangles each (nu = 17: 11,560 triangles in
    all, against the paper's 11,904 elements), a wave along +z polarised along x, solved to the paper's residual
    1e-3, then the time-averaged force on the left sphere from the Maxwell stress tensor on a sphere around it.
    Reports the wall time from mesh to force (plans built inside it) and the force for 1 mW/um^2."""
    import torch
    from synthetic import icosphere, nystrom3, union
    from paper_1211_7177_amd import materials, postprocess as pp
    from paper_1211_7177_amd.solver import MultiBemProblem
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m, treg = union([icosphere(nu), icosphere(nu)], [[-2.25, 0.0, 0.0], [2.25, 0.0, 0.0]])
    q = nystrom3(m)
    reg = treg[q["point_tri"]]
    eps = complex(materials.gold_drude(500e-9))
    k0 = float(materials.wavenumber(500e-9, 100e-9))
    pb = MultiBemProblem(q, reg, k0, [eps, eps], order=16, order32=6, translate32="bf16x3")
    d, pol = [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]
    x, info = pb.solve(pb.rhs_planewave(d, pol), tol=1e-3, restart=200, maxit=2000, mixed=True, inner_tol=5e-2)
    F = pp.optical_force(pb, x, d, pol, k0, 1.6, center=[-2.25, 0.0, 0.0], nt=32, nph=64)[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": "gold_dimer_r100nm_gap250nm_lambda500nm_%dtri_%dnodes" % (len(m.triangles), q["points"].shape[0]),
           "eps_gold": str(eps), "k0_per_100nm": k0, "tol": 1e-3, "seconds_mesh_to_force": dt,
           "iterations": info["iterations"], "refinements": info["refinements"], "residual": info["residual"],
           "force_left_sphere_N_at_1mW_per_um2": [float(v) for v in materials.force_newtons(F, 1e9, 1e-7)]}
    # outside the timed part: the same force from a solve converged to 1e-6
    x6, _ = pb.solve(pb.rhs_planewave(d, pol), tol=1e-6, restart=200, maxit=2000, mixed=True, inner_tol=5e-3)
    F6 = pp.optical_force(pb, x6, d, pol, k0, 1.6, center=[-2.25, 0.0, 0.0], nt=32, nph=64)[0]
    out["force_rel_diff_vs_1e-6_solve"] = float(np.linalg.norm(F - F6) / np.linalg.norm(F6))
    pb.close()
    # the force spectrum of the appendix's figure: F_z on the left sphere from 400 to 700 nm (solves to 1e-3)
    spec = []
    t1 = time.perf_counter()
    for lam_nm in range(400, 701, 20):
        e_l = complex(materials.gold_drude(lam_nm * 1e-9))
        k_l = float(materials.wavenumber(lam_nm * 1e-9, 100e-9))
        pl = MultiBemProblem(q, reg, k_l, [e_l, e_l], order=16, order32=6, translate32="bf16x3")
        xl, il = pl.solve(pl.rhs_planewave(d, pol), tol=1e-3, restart=200, maxit=2000, mixed=True, inner_tol=5e-2)
        Fl = pp.optical_force(pl, xl, d, pol, k_l, 1.6, center=[-2.25, 0.0, 0.0], nt=32, nph=64)[0]
        spec.append([lam_nm, float(materials.force_newtons(Fl, 1e9, 1e-7)[2] * 1e12)])
        pl.close()
    out["force_z_pN_vs_wavelength_nm"] = spec
    out["spectrum_seconds"] = time.perf_counter() - t1
    log("dimer", out)
    return out


def torus_section(args, log):
    """The silver-like torus system (R = 1, r = 0.3, 20,000 triangles, 60,000 nodes, eps = -15 + 1i, k0 R = 4,
    depth 5): timed mixed-precision solves (FP32 FMM and Krylov vectors inside FP64 refinement) against the plain
    FP64 solve, both to a relative FP64 residual of args.tol, with their forward errors against the oracle's own
    solution of the same system when it is present (tests/golden), the FMM product rates and the roofline of the
    FP32 near field and translations."""
    import torch
    from paper_1211_7177_amd.solver import BemProblem
    from synthetic import config_mesh, nystrom3, plane_waves, seed_for, CONFIGS

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = CONFIGS[2]
    mesh = config_mesh(2)
    nodes = nystrom3(mesh)
    n = nodes["points"].shape[0]
    k0, eps, depth = cfg["k0"], cfg["eps"], cfg["depth"]
    d, pol = plane_waves(1, seed_for(2, "dirs"), seed_for(2, "pols"))

    tuned = None
    if args.autotune:
        from paper_1211_7177_amd.autotune import tune_solve
        best, table = tune_solve(nodes, k0, eps, d, pol, tol=args.tol, orders32=(4, 5, 6),
                                 translates=("bf16x3", "fp32"), inner_tols=(args.inner_tol,), order64=args.order64,
                                 depths=(depth - 1, depth, depth + 1), restart=args.restart)
        tuned = {"chosen": best, "table": table}
        log("autotune", best)
        if best is not None:
            args.order32, args.translate32, depth = best["order32"], best["translate"], best["depth"]
    t0 = time.perf_counter()
    pb = BemProblem(nodes, k0, eps, order=args.order64, depth=depth, order32=args.order32, tol=args.tol64,
                    translate32=args.translate32)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    log("plans built in %.2f s" % plan_s)
    if args.graphs:
        pb.use_graphs(True)
    info64 = pb.p0.info()
    info32 = pb.p0_32.info()
    rhs = pb.rhs_planewave(d, pol)

    def step(serial=args.serial):
        return pb.solve(rhs, tol=args.tol, mixed=True, inner_tol=args.inner_tol, restart=args.restart, maxit=2000,
                        serial=serial, inner_reorth=args.inner_reorth)

    for _ in range(args.torus_warmup):
        _, wi = step()
        log("torus warmup solve", wi["iterations"], wi["refinements"], wi["residual"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.torus_steps):
        x, inf = step()
        infos.append(inf)
        log("torus timed solve", inf["iterations"], inf["refinements"], inf["residual"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.torus_steps
    solves_per_s = args.torus_steps / dt
    last = infos[-1]
    # one more solve of the same system with HIP events around the near-field
    # and translation launches of both FP32 plans; the roofline below uses their
    # per-launch averages.  It runs the two products of each application one
    # after the other, so that an event pair brackets its kernel alone, and it
    # is kept out of the timed region.  Two plane-wave right-hand-side kernels
    # (k_rhs_planewave) bracket it so that a kernel trace can be cut to it.
    for p in (pb.p0_32, pb.p1_32):
        p.profile(True, stages=("p2p", "m2l"))
        p.profile_read(reset=True)
    pb.rhs_planewave(d, pol)
    torch.cuda.synchronize()
    step(serial=True)
    torch.cuda.synchronize()
    pb.rhs_planewave(d, pol)
    torch.cuda.synchronize()
    timed = {}
    for p in (pb.p0_32, pb.p1_32):
        for st, (ms, cnt) in p.profile_read(reset=True).items():
            a0, c0 = timed.get(st, (0.0, 0))
            timed[st] = (a0 + ms, c0 + cnt)
        p.profile(False)
    log("profiled solve: stage totals (ms, launches)", {k: v for k, v in timed.items() if v[1]})

    # batched right-hand sides (outside the timed region): one lockstep solve of
    # args.batch seeded plane waves through plans built for that many columns
    batched = None
    if args.batch > 1:
        pbb = BemProblem(nodes, k0, eps, order=args.order64, depth=depth, order32=args.order32, tol=args.tol64,
                         translate32=args.translate32, nrhs_max=args.batch)
        db, pob = plane_waves(args.batch, seed_for(2, "dirs"), seed_for(2, "pols"))
        rb = pbb.rhs_planewave(db, pob)
        pbb.solve(rb, tol=args.tol, mixed=True, inner_tol=args.inner_tol, restart=args.restart, maxit=2000,
                  inner_reorth=args.inner_reorth)
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        _, ib = pbb.solve(rb, tol=args.tol, mixed=True, inner_tol=args.inner_tol, restart=args.restart,
                          maxit=2000, inner_reorth=args.inner_reorth)
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb0
        batched = {"nrhs": args.batch, "rhs_solves_per_s": args.batch / tb, "ms_per_batch": 1e3 * tb,
                   "iterations": ib["iterations"], "refinements": ib["refinements"], "residual": ib["residual"],
                   "speedup_per_rhs_vs_single": (args.batch / tb) / solves_per_s}
        log("batched", batched)
        pbb.close()

    # adjoint solve A^H lam = b of the same system (the backward pass of a gradient), mixed precision with
    # the same options, outside the timed region; one untimed solve first
    adjoint = None
    if not args.skip_adjoint_solve:
        kw_adj = dict(tol=args.tol, mixed=True, inner_tol=args.inner_tol, restart=args.restart, maxit=2000,
                      inner_reorth=args.inner_reorth, adjoint=True)
        pb.solve(rhs, **kw_adj)
        torch.cuda.synchronize()
        ta0 = time.perf_counter()
        _, ia = pb.solve(rhs, **kw_adj)
        torch.cuda.synchronize()
        ta = time.perf_counter() - ta0
        adjoint = {"solves_per_s": 1.0 / ta, "ms_per_solve": 1e3 * ta, "iterations": ia["iterations"],
                   "refinements": ia["refinements"], "residual": ia["residual"]}
        log("adjoint solve", adjoint)

    # plain FP64 solve (reference path) and matvec rates, outside the timed region
    fp64 = None
    if not args.skip_fp64_solve:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x64, inf64 = pb.solve(rhs, tol=args.tol, mixed=False, restart=args.restart, maxit=2000)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        log("fp64 solve %.3f s" % t64, inf64["iterations"], inf64["residual"])
        diff = (torch.linalg.vector_norm(x64 - x) / torch.linalg.vector_norm(x64)).item()
        fp64 = {"solves_per_s": 1.0 / t64, "ms_per_solve": 1e3 * t64, "iterations": inf64["iterations"],
                "bem_applies": inf64["matvecs64"], "residual": inf64["residual"],
                "rel_diff_vs_mixed_solution": diff}
    # forward error of both timed solutions against the oracle's own solution of the same discrete system
    # (fGMRES on the direct-sum operator to 1e-10, written by tests/golden/make_torus_oracle_solution.py)
    forward = None
    ref_path = os.path.join(ROOT, "tests", "golden", "torus60k_oracle_solution.npy")
    if os.path.exists(ref_path):
        xr = np.load(ref_path)
        nr = np.linalg.norm(xr)
        forward = {"mixed": float(np.linalg.norm(x[0].cpu().numpy() - xr) / nr)}
        if fp64 is not None:
            forward["fp64"] = float(np.linalg.norm(x64[0].cpu().numpy() - xr) / nr)
        meta = os.path.join(ROOT, "tests", "golden", "torus60k_oracle_solution.json")
        if os.path.exists(meta):
            with open(meta) as f:
                forward["oracle_solution"] = json.load(f)
        log("forward error against the oracle solution", forward)

    # FMM matvec rates and stage profile (HIP events on the stream the kernels run on)
    rates = {}
    adj_rates = {}
    prof = {}
    for tag, plan, cdt in (("fp64", pb.p0, torch.complex128), ("fp32", pb.p0_32, torch.complex64)):
        a = torch.randn(1, n, 3, dtype=cdt, device=dev)
        b = torch.randn(1, n, 3, dtype=cdt, device=dev)
        y = plan.matvec(a, b)
        torch.cuda.synchronize()
        reps = 10
        t1 = time.perf_counter()
        for _ in range(reps):
            plan.matvec(a, b, out=y)
        torch.cuda.synchronize()
        rates[tag] = reps / (time.perf_counter() - t1)
        plan.matvec_adjoint(y)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            plan.matvec_adjoint(y)
        torch.cuda.synchronize()
        adj_rates[tag] = reps / (time.perf_counter() - t1)
        plan.profile(True)
        plan.profile_read(reset=True)
        for _ in range(reps):
            plan.matvec(a, b, out=y)
        prof[tag] = plan.profile_read(reset=True)
        plan.profile(False)
        log(tag, "matvec/s %.1f adjoint/s %.1f" % (rates[tag], adj_rates[tag]), prof[tag])

    # roofline of the dominant FP32 kernel of the solve (both FP32 plans): the
    # S|R translation kernel (its launches of all levels) or the near field
    inf = info32
    mv32 = timed["p2p"][1]                      # one near-field launch per FP32 matvec
    p2p_ms = timed["p2p"][0]
    tr_ms, tr_launches = timed["m2l"]
    p2p_fl = P2P_FLOPS_PER_PAIR * p2p_pairs(inf, n)
    p2p_tf = p2p_fl / (p2p_ms / mv32 * 1e-3) / 1e12
    tr_fl = sr_flops(inf) * mv32
    tr_by = sr_bytes(inf, 8) * mv32
    tr_tf = tr_fl / (tr_ms * 1e-3) / 1e12
    tr_gbs = tr_by / (tr_ms * 1e-3) / 1e9
    if args.translate32 == "bf16x3":
        tr_name, tr_peak = "k_translate_bf3 S|R (role 1; split-BF16 MFMA, FP32 accumulate)", PEAK["bf16_TF"]
    else:
        tr_name, tr_peak = "k_translate_os S|R (FP32 MFMA)", PEAK["fp32_TF"]
    # below the ridge point (peak flops / HBM bandwidth) the translations are bound by memory
    tr_hbm = tr_fl / tr_by < tr_peak * 1e12 / (PEAK["hbm_GBs"] * 1e9)
    stages_rf = {
        "p2p": {"kernel": "k_p2p32 (near field, FP32 VALU)", "bound": "alu", "achieved": p2p_tf,
                "peak": PEAK["fp32_TF"], "unit": "TFLOP/s", "frac": p2p_tf / PEAK["fp32_TF"], "traffic": None,
                "per_launch_flops": p2p_fl, "avg_launch_ms": p2p_ms / mv32, "launches": mv32,
                "gpairs_per_s": p2p_pairs(inf, n) / (p2p_ms / mv32 * 1e-3) / 1e9},
        "translate": {"kernel": tr_name, "bound": "hbm" if tr_hbm else "mfma",
                      "achieved": tr_gbs if tr_hbm else tr_tf,
                      "peak": PEAK["hbm_GBs"] if tr_hbm else tr_peak,
                      "unit": "GB/s" if tr_hbm else "TFLOP/s",
                      "frac": tr_gbs / PEAK["hbm_GBs"] if tr_hbm else tr_tf / tr_peak, "traffic": None,
                      "per_launch_bytes": tr_by / max(1, tr_launches), "per_launch_flops": tr_fl / max(1, tr_launches),
                      "avg_launch_ms": tr_ms / max(1, tr_launches), "launches": tr_launches,
                      "mfma_view": {"achieved_TFLOPs": tr_tf, "peak_TFLOPs": tr_peak, "frac": tr_tf / tr_peak}},
    }
    stages_rf["translate"]["traffic"] = measured_traffic("k_translate_bf3 S|R") if args.translate32 == "bf16x3" \
        else None
    stages_rf["p2p"]["traffic"] = measured_traffic("k_p2p32")
    dominant = "p2p" if p2p_ms >= tr_ms else "translate"
    roofline = dict(stages_rf[dominant])
    log("roofline", stages_rf)

    ring = split_ring_section(log) if args.split_ring else None
    dimer = dimer_section(log) if args.dimer else None

    # accuracy against the oracle: FP64 direct-sum residual of the GPU solutions on sampled rows
    acc = None
    if not args.no_cpu_baseline:
        b_h = rhs[0].cpu().numpy()
        acc = {"rows": args.cpu_rows,
               "mixed": oracle_residual_rows(nodes, k0, eps, x[0].cpu().numpy(), b_h, args.cpu_rows)}
        if fp64 is not None:
            acc["fp64"] = oracle_residual_rows(nodes, k0, eps, x64[0].cpu().numpy(), b_h, args.cpu_rows)
        log("oracle residual on sampled rows", acc)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(nodes, k0, eps, args.cpu_sample_rows or n,
                           fp64["bem_applies"] if fp64 else last["matvecs64"] + last["matvecs32"])

    out = {
        "solves_per_s": solves_per_s,
        "ms_per_solve": ms_per_step,
        "timed_solves": args.torus_steps,
        "precision": "FP32 FMM (split-BF16 MFMA translations with FP32 accumulation when translate_fp32 is "
                     "bf16x3) and FP32 inner Krylov vectors; FP64 self-triangle corrections, inner products, "
                     "Hessenberg/Givens, residuals and the refinement iterate",
        "config": {"workload": "torus_R1_r0.3_20000tri_60000nodes_eps-15+1i_k0R4_depth5_planewave",
                   "nodes": n, "unknowns": 6 * n, "depth": depth,
                   "order_fp64": info64["order_level"] if args.order64 <= 0 else args.order64, "tol_fp64": args.tol64,
                   "order_fp32": args.order32, "translate_fp32": args.translate32, "tol": args.tol,
                   "restart": args.restart, "inner_tol": args.inner_tol,
                   "inner_gram_schmidt": "two passes (DGKS)" if args.inner_reorth else "one classical pass"},
        "solve": {"iterations": last["iterations"], "refinements": last["refinements"],
                  "bem_applies_fp32": last["matvecs32"], "bem_applies_fp64": last["matvecs64"],
                  "residual": last["residual"], "fp64_fallback": last["fp64_fallback"]},
        "batched": batched,
        "autotune": tuned,
        "fp64_solve": fp64,
        "forward_error_vs_oracle_solution": forward,
        "adjoint_solve": adjoint,
        "split_ring": ring,
        "gold_dimer": dimer,
        "speedup_vs_fp64_solve": (solves_per_s / fp64["solves_per_s"]) if fp64 else None,
        "fmm_matvecs_per_s": rates,
        "fmm_adjoint_matvecs_per_s": adj_rates,
        "unknowns_matvec_per_s": {k: 3 * n * v for k, v in rates.items()},
        "stage_ms_per_matvec": {t: {s: v[0] / 10.0 for s, v in prof[t].items()} for t in prof},
        "plan_s_4plans": plan_s,
        "plan_info_fp64": {k: info64[k] for k in ("nbox", "m2l_pairs", "p2p_pairs", "device_bytes")},
        "oracle_residual_sampled_rows": acc,
        "roofline": roofline,
        "roofline_stages": stages_rf,
        "profiled_solve_kernel_ms": {s: v[0] for s, v in timed.items() if v[1]},
        "cpu_baseline": cpu,
    }
    pb.close()
    return out


def oracle_residual_rows(nodes, k0, eps, x, b, nrows):
    """|b - A x| / |b| over seeded sample rows, A the oracle's direct-sum 6N system."""
    from oracle.corrections import self_blocks
    from oracle.direct import apply_corrections
    from oracle.kernel import wavenumber
    from oracle.native import point_sum_c
    from synthetic import seed_for

    n = nodes["points"].shape[0]
    rows = np.sort(np.random.default_rng(seed_for(2, "rows")).choice(n, nrows, replace=False))
    pts, nrm, w, pt = nodes["points"], nodes["normals"], nodes["weights"], nodes["point_tri"]
    eps = complex(eps)
    k1 = wavenumber(k0, eps)
    phi, psi = x[:, :3], x[:, 3:]
    tphi = phi + ((1 - eps) / eps) * nrm * np.sum(nrm * phi, axis=1, keepdims=True)
    # self-triangle blocks only for the triangles of the sampled rows
    tris = np.unique(pt[rows])
    sub = np.concatenate([np.nonzero(pt == t)[0] for t in tris])
    remap = {t: i for i, t in enumerate(tris)}
    sub_nodes = {"points": pts[sub], "normals": nrm[sub], "point_tri": np.array([remap[t] for t in pt[sub]]),
                 "tri_vertices": nodes["tri_vertices"][tris]}
    where = {g: i for i, g in enumerate(sub)}
    loc = np.array([where[r] for r in rows])

    def op(k, a, bb):
        y = point_sum_c(pts, nrm, w, pt, k, a, bb, rows=rows)
        blk = self_blocks(sub_nodes["points"], sub_nodes["normals"], sub_nodes["point_tri"],
                          sub_nodes["tri_vertices"], k)
        yc = apply_corrections(sub_nodes["normals"], sub_nodes["point_tri"], blk, a[sub], bb[sub])
        return y + yc[loc]

    r0 = 0.5 * phi[rows] + op(k0, phi, -psi)
    r1 = 0.5 * tphi[rows] - op(k1, tphi, -psi)
    ax = np.concatenate([r0, r1], axis=1)
    return float(np.linalg.norm(b[rows] - ax) / np.linalg.norm(b[rows]))


def cpu_baseline(nodes, k0, eps, rows, applies_per_solve):
    """The FP64 oracle's direct-sum BEM apply on a seeded sample of target rows
    (both wavenumbers), scaled to a full apply and to one solve."""
    from oracle.kernel import wavenumber
    from oracle.native import point_sum_c
    from synthetic import complex_normal, seed_for

    n = nodes["points"].shape[0]
    rng = np.random.default_rng(seed_for(2, "rows"))
    sel = np.arange(n) if rows >= n else np.sort(rng.choice(n, rows, replace=False))
    a = complex_normal((n, 3), seed_for(2, "a"))
    b = complex_normal((n, 3), seed_for(2, "b"))
    k1 = wavenumber(k0, eps)
    t0 = time.perf_counter()
    for k in (k0, k1):
        point_sum_c(nodes["points"], nodes["normals"], nodes["weights"], nodes["point_tri"], k, a, b, rows=sel)
    dt = time.perf_counter() - t0
    apply_s = dt * n / len(sel)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": 1.0 / (apply_s * applies_per_solve), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": "direct-sum BEM apply (both wavenumbers, FP64 oracle) on %d of %d target rows, %.2f s, "
                      "scaled by n/rows to one apply (%.1f s) and by the %d applies of one FP64 fGMRES solve" %
                      (len(sel), n, dt, apply_s, applies_per_solve),
            "applies_per_s": 1.0 / apply_s}




def _wsize(p):
    """sum_{n<p} (2n+1)^2: entries of the rotation matrices of degrees below p."""
    return p * (2 * p - 1) * (2 * p + 1) // 3


def _csum(p):
    """sum_{|m|<p} (p-|m|)^2: entries of the coaxial shift of order p."""
    return p * p + (p - 1) * p * (2 * p - 1) // 3


def hf_translation_flops(p):
    """Algorithmic flops of one rotation / coaxial-shift / rotation translation of the 3 channels at order p:
    two real rotations of a complex vector (4 flops per entry) and one complex coaxial shift (8 flops per entry)."""
    return 3 * (8 * _wsize(p) + 8 * _csum(p))


C5_NAME = "prolate_ellipsoid_4x1x1_1003520tri_3010560nodes_eps-1e4+1e2i_k0a40_depth8"


def c5_workload(args, log):
    """The large PEC-like prolate ellipsoid: plans, timed FP32 products, FP64 products, roofline, the oracle leg
    on sampled rows and one mixed-precision solve."""
    import torch
    from paper_1211_7177_amd.solver import BemProblem
    from synthetic import CONFIGS, complex_normal, config_mesh, nystrom3, plane_waves, seed_for
    cfg = CONFIGS[5]
    t0 = time.perf_counter()
    nodes = nystrom3(config_mesh(5))
    n = nodes["points"].shape[0]
    log("c5 mesh: %d nodes in %.1f s" % (n, time.perf_counter() - t0))
    t0 = time.perf_counter()
    pb = BemProblem(nodes, cfg["k0"], cfg["eps"], order=0, depth=cfg["depth"], order32=0, tol=args.c5_tol64,
                    tol32=args.c5_tol32)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    infos = {t: p.info() for t, p in (("k0_fp64", pb.p0), ("k1_fp64", pb.p1), ("k0_fp32", pb.p0_32),
                                      ("k1_fp32", pb.p1_32))}
    log("c5 plans built in %.1f s" % plan_s, {t: (i["order_level"], i["far_lmin"], i["device_bytes"] / 1e9)
                                              for t, i in infos.items()})
    a64 = complex_normal((1, n, 3), seed_for(5, "a"))
    b64 = complex_normal((1, n, 3), seed_for(5, "b"))
    ga = {"fp32": torch.from_numpy(a64.astype(np.complex64)).cuda(),
          "fp64": torch.from_numpy(a64).cuda()}
    gb = {"fp32": torch.from_numpy(b64.astype(np.complex64)).cuda(),
          "fp64": torch.from_numpy(b64).cuda()}
    plans = {"fp32": (pb.p0_32, pb.p1_32), "fp64": (pb.p0, pb.p1)}
    ys = {t: (torch.empty_like(ga[t]), torch.empty_like(ga[t])) for t in plans}

    # one step = one application of the 6N operator (eqs. 2.9-2.13): split, the k0 and k1 FMM products
    # (their near fields in one launch in FP32), corrections, combine; x = (a, b) as (Phi, Psi)
    xs = {"fp32": torch.cat([ga["fp32"], gb["fp32"]], dim=2).contiguous(),
          "fp64": torch.cat([ga["fp64"], gb["fp64"]], dim=2).contiguous()}
    rs = {t: torch.empty_like(xs[t]) for t in xs}

    def step(t):
        if t == "fp32":
            pb.apply32(xs[t], out=rs[t])
        else:
            rs[t] = pb.apply(xs[t])

    for _ in range(args.warmup):
        step("fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step("fp32")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms32 = 1e3 * dt / args.steps
    log("c5 FP32 applications: %.2f ms per step (%d steps)" % (ms32, args.steps))
    # per-step spread (each step synchronised on its own; outside the timed loop)
    per = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        step("fp32")
        torch.cuda.synchronize()
        per.append(1e3 * (time.perf_counter() - t1))
    spread = {"p10_ms": float(np.percentile(per, 10)), "median_ms": float(np.median(per)),
              "p90_ms": float(np.percentile(per, 90))}
    step("fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps64 = 3
    for _ in range(reps64):
        step("fp64")
    torch.cuda.synchronize()
    ms64 = 1e3 * (time.perf_counter() - t0) / reps64
    log("c5 FP64 applications: %.2f ms per step" % ms64, "FP32 spread", spread)
    # the plans' own products on (a, b), for the oracle check of each wavenumber's operator
    for t, (p0, p1) in plans.items():
        p0.matvec(ga[t], gb[t], out=ys[t][0])
        p1.matvec(ga[t], gb[t], out=ys[t][1])
    torch.cuda.synchronize()

    # stage profile (HIP events on the plans' stream) of the exterior FP32 plan
    prof = {}
    for t in ("fp32", "fp64"):
        p0 = plans[t][0]
        p0.profile(True)
        p0.profile_read(reset=True)
        reps = 3 if t == "fp32" else 1
        for _ in range(reps):
            p0.matvec(ga[t], gb[t], out=ys[t][0])
        torch.cuda.synchronize()
        prof[t] = {k: (v[0] / reps, v[1] // reps) for k, v in p0.profile_read(reset=True).items() if v[1]}
        p0.profile(False)
    log("c5 exterior stage ms per product", prof)
    inf = infos["k0_fp32"]
    p2p_pairs = inf["p2p_pairs"] - 3 * n
    p2p_fl = P2P_FLOPS_PER_PAIR * p2p_pairs
    L = cfg["depth"]
    pl = inf["order_level"]
    m2l_fl = sum(inf["m2l_pairs"][l] * hf_translation_flops(pl[l]) for l in range(len(inf["m2l_pairs"])) if pl[l])
    fine_fl = inf["m2l_pairs"][L] * hf_translation_flops(pl[L])
    st = prof["fp32"]
    p2p_ms, m2l_ms, fine_ms = st["p2p"][0], st["m2l"][0], st["m2l_fine"][0]
    stages_rf = {
        "p2p": {"kernel": "k_p2p32 (near field, FP32 VALU)", "bound": "alu", "peak": PEAK["fp32_TF"],
                "unit": "TFLOP/s", "achieved": p2p_fl / (p2p_ms * 1e-3) / 1e12, "per_launch_flops": p2p_fl,
                "flops_per_unit": P2P_FLOPS_PER_PAIR, "unit_of_work": "(target, source) pair",
                "units_per_launch": p2p_pairs, "avg_launch_ms": p2p_ms, "launches_per_product": 1,
                "traffic": measured_traffic("k_p2p32 c5"),
                "gpairs_per_s": p2p_pairs / (p2p_ms * 1e-3) / 1e9},
        "m2l_fine": {"kernel": "k_hf_m2l_w (finest-level S|R by rotation / coaxial shift / rotation, FP32 VALU)",
                     "bound": "alu", "peak": PEAK["fp32_TF"], "unit": "TFLOP/s",
                     "achieved": fine_fl / (fine_ms * 1e-3) / 1e12, "per_launch_flops": fine_fl,
                     "flops_per_unit": hf_translation_flops(pl[L]), "unit_of_work": "S|R translation (3 channels)",
                     "units_per_launch": inf["m2l_pairs"][L], "order": pl[L], "avg_launch_ms": fine_ms,
                     "launches_per_product": 1, "traffic": measured_traffic("k_hf_m2l_w c5")},
        "m2l_all_levels": {"kernels": "k_hf_fwd / k_hf_coax / k_hf_back (orders > 20), k_hf_m2l_w (orders <= 20)",
                           "bound": "alu", "peak": PEAK["fp32_TF"], "unit": "TFLOP/s",
                           "achieved": m2l_fl / (m2l_ms * 1e-3) / 1e12, "flops_per_product": m2l_fl,
                           "ms_per_product": m2l_ms, "pairs_per_level": inf["m2l_pairs"], "order_per_level": pl},
    }
    for v in stages_rf.values():
        v["frac"] = v["achieved"] / v["peak"]
    dominant = "m2l_fine" if fine_ms >= p2p_ms else "p2p"
    roofline = {k: v for k, v in stages_rf[dominant].items()}
    log("c5 roofline", stages_rf)

    # the 18.1M-unknown system for a seeded plane wave, in nested mode (FP64 fGMRES preconditioned by FP32
    # fGMRES cycles of up to 100 steps), run in calls of --c5-solve-chunk iterations that each resume from the
    # previous iterate, until the FP64 residual reaches 1e-6 or the wall-clock budget is spent
    solve = None
    if args.c5_solve_s > 0:
        d, pol = plane_waves(1, seed_for(5, "dirs"), seed_for(5, "pols"))
        rhs = pb.rhs_planewave(d, pol)
        torch.cuda.synchronize()
        x, its, m32, m64, hist = None, 0, 0, 0, []
        kw = dict(tol=1e-6, mixed="nested", inner_tol=1e-2, restart=100, maxit=args.c5_solve_chunk,
                  raise_on_noconv=False)
        t0 = time.perf_counter()
        while True:
            x, info = pb.solve(rhs, x0=x, **kw)
            torch.cuda.synchronize()
            its += info["iterations"]
            m32 += info["matvecs32"]
            m64 += info["matvecs64"]
            el = time.perf_counter() - t0
            hist.append((its, info["residual"], round(el, 2)))
            log("c5 solve: %d iterations, FP64 residual %.3e, %.1f s" % (its, info["residual"], el))
            if info["residual"] <= 1e-6 or el >= args.c5_solve_s:
                break
        ts = time.perf_counter() - t0
        solve = {"seconds": ts, "iterations": its, "residual": hist[-1][1], "converged": hist[-1][1] <= 1e-6,
                 "solves_per_s": (1.0 / ts) if hist[-1][1] <= 1e-6 else None,
                 "bem_applies_fp32": m32, "bem_applies_fp64": m64,
                 "fp32_applies_per_s_in_solve": m32 / ts, "history_iterations_residual_s": hist,
                 "mode": "nested: FP64 fGMRES(100) preconditioned by FP32 fGMRES cycles (<= 100 steps, "
                         "inner tol 1e-2), restarted from the iterate every %d iterations" % args.c5_solve_chunk,
                 "tol": 1e-6, "budget_s": args.c5_solve_s}
        log("c5 solve", solve)
        del x, rhs

    cpu = None
    if not args.no_cpu_baseline:
        cpu, acc = c5_cpu_baseline(nodes, cfg, a64[0], b64[0], args.c5_rows,
                                   {t: (ys[t][0][0].cpu().numpy(), ys[t][1][0].cpu().numpy()) for t in plans})
        log("c5 oracle leg", cpu, acc)
    else:
        acc = None
    out = {
        "value": 1e3 / ms32, "ms_per_step": ms32, "step_spread_fp32": spread,
        "config": {"workload": C5_NAME, "nodes": n, "unknowns": 6 * n, "depth": cfg["depth"], "k0": cfg["k0"],
                   "eps": str(cfg["eps"]), "k1": str(pb.k1), "tol_fp32": args.c5_tol32, "tol_fp64": args.c5_tol64,
                   "order_per_level_fp32": infos["k0_fp32"]["order_level"],
                   "order_per_level_fp64": infos["k0_fp64"]["order_level"],
                   "interior_plan": "local only (far field damped below 1e-8 / 1e-16 at every level)",
                   "step": "one application of the 6N operator with the FP32 plans (bem_apply32: split, FMM "
                           "products at k0 and k1 with one fused near-field launch, FP64-built self-triangle "
                           "blocks, combine) on a seeded complex64 vector"},
        "bem_matvecs_per_s": {"fp32": 1e3 / ms32, "fp64": 1e3 / ms64},
        "unknowns_matvec_per_s": {"fp32": 6 * n * 1e3 / ms32, "fp64": 6 * n * 1e3 / ms64},
        "speedup_fp32_vs_fp64": ms64 / ms32,
        "stage_ms_per_product_k0": prof,
        "plan_s_4plans": plan_s,
        "plan_info": {t: {k: i[k] for k in ("nbox", "m2l_pairs", "p2p_pairs", "device_bytes", "order_level",
                                            "far_lmin")} for t, i in infos.items()},
        "roofline": roofline, "roofline_stages": stages_rf,
        "product_error_vs_oracle_rows": acc,
        "solve": solve,
        "cpu_baseline": cpu,
    }
    pb.close()
    return out


def c5_cpu_baseline(nodes, cfg, a, b, nrows, gpu_rows):
    """The oracle leg of the large ellipsoid: its direct FP64 sum of both wavenumbers' operators (point sum plus
    LINEAR self-triangle blocks) on `nrows` seeded target rows with all host cores, timed and scaled to one full
    BEM application; the same timing on one core over a smaller sample (a child process with
    OMP_NUM_THREADS=1); and the relative error of the GPU products on those rows."""
    import subprocess
    from oracle.corrections import self_blocks
    from oracle.direct import apply_corrections
    from oracle.kernel import wavenumber
    from oracle.native import point_sum_c
    from synthetic import seed_for
    n = nodes["points"].shape[0]
    rows = np.sort(np.random.default_rng(seed_for(5, "rows")).choice(n, nrows, replace=False))
    k0 = cfg["k0"]
    k1 = wavenumber(k0, cfg["eps"])
    pts, nrm, w, pt = nodes["points"], nodes["normals"], nodes["weights"], nodes["point_tri"]
    tris = np.unique(pt[rows])
    sub = (3 * tris[:, None] + np.arange(3)[None, :]).reshape(-1)
    remap = np.repeat(np.arange(len(tris)), 3)
    loc = np.searchsorted(sub, rows)
    t0 = time.perf_counter()
    ref = {}
    for tag, k in (("k0", k0), ("k1", k1)):
        y = point_sum_c(pts, nrm, w, pt, k, a, b, rows=rows)
        blk = self_blocks(pts[sub], nrm[sub], remap, nodes["tri_vertices"][tris], k, mode="linear")
        ref[tag] = y + apply_corrections(nrm[sub], remap, blk, a[sub], b[sub], rows=loc)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    acc = {}
    for t, (y0, y1) in gpu_rows.items():
        acc[t] = {"k0": float(np.linalg.norm(y0[rows] - ref["k0"]) / np.linalg.norm(ref["k0"])),
                  "k1": float(np.linalg.norm(y1[rows] - ref["k1"]) / np.linalg.norm(ref["k1"])),
                  "rows": int(nrows)}
    # one core, 32 rows, in a child process (the OpenMP pool of this one is already sized)
    r1 = 32
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r)\n"
            "from synthetic import config_mesh, nystrom3, complex_normal, seed_for\n"
            "from oracle.native import point_sum_c\nfrom oracle.kernel import wavenumber\n"
            "q = nystrom3(config_mesh(5)); n = q['points'].shape[0]\n"
            "a = complex_normal((n, 3), seed_for(5, 'a')); b = complex_normal((n, 3), seed_for(5, 'b'))\n"
            "rows = np.arange(0, n, n // %d)[:%d].astype(np.int64)\n"
            "t = time.perf_counter()\n"
            "for k in (%r, wavenumber(%r, %r)):\n"
            "    point_sum_c(q['points'], q['normals'], q['weights'], q['point_tri'], k, a, b, rows=rows)\n"
            "print(time.perf_counter() - t)\n") % (ROOT, r1, r1, k0, k0, cfg["eps"])
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = None
    try:
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        one = float(res.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError):
        one = None
    apply_s = dt * n / nrows
    cpu = {"value": 1.0 / apply_s, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
           "sample": "FP64 oracle direct sum of both wavenumbers (point sum + self-triangle blocks) on %d of %d "
                     "seeded target rows against all sources, %.2f s with %d threads, scaled by n/rows to one full "
                     "application of the two operators (%.0f s)" % (nrows, n, dt, cores, apply_s),
           "seconds_per_full_apply_extrapolated": apply_s}
    if one is not None:
        apply1 = one * n / r1
        cpu["one_core"] = {"value": 1.0 / apply1, "unit": "matvecs/s", "cores": 1,
                           "sample": "point sums of both wavenumbers on %d rows, %.2f s, scaled to one full "
                                     "application (%.0f s)" % (r1, one, apply1)}
    return cpu, acc


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(torch.device("cuda:0"))
    if args.copy_calibration:
        # a device-to-device copy of known size, for scaling the HBM byte counters of a profiled run
        buf = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").uniform_()
        torch.cuda.synchronize()
        buf2 = buf.clone()
        torch.cuda.synchronize()
        log("copy calibration: 256 MiB device-to-device copy done", buf2.numel())
        del buf, buf2
    c5 = c5_workload(args, log)
    torus = None if args.skip_torus else torus_section(args, log)
    c3 = c3_section(args, log) if args.c3 else None
    out = {
        "metric": "FMM matvecs/s & GMRES solves/s at 1e-6 rel err, FP32/batched vs plain FP64",
        "value": c5["value"],
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": c5["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": c5["config"],
        "roofline": c5["roofline"],
        "cpu_baseline": c5["cpu_baseline"],
        "c5": {k: v for k, v in c5.items() if k not in ("value", "ms_per_step", "config", "roofline", "cpu_baseline")},
        "torus": torus,
        "c3_batched_three_meshes": c3,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
