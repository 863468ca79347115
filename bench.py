#!/usr/bin/env python3
"""Benchmark of the recursive-skeletonization hot path on one MI355X.

One step = one factorization of the workload's boundary operator followed by
the solve of all its right-hand sides to a relative residual of 1e-8
(device-resident in and out): ID-matrix assembly, pivoted QR, diagonal-block
assembly, elimination, border and root, the U / X_D^{-1} / V sweeps and the
iterative refinement with the exact float64 residual.  The quadtree and the
geometry upload happen once before the timed region (their time is reported
as setup_ms, never inside `value`).

Default workload: the 131072-node boundary (outer circle of radius 40 and 64
ellipses, 262336 unknowns) with 16 right-hand sides.  Forms: "mixed" (float32
factor application, float64 pivoted QR / inverses / root / residual, ID
tolerance per workload) and "plain" (float64 throughout, ID tolerance 1e-10);
both refine to 1e-8.  The first form listed is `value`.  A second line of
work, the many-geometry batch (mixed, level-synchronous launches across
geometries, against the float64 path run geometry by geometry), is reported
beside it under "batch" (skip with --batch-size 0).

value = right-hand sides solved per second including their factorization
      = nrhs * steps / (time of `steps` factor+solve steps).

Prints one JSON line.  `--gpus` above 1 is not supported (single-GPU build).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X published FP64 vector / matrix peak
FP32_MFMA_PEAK_TFLOPS = 157.3    # MI355X published dense FP32 matrix peak
BREAKDOWN_STEPS = 2                # untimed steps after the timed region, every kernel family timed
HBM_PEAK_GBS = 8000.0

# roofline: the kernel family whose launches the timed region brackets with
# events (timing mode 3 = pivoted QR, 4 = exact operator apply)
WORKLOADS = {
    "circle40_64holes": dict(desc="outer circle R=40 (16384 nodes) + 64 random ellipses (1792 nodes each), "
                                  "262144 unknowns + 192 border, seed 3", nrhs=16, seed=3, tol_mixed=1e-7,
                             roofline="apply_operator"),
    "circle10_8holes": dict(desc="outer circle R=10 (4096 nodes) + 8 random ellipses (1024 nodes each), "
                                 "24576 unknowns + 24 border, seed 2", nrhs=4, seed=2, tol_mixed=1e-6,
                            roofline="cpqr"),
    "ellipse_2048": dict(desc="ellipse semi-axes 1.0/0.6, 2048 nodes, 4096 unknowns", nrhs=1, seed=1,
                         tol_mixed=1e-6, roofline="cpqr"),
}
TIMING_MODE = {"cpqr": 3, "apply_operator": 4}


def batch_geometries(n):
    """Members 0, k, 2k, ... of the 512-geometry batch (k = 512 // n): n geometries."""
    import workloads as W

    stride = max(1, 512 // n)
    return [W.workload_batch_member(i * stride) for i in range(n)]


def run_batch(args, forms):
    """Many geometries: mixed precision, factored level-synchronously
    (rs_factor_batch) and solved interleaved (rs_solve_batch), 16 right-hand
    sides each, against the plain float64 path on the same geometries one
    after another.  The geometries go through in parts of at most
    args.batch_chunk (device memory: about 20 KB per unknown while a part is
    factored and solved); a step is every part's factor + solve, the timed
    region the sum over the parts (each part's solvers are set up and warmed
    up before its timed steps)."""
    import numpy as np
    import torch

    from paper_2001_11619_amd import RSSolver, factor_batch, solve_batch
    from workloads import boundary_data, exterior_forces_for_geometry

    nb, nrhs = args.batch_size, 16
    chunk = max(1, min(nb, getattr(args, "batch_chunk", nb)))
    geoms = batch_geometries(nb)
    fs = [boundary_data(g, exterior_forces_for_geometry(g, nrhs, seed=100 + i)) for i, g in enumerate(geoms)]
    out = {}
    for form in forms:
        kw = dict(tol=args.tol_plain, precision=0) if form == "plain" else dict(tol=args.tol_mixed, precision=1)
        el, setup_ms, res = 0.0, 0.0, 0.0
        for c0 in range(0, nb, chunk):
            gs, fc = geoms[c0:c0 + chunk], fs[c0:c0 + chunk]
            t0 = time.perf_counter()
            sv = [RSSolver.from_geometry(g, refine_max=20, refine_tol=1e-8, **kw) for g in gs]
            setup_ms += 1e3 * (time.perf_counter() - t0)
            stream = torch.cuda.current_stream().cuda_stream
            for s in sv:
                s.set_stream(stream)
            fd = [torch.tensor(np.ascontiguousarray(f.T), dtype=torch.float64, device="cuda") for f in fc]
            xd = [torch.empty((nrhs, g.n_system), dtype=torch.float64, device="cuda") for g in gs]

            def step():
                if form == "plain":
                    for s, f_, x_ in zip(sv, fd, xd):
                        s.factor()
                        s.solve_dev(f_, x_)
                else:
                    factor_batch(sv)
                    solve_batch(sv, fd, xd)

            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step()
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            res = max([res] + [float(np.max(s.solve(f, residual=True)[1])) for s, f in zip(sv, fc)])
            print("bench: batch %s, geometries %d..%d done (%.1f s timed so far)"
                  % (form, c0, c0 + len(gs) - 1, el), file=sys.stderr, flush=True)
            for s in sv:
                s.close()
            del sv, fd, xd
        out[form] = {"value": nb * nrhs * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                     "setup_ms": setup_ms, "max_rel_residual": res, "parts": (nb + chunk - 1) // chunk}
    unknowns = [g.n_system for g in geoms]
    head = out[forms[0]]
    js = {
        "metric": "RS factor s + solves/s at 1e-8 rel. residual, mixed-batched vs FP64 plain",
        "value": head["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if forms[0] == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "batch%d_of_512" % nb, "geometries": nb, "nrhs_each": nrhs,
                   "geometries_per_launch": chunk,
                   "unknowns_min": min(unknowns), "unknowns_max": max(unknowns),
                   "unknowns_total": int(sum(unknowns)), "form": forms[0]},
        "max_rel_residual": head["max_rel_residual"], "setup_ms": head["setup_ms"],
    }
    for fm in forms[1:]:
        js["form_" + fm] = out[fm]
        js["speedup_vs_" + fm] = head["value"] / out[fm]["value"]
    return js


def run_evolve(args):
    """Evolving domain: the 64-hole geometry, one ellipse moved per step
    (translation 0.05 N(0, I), rotation U[-0.1, 0.1]), the factorization
    updated (only boxes whose inputs changed are recompressed) and 16
    right-hand sides solved to 1e-8; one full refactorization timed beside."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2001_11619_amd import RSSolver
    from workloads import boundary_data, exterior_forces_for_geometry

    g = W.workload_circle40_64holes()
    nrhs = 16
    kw = dict(tol=args.tol_mixed, precision=1, refine_max=20, refine_tol=1e-8)
    s = RSSolver.from_geometry(g, **kw)
    s.set_stream(torch.cuda.current_stream().cuda_stream)
    root = tuple(s.boxes()["geom"][0])
    s.factor()
    rng = np.random.Generator(np.random.PCG64(5))
    upd, sol, res, recomp = [], [], [], []
    t_all = time.perf_counter()
    for t in range(args.evolve_steps):
        print("evolve: step %d" % t, file=sys.stderr, flush=True)
        g, moved = W.move_hole(g, 1 + t % g.n_holes if args.evolve_all else 1, rng)
        s.update_moved_nodes(moved, g.xy[moved], g.normal[moved], g.weight[moved], g.curvature[moved],
                             hole_xy=g.hole_xy)
        st = s.stats()
        upd.append(st["ms_update"])
        recomp.append(st["boxes_recomputed"])
        f = boundary_data(g, exterior_forces_for_geometry(g, nrhs, seed=t))
        x, r = s.solve(f, residual=True)
        sol.append(s.stats()["ms_solve"])
        res.append(float(np.max(r)))
    el = time.perf_counter() - t_all
    g.root = np.array(root)
    fresh = RSSolver.from_geometry(g, root=root, **kw)
    fresh.set_stream(torch.cuda.current_stream().cuda_stream)
    fresh.factor()
    fresh.factor()
    refactor_ms = fresh.stats()["ms_factor"]
    nbox = int(np.sum(fresh.boxes()["n"][1:] > 0))
    # Section 2.8: the updated factorization is the fresh one of the new
    # geometry (same root): the solves agree bitwise
    f = boundary_data(g, exterior_forces_for_geometry(g, nrhs, seed=999))
    p8 = bool(np.array_equal(s.solve(f), fresh.solve(f)))
    fresh.close()
    s.close()
    return {
        "metric": "RS factorization update (Section 2.8) vs full refactor, mixed precision, 16 rhs to 1e-8",
        "value": float(np.median(upd)), "unit": "ms/update", "higher_is_better": False, "n_gpus": 1,
        "steps": args.evolve_steps, "data": "synthetic", "dtype": "f32+f64",
        "config": {"workload": "circle40_64holes_evolving", "nrhs": nrhs, "moved_nodes_per_step": int(len(moved)),
                   "tol": args.tol_mixed},
        "update_ms_median": float(np.median(upd)), "update_ms_max": float(np.max(upd)),
        "refactor_ms": refactor_ms, "speedup_update_vs_refactor": refactor_ms / float(np.median(upd)),
        "boxes_recomputed_median": float(np.median(recomp)), "boxes_total": nbox,
        "solve_ms_median": float(np.median(sol)), "max_rel_residual": float(np.max(res)),
        "update_equals_refactor_bitwise": p8,
        "update_ms_per_step": upd, "residual_per_step": res, "wall_s": el,
    }


def run_holes(args):
    """Holes inserted and deleted (the experiment of Section 4.2 on the 64-hole
    workload): one new ellipse of 1792 nodes inserted, then hole 1 deleted,
    each applied with rs_update_geometry (only boxes whose inputs changed are
    recompressed) and timed against a full factorization of the same new
    boundary with the same root; 16 right-hand sides refined to 1e-8 after
    each change; the updated solve compared bitwise with the fresh one."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2001_11619_amd import RSSolver
    from workloads import boundary_data, exterior_forces_for_geometry

    g = W.workload_circle40_64holes()
    nrhs = 16
    kw = dict(tol=args.tol_mixed, precision=1, refine_max=20, refine_tol=1e-8)
    s = RSSolver.from_geometry(g, **kw)
    s.set_stream(torch.cuda.current_stream().cuda_stream)
    root = tuple(s.boxes()["geom"][0])
    g.root = np.array(root)
    s.factor()
    rng = np.random.Generator(np.random.PCG64(6))
    out = {}
    for step in ("insert", "delete"):
        print("holes: %s" % step, file=sys.stderr, flush=True)
        if step == "insert":
            g2, oon = W.insert_hole(g, rng, 1792)
        else:
            g2, oon = W.delete_hole(g, 1)
        g2.root = np.array(root)
        s.update_geometry(g2.xy, g2.normal, g2.weight, g2.curvature, g2.curve_id, oon, hole_xy=g2.hole_xy)
        st = s.stats()
        fresh = RSSolver.from_geometry(g2, root=root, **kw)
        fresh.set_stream(torch.cuda.current_stream().cuda_stream)
        fresh.factor()
        fresh.factor()
        f = boundary_data(g2, exterior_forces_for_geometry(g2, nrhs, seed=7))
        x, r = s.solve(f, residual=True)
        out[step] = {"update_ms": st["ms_update"], "refactor_ms": fresh.stats()["ms_factor"],
                     "speedup": fresh.stats()["ms_factor"] / st["ms_update"],
                     "boxes_recomputed": st["boxes_recomputed"],
                     "boxes_total": int(np.sum(fresh.boxes()["n"][1:] > 0)),
                     "n_nodes": g2.n_nodes, "n_holes": g2.n_holes, "max_rel_residual": float(np.max(r)),
                     "update_equals_refactor_bitwise": bool(np.array_equal(x, fresh.solve(f)))}
        fresh.close()
        g = g2
    s.close()
    return {"metric": "RS factorization update after hole insertion / deletion (Sections 2.8, 4.2) vs full "
                      "refactor, mixed precision", "value": out["insert"]["speedup"], "unit": "x",
            "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "f32+f64",
            "config": {"workload": "circle40_64holes_holes", "nrhs": nrhs, "tol": args.tol_mixed,
                       "inserted_nodes": 1792}, **out}


def run_laplace(args):
    """The heat-flux workload of Section 4.4.1 (Laplace Neumann, kernel 1):
    16384 nodes on a starfish holding two starfish holes 16% of its size,
    flux 0 / +1 / -1 (eq. neumanndata), holes at theta = (0.4, 3.0) on their
    path (away from the mirror-symmetric (0, pi), where the gradient of the
    objective vanishes by symmetry).  Timed: the
    factorization and the refined solve of the base geometry, then one step
    of the section's finite-difference gradient of the objective d u / d x at
    the centre (fourth-order stencil: theta_i +- h, +- 2h, eight related
    geometries) three ways -- eight fresh factorizations in one batch, the
    eight updates of factored contexts in one batch (Scheme A's independent
    updates, in shared launches), and one context updated eight times in
    turn -- each followed by the eight refined solves and evaluations."""
    import numpy as np
    import torch

    from paper_2001_11619_amd import RSSolver, factor_batch, solve_batch, update_moved_nodes_batch
    from workloads import neumann_flux, starfish_geometry

    n, theta, h = 16384, (0.4, 3.0), 0.01
    kw = dict(kernel=1, tol=args.laplace_tol, precision=1, refine_max=20, refine_tol=1e-10,
              root=(0.0, 0.0, 2.6))
    stream = torch.cuda.current_stream().cuda_stream
    centre = np.zeros((1, 2))

    def make(g):
        sv = RSSolver.from_geometry(g, **kw)
        sv.set_stream(stream)
        return sv

    def moved(g0, g1):
        m = np.nonzero(np.any(g0.xy != g1.xy, axis=1))[0].astype(np.int32)
        return (m, g1.xy[m], g1.normal[m], g1.weight[m], g1.curvature[m])

    def solve_obj(sv, g):
        x = sv.solve(RSSolver.embed_scalar(neumann_flux(g.curve_id)))
        return float(sv.evaluate(centre, x)[0, 1]), sv.stats()["refine_iters"]

    # the eight solves of a step: device-resident, interleaved (rs_solve_batch);
    # then the objective of each from its density
    def solve_all(svs):
        solve_batch(svs, [f_dev] * len(svs), x_dev[:len(svs)])
        torch.cuda.synchronize()
        return [float(sv.evaluate(centre, xd[0].cpu().numpy())[0, 1]) for sv, xd in zip(svs, x_dev)]

    base = starfish_geometry(n, *theta)
    f_dev = torch.tensor(RSSolver.embed_scalar(neumann_flux(base.curve_id))[None, :], dtype=torch.float64,
                         device="cuda").contiguous()
    x_dev = [torch.empty((1, 2 * n), dtype=torch.float64, device="cuda") for _ in range(8)]
    s = make(base)
    for _ in range(1 + args.warmup):
        s.factor()
    fac_ms = []
    for _ in range(args.steps):
        s.factor()
        fac_ms.append(s.stats()["ms_factor"])
    # roofline of the factorization's largest kernel family, the pivoted QR
    # (timing mode 3: events around its launches only), with the method's own
    # flop count per factorization
    s.set_kernel_timing(3)
    s.kernel_times(reset=True)
    s.factor()
    qr_launches, qr_ms = s.kernel_times(reset=True).get("cpqr", (0, 0.0))
    s.set_kernel_timing(0)
    qr_work = float(s.stats()["flops_id"])
    roof = None
    if qr_ms > 0:
        ach = qr_work / (qr_ms / 1e3) / 1e12
        roof = {"bound": "alu", "kernel": "cpqr", "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                "work": qr_work, "work_unit": "flops per factorization (sum of the boxes' pivoted-QR + T counts)",
                "launches_per_step": qr_launches, "ms_per_step": qr_ms}
    obj0, it0 = solve_obj(s, base)
    sol_ms = []
    for _ in range(args.steps):
        solve_obj(s, base)
        sol_ms.append(s.stats()["ms_solve"])
    shifts = [(k * h, 0.0) for k in (-2, -1, 1, 2)] + [(0.0, k * h) for k in (-2, -1, 1, 2)]
    geoms = [starfish_geometry(n, theta[0] + a, theta[1] + b) for a, b in shifts]
    out = {}
    # eight fresh factorizations, one batch
    print("laplace: fresh batch", file=sys.stderr, flush=True)
    fresh = [make(gk) for gk in geoms]
    factor_batch(fresh)
    torch.cuda.synchronize()
    t = time.perf_counter()
    factor_batch(fresh)
    torch.cuda.synchronize()
    out["fresh_batch_factor_ms"] = 1e3 * (time.perf_counter() - t)
    # eight updates of factored contexts, one batch
    print("laplace: update batch", file=sys.stderr, flush=True)
    ctx = [make(base) for _ in geoms]
    factor_batch(ctx)
    update_moved_nodes_batch(ctx, [moved(base, gk) for gk in geoms])      # warm-up of the update path
    update_moved_nodes_batch(ctx, [moved(gk, base) for gk in geoms])
    torch.cuda.synchronize()
    t = time.perf_counter()
    update_moved_nodes_batch(ctx, [moved(base, gk) for gk in geoms])
    torch.cuda.synchronize()
    out["batch_update_ms"] = 1e3 * (time.perf_counter() - t)
    solve_all(ctx)                      # warm-up (graph capture of the refinement)
    torch.cuda.synchronize()
    t = time.perf_counter()
    objs = solve_all(ctx)
    out["solves_and_objective_ms"] = 1e3 * (time.perf_counter() - t)
    solve_all(fresh)
    out["objectives_fresh_equal_updated"] = bool(solve_all(fresh) == objs)
    xf = fresh[0].solve(RSSolver.embed_scalar(neumann_flux(geoms[0].curve_id)))
    xu = ctx[0].solve(RSSolver.embed_scalar(neumann_flux(geoms[0].curve_id)))
    out["update_equals_fresh_bitwise"] = bool(np.array_equal(xf, xu))
    # one context updated eight times in turn
    print("laplace: sequential updates", file=sys.stderr, flush=True)
    t = time.perf_counter()
    prev = base
    upd = []
    for gk in geoms:
        s.update_moved_nodes(*moved(prev, gk))
        upd.append(s.stats()["ms_update"])
        solve_obj(s, gk)
        prev = gk
    out["sequential_update_and_solve_ms"] = 1e3 * (time.perf_counter() - t)
    out["sequential_update_ms_median"] = float(np.median(upd))
    o = np.array(objs)
    grad = [float((-o[3] + 8 * o[2] - 8 * o[1] + o[0]) / (12 * h)), float((-o[7] + 8 * o[6] - 8 * o[5] + o[4]) / (12 * h))]
    # the step's geometries come fastest from the batch of fresh factorizations
    # (the batched update is timed beside it)
    step_ms = out["fresh_batch_factor_ms"] + out["solves_and_objective_ms"]
    out["fd_step_ms_with_batch_update"] = out["batch_update_ms"] + out["solves_and_objective_ms"]
    for sv in fresh + ctx + [s]:
        sv.close()
    return {
        "metric": "Laplace Neumann (Section 4.4.1) finite-difference step: eight related geometries factored "
                  "in one batch, solved to 1e-10 and the objective evaluated",
        "value": 8 * 1e3 / step_ms, "unit": "geometries/s", "higher_is_better": True, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "dtype": "f32+f64",
        "config": {"workload": "starfish16384_2holes_laplace", "n_nodes": n, "theta": list(theta), "fd_h": h,
                   "tol": args.laplace_tol, "refine_tol": 1e-10},
        "roofline": roof,
        "factor_ms_median": float(np.median(fac_ms)), "solve_ms_median": float(np.median(sol_ms)),
        "refine_iters": int(it0), "objective_du_dx_centre": obj0, "fd_gradient": grad,
        "fd_step_ms": step_ms, **out,
    }


def make_geometry(name):
    import workloads as W

    return {"circle10_8holes": W.workload_circle10_8holes, "ellipse_2048": W.workload_ellipse_2048,
            "circle40_64holes": W.workload_circle40_64holes}[name]()


def cpu_baseline(geom, f, tol, full, budget_s=15.0):
    """The CPU oracle (plain level-parallel RS, float64) on the host cores.

    full=True: the oracle factors the whole workload and solves it, three
    times (median); value = nrhs / time.  full=False (workloads whose oracle
    factorization takes far longer than the bench should run): a sample of the
    workload.  The deepest level's boxes are compressed by the oracle with
    their exact inputs (at that level every unknown is active) until
    `budget_s` seconds are spent; the time per box, times the number of boxes
    at that level, stands for the factorization.  Upper levels, the root and
    the solve are left out, so value = nrhs / that time bounds the oracle's
    throughput from above."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.rs import RSFactorization, RSParams

    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    nrhs = f.shape[1]
    if full:
        tf, ts = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            orc = RSFactorization(geom, RSParams(tol=tol)).factor()
            t1 = time.perf_counter()
            orc.solve(f)
            t2 = time.perf_counter()
            tf.append(t1 - t0)
            ts.append(t2 - t1)
        tot = float(np.median(np.array(tf) + np.array(ts)))
        return {"value": nrhs / tot, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
                "sample": "3 full factorizations + direct solves of the same workload (%d rhs), median: "
                          "factor %.2f s, solve %.3f s" % (nrhs, float(np.median(tf)), float(np.median(ts)))}
    # sample: the oracle's compression of a stratified random sample of boxes at
    # every level below the top two, each with its exact inputs.  The level-start
    # active sets and the children's skeletons come from the GPU's float64
    # factorization of the same workload (same tree, tolerance and pivot rule as
    # the oracle with the "key20" rule), so each sampled box is compressed from
    # the unknowns and near field the full oracle run would give it.
    import torch

    from oracle.rs import BoxFactor
    from paper_2001_11619_amd import RSSolver

    gpu = RSSolver.from_geometry(geom, tol=tol)
    gpu.set_stream(torch.cuda.current_stream().cuda_stream)
    gpu.factor()
    bx = gpu.boxes()
    orc = RSFactorization(geom, RSParams(tol=tol, pivot="key20"))
    nb = len(orc.boxes)
    skel = [gpu.skeleton(b) if bx["n"][b] > 0 and b > 0 else np.zeros(0, np.int64) for b in range(nb)]
    gpu.close()
    active = np.ones(geom.n_dofs, dtype=bool)
    rng = np.random.Generator(np.random.PCG64(0))
    top = 2
    per_level = budget_s / max(1, orc.L - top)
    est, sampled, total = 0.0, 0, 0
    for l in range(orc.L, 0, -1):
        bl = orc.levels(l)
        snap = active.copy()
        if l > top:
            t_level, done = 0.0, 0
            for i in rng.permutation(len(bl)):
                t0 = time.perf_counter()
                orc.compress(bl[int(i)], snap)
                t_level += time.perf_counter() - t0
                done += 1
                if t_level > per_level:
                    break
            est += t_level / done * len(bl)
            sampled += done
            total += len(bl)
        for b in bl:
            I = orc.box_dofs(b)
            S = np.sort(skel[b.id].astype(np.int64))
            # a stand-in whose skeleton is the GPU's (I = S, identity order); its
            # X_SS block (values only, no effect on any box's shapes) is the identity
            orc.fac[b.id] = BoxFactor(b.id, l, S, np.arange(S.size), S.size, None, None, None, None,
                                      np.eye(S.size))
            active[np.setdiff1d(I, S)] = False
    return {"value": nrhs / est, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": "oracle compression of %d of the %d boxes of levels %d..%d (a random sample per level; "
                      "each box's unknowns and near field from the GPU's float64 factorization, its children's "
                      "X_SS blocks stood in by identities), scaled per level: %.1f s for %d rhs.  The top %d "
                      "levels, the root and the solve are not counted, so the value is an upper bound on "
                      "the oracle's throughput" % (sampled, total, orc.L, top + 1, est, nrhs, top)}


def run_form(geom, f, form, steps, warmup, tol_plain, tol_mixed, roof_family):
    """Time `steps` factor + refined solve steps of one form ("plain" or "mixed")."""
    import numpy as np
    import torch

    from paper_2001_11619_amd import RSSolver

    nrhs = f.shape[1]
    kw = dict(tol=tol_plain, precision=0) if form == "plain" else dict(tol=tol_mixed, precision=1)
    t0 = time.perf_counter()
    s = RSSolver.from_geometry(geom, refine_max=20, refine_tol=1e-8, **kw)
    setup_ms = 1e3 * (time.perf_counter() - t0)
    s.set_stream(torch.cuda.current_stream().cuda_stream)
    fd = torch.tensor(np.ascontiguousarray(f.T), dtype=torch.float64, device="cuda")
    xd = torch.empty((nrhs, geom.n_system), dtype=torch.float64, device="cuda")

    def step():
        s.factor()
        s.solve_dev(fd, xd)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the timed region records HIP events around the roofline family only; the
    # per-family breakdown comes from two more steps with every family and
    # host phase timed, after the timed region
    s.set_kernel_timing(TIMING_MODE[roof_family])
    s.kernel_times(reset=True)
    torch.cuda.synchronize()
    fac_ms, sol_ms, iters = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        st = s.stats()
        fac_ms.append(st["ms_factor"])
        sol_ms.append(st["ms_solve"])
        iters.append(st["refine_iters"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktimes = s.kernel_times(reset=True)
    s.set_kernel_timing(True)
    for _ in range(BREAKDOWN_STEPS):
        step()
    torch.cuda.synchronize()
    kbreak = s.kernel_times(reset=True)
    s.set_kernel_timing(False)
    st = s.stats()
    x, res = s.solve(f, residual=True)     # accuracy check outside the timed region
    s.close()
    return {
        "elapsed": elapsed, "setup_ms": setup_ms, "ktimes": ktimes, "kbreak": kbreak, "stats": st,
        "factor_s": float(np.median(fac_ms)) / 1e3, "solve_s": float(np.median(sol_ms)) / 1e3,
        "refine_iters": int(max(iters)), "iters_per_step": [int(i) for i in iters],
        "max_rel_residual": float(np.max(res)), "value": nrhs * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
    }


# counter summaries (copy-calibrated FETCH_SIZE + WRITE_SIZE per launch) of
# the roofline kernels, valid while the listed sources are unchanged
TRAFFIC = {
    "cpqr": (os.path.join(ROOT, "profiles", "hbm_traffic_cpqr_circle10_8holes.md"), ("rs_qr.hip", "rs_device.h")),
    "apply_operator": (os.path.join(ROOT, "profiles", "hbm_traffic_apply_circle40_64holes.md"),
                       ("rs_apply.hip", "rs_device.h")),
    "apply_correction": (os.path.join(ROOT, "profiles", "hbm_traffic_apply_correction_circle40_64holes.md"),
                         ("rs_apply.hip", "rs_device.h")),
}


def kernel_source_hash(names):
    import hashlib

    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2001_11619_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(fam, workload, form, tol):
    """HBM bytes per launch (per step for the QR family) of the roofline kernel family from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE runs, copy-calibrated), or None
    when the summary is for another workload, form or tolerance ("any" where
    they do not change the kernel's work), or the kernels changed since."""
    if fam not in TRAFFIC or not os.path.exists(TRAFFIC[fam][0]):
        return None
    path, srcs = TRAFFIC[fam]
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("workload") != workload or vals.get("form") not in (form, "any"):
        return None
    if vals.get("tol") != "any":
        try:
            if float(vals.get("tol", "nan")) != tol:
                return None
        except ValueError:
            return None
    if vals.get("kernel_source_sha256") != kernel_source_hash(srcs):
        return None
    # the apply families are counted per launch, the QR family per step (one
    # factorization), matching the roofline's traffic_unit
    for unit in ("launch", "step"):
        try:
            return float(vals["fetch_bytes_per_" + unit]) + float(vals["write_bytes_per_" + unit])
        except (KeyError, ValueError):
            continue
    return None


def roofline_of(run, steps, nrhs, n_nodes, workload, form, tol, fam):
    """Roofline of the workload's dominant kernel family, timed live with HIP
    events around each of its launches in the timed region.

    apply_operator (the exact float64 residual, O(N^2)): per launch N (N - 1)
    target-source node pairs, each 26 flops for the stresslet entries plus
    8 flops per right-hand-side column for the 2 x 2 block times the density
    (the per-pair count of the work model), over the average launch time.
    cpqr (the IDs): per factorization sum over boxes of the pivoted QR to rank
    k plus T, 4mnk - 2(m+n)k^2 + (4/3)k^3 + k^2 r, over the family's time per
    step.  Both are float64 vector arithmetic: peak 78.6 TFLOP/s."""
    st, ktimes = run["stats"], run["ktimes"]
    dev = {k: v for k, v in run["kbreak"].items() if not k.startswith("host:") and "." not in k}
    dominant = max(dev, key=lambda k: dev[k][1]) if dev else None
    if fam not in ktimes:
        return None
    launches, tot_ms = ktimes[fam]
    if fam == "apply_operator":
        pairs = float(n_nodes) * (n_nodes - 1)
        work = pairs * (26.0 + 8.0 * nrhs)
        per_launch_s = tot_ms / 1e3 / launches
        unit_desc = "flops per launch: N(N-1) node pairs x (26 + 8 nrhs)"
    else:
        work = st["flops_id"]
        per_launch_s = tot_ms / 1e3 / steps
        unit_desc = "flops per factorization (sum of the boxes' pivoted-QR + T counts)"
    achieved = work / per_launch_s / 1e12
    corr = None
    if fam == "apply_operator" and "apply_correction" in ktimes:
        # the float32 image of a refinement correction: the 2 x 2 blocks times
        # the columns on FP32 matrix cores, 8 nrhs flops per node pair
        cl, cms = ktimes["apply_correction"]
        cwork = float(n_nodes) * (n_nodes - 1) * 8.0 * nrhs
        cach = cwork / (cms / 1e3 / cl) / 1e12
        corr = {"bound": "mfma", "kernel": "apply_correction", "achieved": cach,
                "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": cach / FP32_MFMA_PEAK_TFLOPS,
                "work": cwork, "work_unit": "FP32 matrix-core flops per launch: N(N-1) node pairs x 8 nrhs",
                "launches_per_step": cl / steps, "ms_per_launch": cms / cl,
                "traffic": measured_traffic("apply_correction", workload, form, tol),
                "traffic_unit": "HBM bytes per launch"}
    return {"bound": "alu", "kernel": fam, "dominant_family": dominant, "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(fam, workload, form, tol),
            "traffic_unit": "HBM bytes per launch" if fam == "apply_operator" else "HBM bytes per step",
            "work": work, "work_unit": unit_desc, "launches_per_step": launches / steps,
            "ms_per_launch": 1e3 * per_launch_s if fam == "apply_operator" else tot_ms / launches,
            "ms_per_step": tot_ms / steps, "correction_image": corr}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="circle40_64holes", choices=sorted(WORKLOADS) + ["batch", "evolve", "holes", "laplace"])
    ap.add_argument("--tol-plain", type=float, default=1e-10)
    ap.add_argument("--tol-mixed", type=float, default=None,
                    help="ID tolerance of the mixed form (default: per workload, the fastest that "
                         "refines to 1e-8 in few iterations)")
    ap.add_argument("--forms", default="mixed,plain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-size", type=int, default=32,
                    help="geometries of the many-geometry line (0: leave it out)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-chunk", type=int, default=128,
                    help="geometries factored together in one level-synchronous batch (device memory)")
    ap.add_argument("--batch-tol-mixed", type=float, default=1e-7)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="before the timed steps, one device copy of this many MiB (the reference "
                         "dispatch for calibrating HBM byte counters)")
    ap.add_argument("--laplace-tol", type=float, default=1e-7)
    ap.add_argument("--evolve-steps", type=int, default=100)
    ap.add_argument("--evolve-all", action="store_true", help="move hole 1, 2, 3, ... in turn")
    args = ap.parse_args()
    if args.tol_mixed is None:
        args.tol_mixed = WORKLOADS.get(args.workload, {}).get("tol_mixed", 1e-7)
    if args.gpus != 1:
        print("bench.py runs on one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from workloads import boundary_data, exterior_forces_for_geometry

    torch.cuda.set_device(0)
    if args.workload == "batch":
        args.tol_mixed = args.batch_tol_mixed
        print(json.dumps(run_batch(args, [x for x in args.forms.split(",") if x])), flush=True)
        return
    if args.workload == "evolve":
        print(json.dumps(run_evolve(args)), flush=True)
        return
    if args.workload == "laplace":
        print(json.dumps(run_laplace(args)), flush=True)
        return
    if args.workload == "holes":
        print(json.dumps(run_holes(args)), flush=True)
        return
    if args.copy_calibration_mb > 0:
        nel = args.copy_calibration_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = WORKLOADS[args.workload]
    geom = make_geometry(args.workload)
    f = boundary_data(geom, exterior_forces_for_geometry(geom, wl["nrhs"], seed=wl["seed"]))
    nrhs = f.shape[1]
    forms = [x for x in args.forms.split(",") if x]
    runs = {}
    for fm in forms:
        print("bench: %s form on %s" % (fm, args.workload), file=sys.stderr, flush=True)
        runs[fm] = run_form(geom, f, fm, args.steps, args.warmup, args.tol_plain, args.tol_mixed, wl["roofline"])
    head = runs[forms[0]]
    tol_head = args.tol_mixed if forms[0] == "mixed" else args.tol_plain
    out = {
        "metric": "RS factor s + solves/s at 1e-8 rel. residual, mixed-batched vs FP64 plain",
        "value": head["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if forms[0] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "desc": wl["desc"], "nrhs": nrhs, "form": forms[0],
                   "tol": tol_head, "refine_tol": 1e-8, "leaf": 64, "n_proxy": 64},
        "factor_s": head["factor_s"],
        "solve_s": head["solve_s"],
        "refine_iters": head["refine_iters"],
        "max_rel_residual": head["max_rel_residual"],
        "setup_ms": head["setup_ms"],
        "kernel_ms_per_step": {k: v[1] / BREAKDOWN_STEPS for k, v in sorted(head["kbreak"].items())},
        "kernel_breakdown_steps": BREAKDOWN_STEPS,
        "roofline": roofline_of(head, args.steps, nrhs, geom.n_nodes, args.workload, forms[0], tol_head,
                                wl["roofline"]),
    }
    for fm in forms[1:]:
        r = runs[fm]
        out["form_" + fm] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                             "factor_s": r["factor_s"], "solve_s": r["solve_s"],
                             "refine_iters": r["refine_iters"],
                             "max_rel_residual": r["max_rel_residual"],
                             "kernel_ms_per_step": {k: v[1] / BREAKDOWN_STEPS
                                                    for k, v in sorted(r["kbreak"].items())},
                             "roofline": roofline_of(r, args.steps, nrhs, geom.n_nodes, args.workload, fm,
                                                     args.tol_plain if fm == "plain" else args.tol_mixed,
                                                     wl["roofline"])}
        out["speedup_vs_" + fm] = head["value"] / r["value"]
        out["factor_speedup_vs_" + fm] = r["factor_s"] / head["factor_s"]
    if args.batch_size > 0:
        print("bench: batch of %d geometries" % args.batch_size, file=sys.stderr, flush=True)
        bargs = argparse.Namespace(**vars(args))
        bargs.steps, bargs.warmup, bargs.tol_mixed = args.batch_steps, 3, args.batch_tol_mixed
        b = run_batch(bargs, forms)
        out["batch"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "steps", "config", "max_rel_residual")}
        for fm in forms[1:]:
            out["batch"]["form_" + fm] = b["form_" + fm]
            out["batch"]["speedup_vs_" + fm] = b["speedup_vs_" + fm]
        out["batch"]["config"]["tol_mixed"] = args.batch_tol_mixed
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        try:
            out["cpu_baseline"] = cpu_baseline(geom, f, args.tol_plain, full=geom.n_nodes <= 20000)
        except Exception as e:      # the GPU figures above stand without it
            out["cpu_baseline"] = {"error": "%s: %s" % (type(e).__name__, e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
