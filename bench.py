#!/usr/bin/env python3
"""Benchmark of the FEA + sensitivity step on one MI355X.

One step = one full pass of the hot path for every design of the workload:
SIMP moduli, the preconditioner set-up (element-block Schwarz inverses,
vertex-grid Galerkin operators, coarsest-grid inverse; or the Jacobi
diagonal), matrix-free PCG to rtol 1e-11 (true residual checked in
double-double), compliance and sensitivities, replayed from captured HIP
graphs.  Inputs (densities) are resident in HBM before timing starts.

Default workload (the largest configuration): a batch of 64 independent
mixed-order cantilever designs of 40 x 20 to 314 x 157 elements (p in
{1, 2, 4}, d in {1, 2, 5} by the dp rule, 1-3 point-load cases each), FP64,
seeded Gaussian-smoothed density fields at mean density 0.5, all solved in
one plan; value = step time / 64.  The 160 x 80 uniform p = 3, d = 4
cantilever is timed beside it as a secondary workload.

Prints one JSON line (metric, value in seconds per design, roofline of the
element-contraction kernel, the plain per-element GPU path at the same
tolerance, CPU-oracle baseline on the host cores, and the launch time of the
density filter of Sec. 2.2 and its chain rule on the same cells, of the
QR-error indicator of Sec. 3.2.3 and the other refinement indicators and
the dp update of Sec. 3.2-3.3 on the solved designs, and of the force
inverter of Sec. 4.1 (input and adjoint solves with ground springs, adjoint
sensitivity) on a 160 x 80 p = 3, d = 4 mesh, all outside the timed step).
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contraction_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1811_09821_amd", "csrc", "mto_kernels.hip")
# tile shapes of the element contraction measured on gfx950, per (p, d, size class)
TILE_CACHE = os.path.join(ROOT, "paper_1811_09821_amd", "tiles_gfx950.txt")


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def workload(k, solid_paths=False):
    from paper_1811_09821_amd import problems as P

    field = ", eased field (solid load paths)" if solid_paths else ""
    if k == 2:
        return [P.config(2, solid_paths)], f"cantilever 160x80, uniform p=3 d=4, FP64, 1 load{field}"
    if k == 3:
        return [P.config(3, solid_paths)], f"mixed dp mesh 200x100, p in {{1,2,4}}, d in {{1,2,5}}, FP64, 1 load{field}"
    if k == 5:
        return [P.config(5, solid_paths)], f"mixed dp mesh 400x200, 3 loads, FP64{field}"
    if k == 4:
        return P.config(4, solid_paths), f"batch of 64 designs 40x20..314x157, mixed dp, 1-3 loads each, FP64{field}"
    if k == 1:
        return [P.config(1)], "MBB 20x10, p=1 d=2, FP64"
    raise SystemExit(f"unknown config {k}")


def _oracle_one(pr):
    """One whole oracle design step (run in a worker process)."""
    from threadpoolctl import threadpool_limits

    from oracle import oracle_solve

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle_solve(**pr.oracle_args())
        return time.perf_counter() - t0


def cpu_baseline(prs, max_designs=16):
    """The oracle as it is, on the host cores: a sample of whole designs of
    the workload (every len(prs) / max_designs-th design), one design per
    worker process (SuperLU is serial; BLAS limited to one thread per
    worker).  Returns (wall seconds per design, designs, workers, summed
    single-design seconds).  Run before the GPU is initialised, so the
    workers are plain forks of a CPU-only process."""
    import multiprocessing as mp

    stride = max(1, len(prs) // max_designs)
    sample = prs[::stride][:max_designs]
    workers = max(1, min(len(sample), 16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        single = pool.map(_oracle_one, sample, chunksize=1)
    wall = time.perf_counter() - t0
    return wall / len(sample), len(sample), workers, sum(single), stride


def time_filter(mto, prs, rho, R, reps=200):
    """Density filter (Sec. 2.2, Eqs. (4)-(5)) and its chain rule on the same
    cells: average launch time over `reps` back-to-back launches, and the
    HBM rate on algorithmic bytes (x, 1/rowsum and y once per cell; an index
    and a weight per nonzero of H)."""
    import torch

    F = mto.Filter(prs, R)
    y = F.apply(rho)
    g = F.grad(y)
    st = torch.cuda.current_stream()
    res = {"R": R, "n_cells": F.n_cells, "nnz": F.nnz}
    nbytes = 24 * F.n_cells + 12 * F.nnz
    for name, fn, x, out in (("apply", mto.lib().mto_filter_apply, rho, y), ("grad", mto.lib().mto_filter_grad, y, g)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(5):
            mto._check(fn(F.handle, mto._ptr(x), mto._ptr(out), mto._stream(st)))
        e0.record(st)
        for _ in range(reps):
            mto._check(fn(F.handle, mto._ptr(x), mto._ptr(out), mto._stream(st)))
        e1.record(st)
        e1.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        res[f"{name}_us"] = round(us, 3)
        res[f"{name}_GBps"] = round(nbytes / (us * 1e-6) / 1e9, 1)
    res["bytes_per_launch"] = nbytes
    res["hbm_frac_apply"] = round(res["apply_GBps"] / 8000.0, 4)
    return res


def time_mechanism(mto, args, steps=3, rtol=1e-13):
    """Force inverter of Sec. 4.1 (half model, ground springs k_in = 1 and
    k_out = 0.001) on a 160 x 80 mesh of p = 3, d = 4 elements: one design =
    the solve of the input and the adjoint load case (graph replay), J = u_out
    and dJ/drho from the bilinear sensitivity kernel.  rtol 1e-13, the
    tolerance its parity tests use: the soft output spring conditions the
    inverter worse than the compliance workloads."""
    import torch

    from paper_1811_09821_amd import problems as P

    pr = P.force_inverter(160, 80, p=3, d=4, volfrac=0.45, seed=8, sigma=8.0)
    plan = mto.Plan(pr, rtol=rtol)
    rho = torch.tensor(pr.rho, device="cuda:0")
    u, c, _ = plan.capture(rho)
    n = plan.instances[0]["n_dof"]
    out = 2 * (pr.out_dof[1] * (pr.nelx + 1) + pr.out_dof[0]) + pr.out_dof[2]
    stats = plan.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stats = plan.replay()
        lam = torch.cat([u[n:2 * n], u[:n]])
        g = plan.adjoint_sensitivity(rho, u, lam)
        J = u[out]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"workload": "force inverter 160x80 (half model), p=3 d=4, springs k_in=1 k_out=0.001, FP64",
            "rtol": rtol, "s_per_design": round(dt, 6), "pcg_iterations": stats["iterations"], "J": float(J),
            "n_free_dofs_per_case": plan.info["n_free_total"] // 2, "grad_norm": float(g[:pr.n_cells].norm())}


def time_adapt(mto, plan, prs, rho, u, reps=5):
    """Refinement indicators of Sec. 3.2 (Kelly, density) on the solved
    designs and the host dp update of Sec. 3.3 on the first design: mean
    time per call."""
    import numpy as np
    import torch

    st = torch.cuda.current_stream()
    res = {}
    for name, fn in (("kelly", lambda: plan.kelly_indicator(u)), ("density", lambda: plan.density_indicator(rho, 1))):
        out = fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            out = fn()
        e1.record(st)
        e1.synchronize()
        res[f"{name}_ms"] = round(e0.elapsed_time(e1) / reps, 4)
        res[f"{name}_out"] = out
    pr = prs[0]
    ga = res.pop("kelly_out")[:pr.nelx * pr.nely].cpu().numpy()
    gd = res.pop("density_out")[:pr.nelx * pr.nely].cpu().numpy()
    t0 = time.perf_counter()
    p_new, theta, dp, cells = mto.dp_update(pr.nelx, pr.nely, pr.p, ga, gd)
    res["dp_update_host_ms"] = round(1e3 * (time.perf_counter() - t0), 3)
    res["refined"] = int((p_new > pr.p).sum())
    res["coarsened"] = int((p_new < pr.p).sum())
    res["cells_per_element"] = cells
    return res


def time_qr(plan, rho, u, reps=5):
    """QR-error indicator (Sec. 3.2.3, Eq. (9)) for every element and load
    case of the solved designs: mean time per call over `reps` calls after
    one untimed call (which builds the order-(p+1) tables)."""
    import torch

    eps = plan.qr_error(rho, u)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        eps = plan.qr_error(rho, u)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"ms_per_call": round(ms, 4), "element_problems": plan.n_eps,
            "element_problems_per_s": round(plan.n_eps / (ms * 1e-3), 1),
            "eps_mean": round(float(eps.mean()), 6), "eps_gt_0.9": int((eps > 0.9).sum())}


def progress(msg):
    """One progress line on stderr (the JSON result goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def traffic_for(config, shapes, path):
    """Scaled FETCH_SIZE + WRITE_SIZE per contraction launch from the committed
    counter summary, if it was taken of the current kernel source, this
    workload and these tile shapes (else None)."""
    if path != "mfma" or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    for rec in tr.get("records", []):
        if (rec.get("kernel_source_sha256_16") == kernel_source_hash() and rec.get("config") == config
                and rec.get("tile_shapes") == shapes):
            return rec.get("bytes_per_launch")
    return None


def tile_shapes(report):
    """'p d ncol ks' of every group from an autotune report."""
    out = []
    for ln in report.strip().splitlines():
        if ln.endswith(": chosen"):
            kv = dict(t.split("=") for t in ln.split(":")[0].split() if "=" in t)
            out.append(f"{kv['p']} {kv['d']} {kv['ncol']} {kv['ks']}")
    return sorted(out)


def run_workload(mto, args, config, prs, path, precond, steps, warmup, tune=True):
    """Plan, tile shapes, capture, `warmup` + `steps` timed replays of the
    whole step, then the contraction timings.  Returns the plan, the
    measurement dict and the bound (rho, u)."""
    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    plan = mto.Plan(prs, kernel_path=path, precond=precond, mg_coarse_max=args.mg_coarse_max,
                    iters_per_launch=args.iters_per_launch)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device=dev)
    report = ""
    if path == mto.PATH_MFMA and tune:
        report = plan.autotune(rho, cache=args.tile_cache or None)
    u, c, g = plan.capture(rho)
    stats = None
    for _ in range(warmup):
        stats = plan.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stats = plan.replay()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_designs = len(prs)
    res = {"s_per_design": elapsed / steps / n_designs, "ms_per_step": 1e3 * elapsed / steps,
           "designs_per_step": n_designs, "stats": stats, "report": report}
    return plan, res, rho, u


def contraction_roofline(plan, rho, stats, config, path_name, shapes):
    """Roofline of the dominant kernel, the element contraction (one PCG
    product K p over all (p, d) groups): useful flops of one product over the
    mean duration of 100 back-to-back launches between two events on the
    plan's stream; the duration inside eagerly run PCG iterations (events on
    each dispatch packet, a few microseconds of dispatch overhead each) is
    reported beside it."""
    it_min = min(stats["iterations"]) if stats else 100
    reps = max(1, min(100, it_min // 3))
    t_loop_ms = plan.time_contraction(rho, reps=reps, in_loop=True)
    t_mv_ms = plan.time_contraction(rho, reps=100)
    flops = plan.info["flops_per_matvec"]
    achieved = flops / (t_mv_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4), "traffic": traffic_for(config, shapes, path_name),
            "kernel": "k_elem_mfma (element contraction of every (p, d) group, PCG search direction)",
            "flops_per_launch": flops, "ms_per_launch": round(t_mv_ms, 5), "launches_timed": 100,
            "ms_per_launch_in_pcg_loop": round(t_loop_ms, 5), "in_loop_reps": reps,
            "frac_in_pcg_loop": round(flops / (t_loop_ms * 1e-3) / 1e12 / PEAK_FP64_MFMA_TFLOPS, 4),
            "tile_shapes": shapes}


def time_stored(mto, args, prs, rho, precond, shapes):
    """The same step with stored element matrices (K_e assembled in the set-up,
    each product reading it: HBM-bound) for the p = 4 groups and the timed
    contraction shapes elsewhere, outside the headline: the alternative to the
    MFMA contraction that the autotuner takes with stored_matrices = 1."""
    import numpy as np
    import torch

    plan = mto.Plan(prs, precond=precond, stored_matrices=1)
    plan.autotune(rho, cache=args.tile_cache or None)
    for s in shapes:
        p, d = (int(v) for v in s.split()[:2])
        if p == 4:
            plan.set_tile(1, -2, p=p, d=d)
    plan.capture(rho)
    plan.replay()
    torch.cuda.synchronize()
    reps = max(2, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        st = plan.replay()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    its = st["iterations"]
    ms = plan.time_contraction(rho, reps=50)
    del plan
    return {"s_per_design": el / len(prs), "ms_per_step": 1e3 * el, "product_ms": round(ms, 5),
            "pcg_iterations": {"mean": round(float(np.mean(its)), 2), "max": max(its)},
            "kernel": "k_elem_stored (p = 4 groups) + the contraction of the other groups"}


def contraction_only(args, prs, desc):
    """Plan, cached tile shapes, then 100 back-to-back launches of the element
    contraction (after the solve set-up), optionally followed by one device
    copy of known size: the command that hardware counters are taken of."""
    import numpy as np
    import torch

    from paper_1811_09821_amd import mto

    plan = mto.Plan(prs)
    rho = torch.tensor(np.concatenate([p.rho for p in prs]), device="cuda:0")
    report = plan.autotune(rho, cache=args.tile_cache or None)
    ms = plan.time_contraction(rho, reps=100)
    out = {"workload": desc, "ms_per_launch": ms, "tile_shapes": tile_shapes(report),
           "flops_per_launch": plan.info["flops_per_matvec"]}
    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * n * 8
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4, help="workload 1..5 (default 4, the 64-design batch)")
    ap.add_argument("--eased-field", action="store_true",
                    help="density fields with solid load paths instead of the plain random field")
    ap.add_argument("--path", choices=["mfma", "plain"], default="mfma")
    ap.add_argument("--precond", choices=["schwarz-mg", "jacobi", "l1-mg"], default="schwarz-mg",
                    help="PCG preconditioner (default: multigrid with element-block Schwarz smoothing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--iters-per-launch", type=int, default=0,
                    help="PCG iterations per captured chunk graph (0: the library default)")
    ap.add_argument("--mg-coarse-max", type=int, default=0,
                    help="DOFs of the coarsest multigrid grid at most (0: the library default)")
    ap.add_argument("--tile-cache", default=TILE_CACHE,
                    help="tile-shape cache file of the autotuner ('' times every shape)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-element GPU path")
    ap.add_argument("--no-stored", action="store_true",
                    help="skip the step with stored element matrices for the p = 4 groups")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary workload (config 2)")
    ap.add_argument("--filter-radius", type=float, default=0.3,
                    help="density-filter radius in element edge lengths for the filter timing (0 skips it)")
    ap.add_argument("--no-qr", action="store_true", help="skip the QR-error indicator timing")
    ap.add_argument("--no-mechanism", action="store_true",
                    help="skip the force inverter (compliant mechanism) timing on a 160x80 p=3 d=4 mesh")
    ap.add_argument("--contraction-only", action="store_true",
                    help="only plan, tile shapes and 100 back-to-back contraction launches (for counter runs)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB (a known-size kernel "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    prs, desc = workload(args.config, args.eased_field)
    if args.contraction_only:
        contraction_only(args, prs, desc)
        return
    # The CPU baseline first, before anything initialises the GPU, so that its
    # workers are forks of a CPU-only process.
    cpu = None
    if not args.no_cpu_baseline:
        progress(f"CPU oracle baseline on a sample of {len(prs)} design(s)")
        t_cpu, n_s, workers, single, stride = cpu_baseline(prs)
        cpu = {"value": t_cpu, "unit": "s/design", "cores": workers,
               "host_cores_available": len(os.sched_getaffinity(0)), "kind": "oracle",
               "sample": f"{n_s} whole design(s) of the same workload (every {stride}-th), one per worker process: "
                         f"assembled sparse K, SuperLU + longdouble refinement, c and dc/drho; BLAS limited to "
                         f"1 thread per worker; value = wall time / designs",
               "single_core_s_per_design": single / n_s}

    import numpy as np
    import torch

    from paper_1811_09821_amd import mto

    dev = torch.device("cuda:0")
    path = mto.PATH_MFMA if args.path == "mfma" else mto.PATH_PLAIN
    precond = {"jacobi": mto.PRECOND_JACOBI, "l1-mg": mto.PRECOND_MG, "schwarz-mg": mto.PRECOND_MG_ASM}[args.precond]
    progress(f"config {args.config}: plan, tiles, capture, {args.warmup} + {args.steps} replays")
    plan, res, rho, u = run_workload(mto, args, args.config, prs, path, precond, args.steps, args.warmup,
                                     tune=not args.no_autotune)
    progress(f"config {args.config}: {res['s_per_design']:.6f} s/design; contraction roofline")
    stats = res["stats"]
    shapes = tile_shapes(res["report"])
    roof = contraction_roofline(plan, rho, stats, args.config, args.path, shapes)
    its = stats["iterations"] if stats else None

    out = {
        "metric": "solve+sensitivity s/design; element-contraction FP64 MFMA % of peak; 1 GPU",
        "value": res["s_per_design"],
        "unit": "s/design",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian-smoothed density fields; the paper's designs exist only as figures)",
        "config": {"workload": desc, "designs_per_step": res["designs_per_step"],
                   "n_systems": plan.n_systems, "n_free_dofs": plan.info["n_free_total"],
                   "n_cells": plan.info["n_cells"], "rtol": 1e-11, "kernel_path": args.path,
                   "preconditioner": args.precond, "parallelism": "single GPU"},
        "pcg_iterations": its if its is None or len(its) <= 8 else
        {"min": min(its), "max": max(its), "mean": round(float(np.mean(its)), 2), "per_system": its},
        "true_rel_residual_max": max(stats["true_rel_residual"]) if stats else None,
        "restarts": stats["restarts"] if stats else None,
        "contraction_mfma_pct_of_peak": roof["frac"] * 100,
        "roofline": roof,
    }
    if res["report"]:
        out["autotune"] = res["report"].strip().splitlines()

    if not args.no_stored and path == mto.PATH_MFMA and any(int(s.split()[0]) == 4 for s in shapes):
        progress("stored element matrices for the p = 4 groups")
        out["stored_element_matrices"] = time_stored(mto, args, prs, rho, precond, shapes)

    if not args.no_plain and path == mto.PATH_MFMA:
        progress("plain per-element path")
        plain = mto.Plan(prs, kernel_path=mto.PATH_PLAIN, precond=precond)
        plain.capture(rho)
        plain.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_p = plain.replay()
        torch.cuda.synchronize()
        out["plain_path"] = {"s_per_design": (time.perf_counter() - t1) / len(prs), "rtol": 1e-11,
                             "contraction_ms_in_pcg_loop": plain.time_contraction(rho, reps=10, in_loop=True),
                             "max_iterations": max(st_p["iterations"]),
                             "kernel": "k_elem_plain (one lane per element column, FP64 VALU)"}
        del plain

    if not args.no_secondary and args.config != 2:
        progress("secondary workload: config 2")
        prs2, desc2 = workload(2, args.eased_field)
        plan2, res2, rho2, _ = run_workload(mto, args, 2, prs2, path, precond, max(args.steps, 20), args.warmup)
        shapes2 = tile_shapes(res2["report"])
        roof2 = contraction_roofline(plan2, rho2, res2["stats"], 2, args.path, shapes2)
        out["secondary"] = {"workload": desc2, "s_per_design": res2["s_per_design"],
                            "pcg_iterations": res2["stats"]["iterations"],
                            "true_rel_residual": res2["stats"]["true_rel_residual"],
                            "roofline": roof2}
        del plan2

    progress("filter, QR-error and refinement indicators, force inverter")
    if args.filter_radius > 0:
        out["density_filter"] = time_filter(mto, prs, rho, args.filter_radius)
    if not args.no_qr:
        out["qr_error"] = time_qr(plan, rho, u)
    if not args.no_qr:
        out["adapt"] = time_adapt(mto, plan, prs, rho, u)
    if not args.no_mechanism:
        out["mechanism"] = time_mechanism(mto, args)

    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * n * 8

    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
