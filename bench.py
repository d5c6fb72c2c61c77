"""Benchmark: DOFs solved per second by global-local MG-preconditioned CG.

Workload (default): 2D Poisson on a 1025x1025 jittered triangulation of the
unit square with 256 clusters of 1-8 degraded cells, P2 elements (4.2M DOFs),
Dirichlet on y = 0, 1, four non-nested coarse levels (513^2 ... 65^2 vertex
grids), combined smoother S_c -> Chebyshev-Jacobi(2) -> S_c with the adjusted
lambda_max, V(2,2) cycle, CG to rtol 1e-8, FP64 on the GPU.

A step is one MG-PCG solve of one synthetic right-hand side (uniform [-1, 1],
seeded, resident in HBM before the timed region) with the hierarchy already
set up; setup time is reported separately.  value = total DOFs solved / time.
The level-0 Chebyshev-Jacobi kernel is timed with HIP events on the library's
stream during the timed steps for the roofline entry.  Extra arms (plain
smoother, mixed precision) are reported as extra fields.  The CPU baseline is
the oracle on a bounded sample (the same recipe at 1/8 of the size per side).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (meshgen recipe, degree, scale, layers, rtol, patch policy[, problem])
    "square_1025_p2": ("square_1025", 2, 1, 1, 1e-8, "merge"),
    "square_1025_p3": ("square_1025", 3, 1, 1, 1e-8, "merge"),
    "cube_129_p1": ("cube_129", 1, 1, 1, 1e-8, "merge"),
    "cube_129_p2": ("cube_129", 2, 1, 1, 1e-8, "merge"),
    "square_p1_4k": ("square_p1_4k", 1, 1, 2, 1e-10, "merge"),
    # patch stress: ~20k separate flattened regions, the regions themselves
    # are the subdomains (no extension layer), ~40 % of the DOFs in patches
    "cube_129_stress_p2": ("cube_129_stress", 2, 1, 0, 1e-8, "overlap"),
    # linear elasticity on the truss-like lattice (vector P1 / P2, E = 6.9e10,
    # nu = 0.33, clamped at x = 0), four levels
    "lattice_96_p1": ("lattice_96", 1, 1, 1, 1e-8, "merge", "elasticity"),
    "lattice_96_p2": ("lattice_96", 2, 1, 1, 1e-8, "merge", "elasticity"),
}
# many-instance workload: 32 unit-cube problems of 50k-3M DOFs, 4 right-hand sides each
BATCH_WORKLOADS = {"cube_batch_32x4": (32, 4, 1), "cube_batch_small": (4, 2, 4)}
PEAK_HBM_GBS = 8000.0
CHEB_KERNEL = "k_cheb"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("solve.hip", "sell_row.h", "mg_internal.h"):
        with open(os.path.join(ROOT, "paper_2402_12947_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, precision: str):
    """HBM bytes per launch of the Chebyshev kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"cheb_step_{workload}_{precision}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_arm(meshes, degree, layers, rtol, steps, warmup, precision="fp64", local=True, timing=False,
            use_graph=False, seed0=1000, sigma=0, policy="merge", smoother="chebyshev", problem="poisson"):
    import torch

    from paper_2402_12947_amd import Solver
    log(f"setup precision={precision} local={local}")
    t0 = time.perf_counter()
    s = Solver(meshes, degree=degree, tau=0.1, layers=layers, precision=precision,
               local_correction=local, adjusted_eig=local, use_graph=use_graph, sell_sigma=sigma, policy=policy,
               global_smoother=smoother, problem=problem)
    setup_s = time.perf_counter() - t0
    n = s.n_free(0)
    log(f"setup done in {setup_s:.2f} s, {n} DOFs; solving")
    bs = [torch.as_tensor(_rhs(n, seed0 + k)).cuda() for k in range(steps + warmup)]
    us = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(steps + warmup)]
    its = []
    for k in range(warmup):
        st = s.pcg(bs[k], us[k], rtol, 1000)
        its.append(st["iterations"])
    if timing:
        s.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(warmup, warmup + steps):
        stats.append(s.pcg(bs[k], us[k], rtol, 1000))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = {"n": n, "setup_s": setup_s, "elapsed_s": elapsed, "iterations": [x["iterations"] for x in stats],
           "converged": all(x["converged"] for x in stats),
           "true_rel_residual": max(x["true_rel_residual"] for x in stats),
           "levels": [s.level_info(l) for l in range(s.n_levels)],
           # the solution of the first timed right-hand side (seed seed0 + warmup)
           "first_seed": seed0 + warmup, "first_solution": us[warmup].cpu().numpy()}
    if timing and smoother == "chebyshev":
        launches, total_ms = s.kernel_time()
        out["cheb_launches"] = launches
        out["cheb_avg_ms"] = total_ms / max(launches, 1)
        out["cheb_bytes"] = s.cheb_bytes()
        s.enable_kernel_timing(False)
    s.close()
    return out


def _rhs(n, seed):
    import meshgen
    return meshgen.random_rhs(n, seed)


def cpu_baseline(recipe, degree, layers, rtol, scale, policy="merge", problem="poisson", budget_s=12.0):
    import meshgen
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        ctx = None
    meshes = meshgen.hierarchy(recipe, seed=0, scale=scale)
    H = oracle.Hierarchy(meshes, tau=0.1, layers=layers,
                         opts=oracle.Options(degree=degree, patch_policy=oracle.OVERLAP if policy == "overlap"
                                             else oracle.MERGE, problem=problem))
    n = H.levels[0].A.shape[0]
    solved, t0 = 0, time.perf_counter()
    its = []
    while True:
        _, it, conv, _ = H.pcg(_rhs(n, 5000 + solved), rtol, 1000)
        its.append(it)
        solved += 1
        el = time.perf_counter() - t0
        if el >= budget_s or solved >= 50:
            break
    if ctx is not None:
        ctx.unregister() if hasattr(ctx, "unregister") else None
    return {"value": n * solved / el, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"{recipe} recipe at 1/{scale} size per side (P{degree}, {n} DOFs, "
                      f"{len(meshes)} levels), {solved} full MG-PCG solves to rtol {rtol:g}, setup untimed, "
                      f"iterations {its[0]}"}


def run_study(scale=4):
    """The paper's Poisson study (Sec. 6.1) on the GPU: multigrid as a stationary
    solver and as a CG preconditioner, plain Chebyshev vs global-local
    smoother, on the reference mesh (no degraded cells), degraded cells on the
    finest level, on every level (Case A) and on the coarse levels only
    (Case B).  One JSON line per (workload, case, smoother)."""
    import torch

    import meshgen
    from paper_2402_12947_amd import MgError, Solver
    for recipe, degree in (("square_1025", 2), ("cube_129", 2)):
        for case in ("ref", "fine", "A", "B"):
            meshes = meshgen.hierarchy(recipe, seed=0, scale=scale, case=case)
            ref_x = None
            for smoother in ("global_local", "plain"):
                local = smoother == "global_local"
                rec = {"study": f"{recipe}/{scale} P{degree}", "case": case, "smoother": smoother}
                try:
                    s = Solver(meshes, degree=degree, tau=0.1, layers=1, local_correction=local, adjusted_eig=local)
                except MgError as e:
                    rec["error"] = str(e)
                    print(json.dumps(rec), flush=True)
                    continue
                n = s.n_free(0)
                b = torch.as_tensor(_rhs(n, 77)).cuda()
                if ref_x is None:  # the solution, from the global-local PCG to rtol 1e-13
                    ref_x = torch.zeros(n, dtype=torch.float64, device="cuda")
                    s.pcg(b, ref_x, 1e-13, 500)
                u = torch.zeros(n, dtype=torch.float64, device="cuda")
                st12 = s.mg_solve(b, u, 1e-300, 12)
                err12 = float(torch.linalg.norm(u - ref_x) / torch.linalg.norm(ref_x))
                st = s.mg_solve(b, torch.zeros_like(u), 1e-8, 300)
                pc = s.pcg(b, torch.zeros_like(u), 1e-8, 500)
                rec.update({"dofs": n, "flagged_level0": s.level_info(0)["n_flagged"],
                            "mg_cycles_to_1e-8": st["iterations"] if st["converged"] else None,
                            "mg_rel_error_after_12_cycles": err12,
                            "mg_residual_after_12_cycles": st12["rel_residual"],
                            "pcg_iterations_to_1e-8": pc["iterations"] if pc["converged"] else None})
                print(json.dumps(rec), flush=True)
                s.close()


def run_batch(name, steps, warmup):
    """Many-instance solve: every instance's hierarchy in mixed precision with
    graph-captured V-cycles, all instances solved together by
    mg_pcg_solve_batch, against the same systems solved one by one in FP64."""
    import torch

    import meshgen
    from paper_2402_12947_amd import Solver, pcg_solve_batch
    count, nrhs, scale = BATCH_WORKLOADS[name]
    log(f"generating {count} instances")
    inst = meshgen.instance_batch(count, seed=0, scale=scale,
                                  progress=lambda i, m, d: log(f"instance {i}: P{d}, {m[0]['cells'].shape[0]} cells"))
    t0 = time.perf_counter()
    fast = []
    for i, (m, d) in enumerate(inst):
        fast.append(Solver(m, degree=d, precision="mixed", use_graph=True))
        log(f"set up instance {i}")
    setup_fast = time.perf_counter() - t0
    ns = [s.n_free(0) for s in fast]
    total = sum(ns) * nrhs
    log(f"mixed+graph setup {setup_fast:.1f} s, {sum(ns)} DOFs x {nrhs} right-hand sides")
    bs = [[torch.as_tensor(_rhs(n, 100 * i + r)).cuda() for r in range(nrhs)] for i, n in enumerate(ns)]
    us = [[torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(nrhs)] for n in ns]
    for _ in range(warmup):
        pcg_solve_batch(fast, bs, us, 1e-8, 1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(steps):
        res = pcg_solve_batch(fast, bs, us, 1e-8, 1000)
        its = [x["iterations"] for x in res["stats"]]
        assert all(x["converged"] for x in res["stats"])
    torch.cuda.synchronize()
    el_fast = time.perf_counter() - t0
    worst_fast = max(x["true_rel_residual"] for x in res["stats"])
    # the same batch with the right-hand sides of an instance one at a time
    # (instances still overlapped): what the block solve saves
    log("unblocked arm: one right-hand side per instance at a time")
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in range(nrhs):
            pcg_solve_batch(fast, [[row[r]] for row in bs], [[row[r]] for row in us], 1e-8, 1000)
    torch.cuda.synchronize()
    el_unblocked = time.perf_counter() - t0
    for s in fast:
        s.close()
    log("FP64 one-by-one baseline")
    t0 = time.perf_counter()
    slow = []
    for i, (m, d) in enumerate(inst):
        slow.append(Solver(m, degree=d, precision="fp64"))
        log(f"set up FP64 instance {i}")
    setup_slow = time.perf_counter() - t0
    for i, s in enumerate(slow):
        s.pcg(bs[i][0], us[i][0], 1e-8, 1000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_slow = []
    for i, s in enumerate(slow):
        for r in range(nrhs):
            its_slow.append(s.pcg(bs[i][r], us[i][r], 1e-8, 1000)["iterations"])
    torch.cuda.synchronize()
    el_slow = time.perf_counter() - t0
    for s in slow:
        s.close()
    value = total * steps / el_fast
    base = total / el_slow
    return {
        "metric": "aggregate DOFs solved/sec to rtol 1e-8 (batched mixed MG-PCG, graph-captured V-cycles)",
        "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": 1e3 * el_fast / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-in-f64", "data": "synthetic (seeded meshes and right-hand sides)",
        "config": {"workload": name, "instances": count, "rhs_per_instance": nrhs, "dofs_total": sum(ns),
                   "setup_s": round(setup_fast, 2), "iterations_min_max": [min(its), max(its)],
                   "worst_true_rel_residual": worst_fast},
        "unblocked_dofs_per_s": total * steps / el_unblocked,
        "one_by_one_fp64": {"dofs_per_s": base, "setup_s": round(setup_slow, 2),
                            "iterations_min_max": [min(its_slow), max(its_slow)]},
        "speedup_vs_one_by_one_fp64": value / base,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="square_1025_p2", choices=sorted(WORKLOADS) + sorted(BATCH_WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--arms", default="gl,plain,mixed", help="comma list of gl, plain, mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay the V-cycle from a hipGraph")
    ap.add_argument("--sigma", type=int, default=0, help="SELL sorting window (0 = library's choice)")
    ap.add_argument("--smoother", default="chebyshev", choices=["chebyshev", "sgs"],
                    help="global smoother S_g of every arm (the roofline entry needs chebyshev)")
    ap.add_argument("--study", action="store_true",
                    help="instead of the benchmark line: the stationary-solver / preconditioner study of "
                         "plain vs global-local smoothing on the reference mesh and Cases A and B")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write kernel (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (single-GPU build); "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    import torch
    import meshgen
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.study:
        run_study()
        return
    if args.workload in BATCH_WORKLOADS:
        print(json.dumps(run_batch(args.workload, args.steps, args.warmup)), flush=True)
        return
    recipe, degree, scale, layers, rtol, policy = WORKLOADS[args.workload][:6]
    problem = WORKLOADS[args.workload][6] if len(WORKLOADS[args.workload]) > 6 else "poisson"
    meshes = meshgen.hierarchy(recipe, seed=0, scale=scale)
    arms = args.arms.split(",")
    main_arm = run_arm(meshes, degree, layers, rtol, args.steps, args.warmup, precision=args.precision,
                       local=True, timing=True, use_graph=args.graph, sigma=args.sigma, policy=policy,
                       smoother=args.smoother, problem=problem)
    n = main_arm["n"]
    value = n * args.steps / main_arm["elapsed_s"]
    extra = {}
    if "plain" in arms:
        p = run_arm(meshes, degree, layers, rtol, max(1, args.steps // 2), 1, precision="fp64", local=False,
                    smoother=args.smoother, problem=problem)
        extra["plain_fp64"] = {"dofs_per_s": p["n"] * len(p["iterations"]) / p["elapsed_s"],
                               "iterations": p["iterations"][0], "setup_s": round(p["setup_s"], 3),
                               "true_rel_residual": p["true_rel_residual"]}
    if "mixed" in arms and args.precision == "fp64":
        mx = run_arm(meshes, degree, layers, rtol, args.steps, 1, precision="mixed", local=True, policy=policy,
                     smoother=args.smoother, problem=problem, timing=args.smoother == "chebyshev")
        extra["global_local_mixed"] = {"dofs_per_s": mx["n"] * len(mx["iterations"]) / mx["elapsed_s"],
                                       "iterations": mx["iterations"][0], "setup_s": round(mx["setup_s"], 3),
                                       "true_rel_residual": mx["true_rel_residual"]}
        if "cheb_avg_ms" in mx:
            # the same level-0 Chebyshev step in FP32 (values 4 bytes, vectors 4 bytes)
            extra["global_local_mixed"]["level0_cheb_fp32"] = {
                "avg_launch_ms": round(mx["cheb_avg_ms"], 5), "algorithmic_bytes_per_launch": mx["cheb_bytes"],
                "achieved_gbs": round(mx["cheb_bytes"] / (mx["cheb_avg_ms"] * 1e-3) / 1e9, 1)}
        if mx["first_seed"] == main_arm["first_seed"]:
            # same right-hand side, same rtol: distance of the mixed-precision
            # solution from the FP64 one (which the parity tests tie to the oracle)
            import numpy as np
            x64, xmx = main_arm["first_solution"], mx["first_solution"]
            extra["global_local_mixed"]["rel_diff_vs_fp64_solution"] = float(
                np.linalg.norm(xmx - x64) / max(np.linalg.norm(x64), 1e-300))
    roofline = None
    if args.smoother == "chebyshev":
        avg_ms = main_arm["cheb_avg_ms"]
        achieved = main_arm["cheb_bytes"] / (avg_ms * 1e-3) / 1e9
        traffic = read_traffic(args.workload, args.precision)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                    "kernel": CHEB_KERNEL, "avg_launch_ms": round(avg_ms, 5),
                    "algorithmic_bytes_per_launch": main_arm["cheb_bytes"], "launches": main_arm["cheb_launches"]}
        # what plain streams reach on this GPU: the Chebyshev step reads about
        # seven bytes for every byte it writes
        from paper_2402_12947_amd.binding import stream_probe
        ceil = {k: round(stream_probe(k), 1) for k in ("read", "copy", "mix7:1")}
        roofline["stream_ceilings"] = ceil
        roofline["frac_of_mix7_1_stream"] = round(achieved / ceil["mix7:1"], 4)
    line = {
        "metric": "DOFs solved/sec to rtol 1e-8 (MG-PCG, global-local smoother)",
        "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * main_arm["elapsed_s"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-in-f64",
        "data": "synthetic (seeded meshes and right-hand sides)",
        "config": {"workload": args.workload, "dofs": n, "levels": len(meshes), "rtol": rtol,
                   "smoother": ("S_c -> Chebyshev-Jacobi(2) -> S_c, V(2,2), adjusted lambda_max"
                                if args.smoother == "chebyshev" else
                                "S_c -> multicolour symmetric Gauss-Seidel -> S_c, V(2,2)"),
                   "problem": problem, "precision": args.precision, "patch_layers": layers,
                   "patch_policy": policy,
                   "iterations": main_arm["iterations"][0],
                   "setup_s": round(main_arm["setup_s"], 3),
                   "true_rel_residual": main_arm["true_rel_residual"],
                   "patches_level0": main_arm["levels"][0]["n_patches"],
                   "patch_colours_one_launch_level0": main_arm["levels"][0]["patch_fused_colours"],
                   "coarsest_dofs": main_arm["levels"][-1]["n_free"], "graph": bool(args.graph),
                   "sell_sigma_level0": main_arm["levels"][0]["sell_sigma"],
                   "sell_padding_level0": round(main_arm["levels"][0]["sell_stored"]
                                                / main_arm["levels"][0]["nnz"], 4),
                   "levels_n_nnz_padding_sigma_idx16_unroll_mask_rpl": [
                       [lv["n_free"], lv["nnz"], round(lv["sell_stored"] / max(1, lv["nnz"]), 4), lv["sell_sigma"],
                        round(lv["sell_nnz16"] / max(1, lv["sell_stored"]), 4), lv["sell_unroll"], lv["sell_mask"],
                        lv["sell_rpl"]]
                       for lv in main_arm["levels"]]},
        "roofline": roofline,
        "arms": extra,
    }
    if args.copy_calibration:
        # a plain streaming kernel of known traffic: dst = 2 * src over 1 GiB,
        # reads 1 GiB and writes 1 GiB (torch's elementwise multiply)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"kernel": "elementwise MulFunctor", "read": src.numel() * 8,
                                          "write": dst.numel() * 8}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(recipe, degree, layers, rtol, scale * 8, policy, problem)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
