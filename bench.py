"""Benchmark: DOFs solved per second to rtol 1e-8 by global-local
MG-preconditioned CG, mixed precision against FP64, with the HBM rate of the
smoother's sparse products.

Workload (default, cube_129_p2): 3D Poisson on the unit cube, tetrahedra of a
129^3 jittered Kuhn grid with 2000 degraded cells, P2 elements (16.8M DOFs),
Dirichlet on x = 0, 1, three non-nested coarse levels (65^3, 33^3, 17^3),
combined smoother S_c -> Chebyshev-Jacobi(2) -> S_c with the adjusted
lambda_max, V(2,2) cycle, CG to rtol 1e-8.

A step is one MG-PCG solve of one synthetic right-hand side (uniform [-1, 1],
seeded, resident in HBM before the timed region) with the hierarchy already
set up; setup time is reported separately.  Every arm solves the same seeded
right-hand sides:
  mixed       global-local, FP32 V-cycle inside FP64 CG (the line's value),
              with the patches of level 1 inherited through the interpolation
              from the finest level's degraded cells (--inherit 1)
  fp64        the same in FP64 throughout
  paper       mixed with the paper's per-level patches only (--inherit 0)
  refined     (patch stress workload only) mixed with one FP64 refinement
              step of every patch solve
  plain_fp64  plain Chebyshev smoother (no S_c, unadjusted lambda_max), FP64
  ref         global-local FP64 on the high-quality reference mesh (the same
              recipe without degraded cells): the iteration count to match
value = DOFs x timed solves / wall time of the mixed arm.  Each CG iteration
of the timed solves is one replay of its captured hipGraph (--eager: host
launches), and the run starts with 10 s of untimed streaming so that the GPU's
clocks and power state settle.  The timed solves run without timing events;
a separate, untimed solve per arm then times every
full Chebyshev step per level and the coarsest solve with HIP events on the
library's stream (the roofline entry and the per-level table).  The CPU
baseline is the oracle on a bounded sample (the same recipe at 1/8 of the
size per side, single-threaded).  The default run then also times the
many-instance solve (32 cubes of 50k-3M DOFs, 4 right-hand sides each, all
solved together by mg_pcg_solve_batch) and reports it under many_instance
(--no-batch skips it; --workload cube_batch_32x4 gives it its own line).

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


def read_traffic(workload: str, precision: str, level: int = 0):
    """HBM bytes per launch of a level's Chebyshev step from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated), if it was taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"cheb_step_{workload}_{precision}_level{level}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def level_bytes(info, precision, cheb_degree=2):
    """Bytes one full Chebyshev step of a level must move.

    s8d: the scope table's unit, 12 nnz + 48 n (FP64) or 8 nnz + 24 n (FP32):
    values and 4-byte column indices once; x, b, D^-1, d read and d, x'
    written.  compressed: what the stored layout needs, 16-bit columns where a
    slice's columns fit them, and d read/written only where the recurrence
    uses it (averaged over the k steps of one polynomial)."""
    v = 4.0 if precision == "mixed" else 8.0
    nnz, n, n16 = info["nnz"], info["n_free"], info["sell_nnz16"]
    s8d = (v + 4.0) * nnz + 6.0 * v * n
    vecs = 4.0 + 2.0 * (cheb_degree - 1) / cheb_degree
    compressed = (v + 2.0) * n16 + (v + 4.0) * (nnz - n16) + v * vecs * n
    return s8d, compressed


def layout_string(levels):
    """The level operators' layout choices as 'sigma,unroll,mask,rpl' per
    level, joined by ';' (what --layout takes to repeat them)."""
    return ";".join(f"{lv['sell_sigma']},{lv['sell_unroll']},{lv['sell_mask']},{lv['sell_rpl']}"
                    for lv in levels if not lv["is_coarsest"])


def parse_layout(text):
    return [[int(v) for v in part.split(",")] for part in text.split(";")] if text else None


def run_arm(meshes, degree, layers, rtol, seeds, warmup, precision="fp64", local=True, timing=True,
            use_graph=False, sigma=0, policy="merge", smoother="chebyshev", problem="poisson", label="",
            layout=None, inherit=0, refine=False, factor_f32=True, coarse_solver=0, coarse_leaf=1024):
    """Sets up one hierarchy, solves seeds[:warmup] untimed, then times the
    solves of seeds[warmup:]; then (timing) one more solve of the first timed
    right-hand side with per-level kernel events, outside the timed region."""
    import torch

    from paper_2402_12947_amd import Solver
    log(f"[{label}] setup precision={precision} local={local}")
    t0 = time.perf_counter()
    s = Solver(meshes, degree=degree, tau=0.1, layers=layers, precision=precision,
               local_correction=local, adjusted_eig=local, use_graph=use_graph, sell_sigma=sigma, policy=policy,
               global_smoother=smoother, problem=problem, sell_layout=layout,
               patch_inherit_levels=inherit if local else 0, patch_refine=refine and local,
               patch_factor_f32=factor_f32, coarse_solver=coarse_solver, coarse_nd_leaf=coarse_leaf)
    setup_s = time.perf_counter() - t0
    n = s.n_free(0)
    log(f"[{label}] setup done in {setup_s:.2f} s, {n} DOFs; {warmup} warm-up + {len(seeds) - warmup} timed solves")
    bs = [torch.as_tensor(_rhs(n, sd)).cuda() for sd in seeds]
    us = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in seeds]
    for k in range(warmup):
        s.pcg(bs[k], us[k], rtol, 1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(warmup, len(seeds)):
        stats.append(s.pcg(bs[k], us[k], rtol, 1000))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps = len(seeds) - warmup
    log(f"[{label}] {steps} solves in {elapsed:.3f} s, iterations {[x['iterations'] for x in stats]}")
    levels = [s.level_info(l) for l in range(s.n_levels)]
    out = {"n": n, "setup_s": setup_s, "elapsed_s": elapsed, "steps": steps,
           "dofs_per_s": n * steps / elapsed, "iterations": [x["iterations"] for x in stats],
           "converged": all(x["converged"] for x in stats),
           "true_rel_residual": max(x["true_rel_residual"] for x in stats),
           "levels": levels, "layout": layout_string(levels),
           "first_seed": seeds[warmup], "first_solution": us[warmup].cpu().numpy()}
    if timing and smoother == "chebyshev":
        u = torch.zeros(n, dtype=torch.float64, device="cuda")
        s.enable_kernel_timing(True)
        s.pcg(bs[warmup], u, rtol, 1000)
        per = []
        for l, info in enumerate(levels):
            launches, total_ms = s.kernel_time(l)
            if launches == 0:
                continue
            avg_ms = total_ms / launches
            if info["is_coarsest"]:
                cb = info["coarse_solve_bytes"]
                kind = (f"coarsest solve (nested dissection, {info['coarse_nd_supernodes']} supernodes)"
                        if info["coarse_nd_supernodes"] else "coarsest solve (packed FP64 inverse)")
                per.append({"level": l, "kernel": kind, "n": info["n_free"],
                            "launches": launches, "avg_us": round(1e3 * avg_ms, 2), "bytes": cb,
                            "gbs": round(cb / (avg_ms * 1e-3) / 1e9, 1), "total_ms": round(total_ms, 3)})
                continue
            s8d, comp = level_bytes(info, precision)
            rows_per_slice = 64 // info["sell_rpl"]
            grid = -(-info["n_free"] // rows_per_slice) * 64   # threads of one launch (64 per slice)
            per.append({"level": l, "kernel": "k_cheb (full step)", "n": info["n_free"], "nnz": info["nnz"],
                        "grid": grid, "unroll_mask_rpl": [info["sell_unroll"], info["sell_mask"], info["sell_rpl"]],
                        "launches": launches, "avg_us": round(1e3 * avg_ms, 2),
                        "bytes_s8d": s8d, "gbs_s8d": round(s8d / (avg_ms * 1e-3) / 1e9, 1),
                        "frac_s8d": round(s8d / (avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                        "bytes_compressed": comp, "gbs_compressed": round(comp / (avg_ms * 1e-3) / 1e9, 1),
                        "total_ms": round(total_ms, 3)})
        s.enable_kernel_timing(False)
        out["kernel_levels"] = per
    s.close()
    return out


def _rhs(n, seed):
    import meshgen
    return meshgen.random_rhs(n, seed)


def cpu_baseline(recipe, degree, layers, rtol, scale, policy="merge", problem="poisson", budget_s=12.0, inherit=0):
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
                                             else oracle.MERGE, problem=problem, inherit_levels=inherit))
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
                      f"{len(meshes)} levels, inherited patches on {inherit} level(s)), {solved} full MG-PCG "
                      f"solves to rtol {rtol:g}, setup untimed, iterations {its[0]}",
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count(),
            "host_affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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
    graph-captured CG iterations, all instances solved together by
    mg_pcg_solve_batch (one host thread), against the same systems solved one
    by one in FP64."""
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
        "metric": "aggregate DOFs solved/sec to rtol 1e-8 (batched mixed MG-PCG, graph-captured CG iterations)",
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


METRIC = "DOFs solved/sec to rtol 1e-8 (mixed vs FP64 MG-PCG); smoother SpMV HBM GB/s"


def _arm_summary(a):
    d = {"dofs_per_s": a["dofs_per_s"], "iterations": a["iterations"], "setup_s": round(a["setup_s"], 3),
         "true_rel_residual": a["true_rel_residual"], "solves_timed": a["steps"],
         "ms_per_solve": round(1e3 * a["elapsed_s"] / a["steps"], 3), "layout": a["layout"]}
    if "kernel_levels" in a:
        d["kernel_levels"] = a["kernel_levels"]
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube_129_p2", choices=sorted(WORKLOADS) + sorted(BATCH_WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"],
                    help="precision of the arm that gives the line's value (the other global-local arm is "
                         "run as well unless --arms drops it)")
    ap.add_argument("--arms", default="mixed,fp64,paper,plain,ref",
                    help="comma list of mixed, fp64, paper (mixed with the paper's per-level patches only), "
                         "plain, ref")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="launch every kernel of the timed solves from the host (default: each CG iteration of "
                         "the global-local arms replayed from its captured hipGraph)")
    ap.add_argument("--gpu-warmup-s", type=float, default=10.0,
                    help="seconds of untimed streaming on the GPU before the first setup (clocks and power "
                         "state settle; 0 = none)")
    ap.add_argument("--sigma", type=int, default=0, help="SELL sorting window (0 = library's choice)")
    ap.add_argument("--inherit", type=int, default=-1,
                    help="coarse levels that also take the patches inherited through the interpolation from the "
                         "finest level's degraded cells (patch_inherit_levels; 0 = the paper's construction, "
                         "which then also runs as an extra mixed arm when this is above 0); default 1, and 0 on "
                         "the patch stress workload, whose inherited components would cover most of level 1")
    ap.add_argument("--refine", action="store_true", help="one FP64 refinement step of every patch solve")
    ap.add_argument("--f64-patch-factor", action="store_true",
                    help="mixed arm: factor the patch systems in FP64 (default: FP32 matrix cores)")
    ap.add_argument("--coarse-solver", type=int, default=0, choices=[0, 1, 2],
                    help="coarsest solve: 0 = library's choice, 1 = dense inverse, 2 = nested dissection")
    ap.add_argument("--coarse-leaf", type=int, default=1024, help="nested dissection: largest leaf")
    ap.add_argument("--layout", default="",
                    help="fix the level operators' layouts of the global-local arms: 'sigma,unroll,mask,rpl' per "
                         "level joined by ';' (an arm's 'layout' field of an earlier run), so that a profiled "
                         "run repeats the layouts of the timed one")
    ap.add_argument("--smoother", default="chebyshev", choices=["chebyshev", "sgs"],
                    help="global smoother S_g of every arm (the roofline entry needs chebyshev)")
    ap.add_argument("--study", action="store_true",
                    help="instead of the benchmark line: the stationary-solver / preconditioner study of "
                         "plain vs global-local smoothing on the reference mesh and Cases A and B")
    ap.add_argument("--no-batch", action="store_true",
                    help="default workload only: skip the many-instance solve (cube_batch_32x4, two batches) "
                         "reported under many_instance")
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
    if args.gpu_warmup_s > 0:
        from paper_2402_12947_amd.binding import stream_probe
        log(f"GPU warm-up: {args.gpu_warmup_s:.0f} s of streaming")
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.gpu_warmup_s:
            stream_probe("mix7:1", 2 << 30, 20)
    if args.study:
        run_study()
        return
    if args.workload in BATCH_WORKLOADS:
        print(json.dumps(run_batch(args.workload, args.steps, args.warmup)), flush=True)
        return
    recipe, degree, scale, layers, rtol, policy = WORKLOADS[args.workload][:6]
    problem = WORKLOADS[args.workload][6] if len(WORKLOADS[args.workload]) > 6 else "poisson"
    if args.inherit < 0:
        args.inherit = 0 if args.workload == "cube_129_stress_p2" else 1
    log(f"generating the {args.workload} hierarchy")
    meshes = meshgen.hierarchy(recipe, seed=0, scale=scale)
    arms = set(args.arms.split(","))
    arms.add(args.precision)
    # every arm solves the same right-hand sides: seeds[:warmup] untimed, the rest timed
    seeds = [1000 + k for k in range(args.warmup + args.steps)]
    common = dict(layers=layers, rtol=rtol, policy=policy, smoother=args.smoother, problem=problem,
                  sigma=args.sigma, inherit=args.inherit, refine=args.refine,
                  factor_f32=not args.f64_patch_factor, coarse_solver=args.coarse_solver,
                  coarse_leaf=args.coarse_leaf)
    res = {}
    for prec in ("mixed", "fp64"):
        if prec in arms:
            res[prec] = run_arm(meshes, degree, seeds=seeds, warmup=args.warmup, precision=prec, local=True,
                                use_graph=not args.eager, label=f"global-local {prec}",
                                layout=parse_layout(args.layout), **common)
    main_arm = res[args.precision]
    n = main_arm["n"]
    extra = {}
    for prec, a in res.items():
        for x in a.get("kernel_levels", []):
            if "bytes_s8d" in x:
                x["traffic_counters"] = read_traffic(args.workload, prec, x["level"])
        extra[f"global_local_{prec}"] = _arm_summary(a)
    if "mixed" in res and "fp64" in res:
        # same right-hand side, same rtol: distance of the mixed-precision
        # solution from the FP64 one (which the parity tests tie to the oracle)
        x64, xmx = res["fp64"]["first_solution"], res["mixed"]["first_solution"]
        assert res["fp64"]["first_seed"] == res["mixed"]["first_seed"]
        extra["global_local_mixed"]["rel_diff_vs_fp64_solution"] = float(
            np.linalg.norm(xmx - x64) / max(np.linalg.norm(x64), 1e-300))
        extra["mixed_speedup_vs_fp64"] = res["mixed"]["dofs_per_s"] / res["fp64"]["dofs_per_s"]
    if "paper" in arms and args.inherit > 0:
        pp = dict(common, inherit=0)
        q = run_arm(meshes, degree, seeds=seeds, warmup=args.warmup, precision="mixed", local=True, timing=False,
                    use_graph=not args.eager, label="global-local mixed, paper's patches", **pp)
        extra["global_local_mixed_paper_patches"] = _arm_summary(q)
        res_paper = q
    else:
        res_paper = None
    if args.workload == "cube_129_stress_p2" and not args.refine and "mixed" in arms:
        # the patch stress configuration names FP64 refinement of the FP32
        # patch solves: the mixed arm once more with it
        rr = run_arm(meshes, degree, seeds=seeds, warmup=args.warmup, precision="mixed", local=True, timing=False,
                     use_graph=not args.eager, label="global-local mixed, refined patch solves",
                     **dict(common, refine=True))
        extra["global_local_mixed_refined_patch_solves"] = _arm_summary(rr)
    if "plain" in arms:
        p = run_arm(meshes, degree, seeds=seeds[:args.warmup + max(1, args.steps // 2)], warmup=args.warmup,
                    precision="fp64", local=False, timing=False, label="plain fp64", **common)
        extra["plain_fp64"] = _arm_summary(p)
        extra["speedup_vs_plain_fp64"] = main_arm["dofs_per_s"] / p["dofs_per_s"]
    if "ref" in arms:
        log("generating the high-quality reference hierarchy (no degraded cells)")
        ref_meshes = meshgen.hierarchy(recipe, seed=0, scale=scale, case="ref")
        r = run_arm(ref_meshes, degree, seeds=seeds[:args.warmup + 1], warmup=args.warmup, precision="fp64",
                    local=True, timing=False, label="reference mesh fp64", **common)
        extra["reference_mesh_fp64"] = {"iterations": r["iterations"], "dofs_per_s": r["dofs_per_s"],
                                        "true_rel_residual": r["true_rel_residual"]}
        its_ref = r["iterations"][0]
        extra["iterations_within_1_of_reference"] = {
            prec: all(abs(i - its_ref) <= 1 for i in a["iterations"]) for prec, a in res.items()}
        if res_paper is not None:
            extra["iterations_within_1_of_reference"]["mixed_paper_patches"] = all(
                abs(i - its_ref) <= 1 for i in res_paper["iterations"])
    roofline = None
    if args.smoother == "chebyshev":
        lv0 = main_arm["kernel_levels"][0]
        achieved = lv0["gbs_s8d"]
        traffic = read_traffic(args.workload, args.precision)
        roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                    "kernel": f"{CHEB_KERNEL} level 0 ({'FP32' if args.precision == 'mixed' else 'FP64'})",
                    "avg_launch_ms": round(lv0["avg_us"] / 1e3, 5), "launches": lv0["launches"],
                    "algorithmic_bytes_per_launch": lv0["bytes_s8d"],
                    "bytes_model": ("8 nnz + 24 n" if args.precision == "mixed" else "12 nnz + 48 n"),
                    "compressed_index_bytes_per_launch": lv0["bytes_compressed"],
                    "compressed_index_gbs": lv0["gbs_compressed"]}
        # what plain streams reach on this GPU: the Chebyshev step reads about
        # seven bytes for every byte it writes
        from paper_2402_12947_amd.binding import stream_probe
        ceil = {k: round(stream_probe(k), 1) for k in ("read", "copy", "mix7:1")}
        roofline["stream_ceilings"] = ceil
        roofline["frac_of_mix7_1_stream"] = round(achieved / ceil["mix7:1"], 4)
    line = {
        "metric": METRIC,
        "value": main_arm["dofs_per_s"], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * main_arm["elapsed_s"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (seeded meshes and right-hand sides)",
        "config": {"workload": args.workload, "dofs": n, "levels": len(meshes), "rtol": rtol,
                   "smoother": ("S_c -> Chebyshev-Jacobi(2) -> S_c, V(2,2), adjusted lambda_max"
                                if args.smoother == "chebyshev" else
                                "S_c -> multicolour symmetric Gauss-Seidel -> S_c, V(2,2)"),
                   "problem": problem,
                   "precision": ("FP32 V-cycle (smoothers, transfers, patch solves) inside FP64 CG; "
                                 "coarsest solve FP64" if args.precision == "mixed" else "FP64"),
                   "patch_layers": layers, "patch_policy": policy,
                   "patch_inherit_levels": args.inherit, "patch_refine": bool(args.refine),
                   "patch_factor": "FP64" if args.f64_patch_factor or args.precision == "fp64" else
                                   "FP32 matrix cores (FP64 where a scaled pivot < 2^-12)",
                   "patches_f32_level0": main_arm["levels"][0]["patches_f32"],
                   "iterations": main_arm["iterations"][0],
                   "setup_s": round(main_arm["setup_s"], 3),
                   "true_rel_residual": main_arm["true_rel_residual"],
                   "patches_level0": main_arm["levels"][0]["n_patches"],
                   "coarsest_dofs": main_arm["levels"][-1]["n_free"], "graph": not args.eager,
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
        log("CPU baseline: the oracle, single-threaded, on the 1/8-size sample")
        line["cpu_baseline"] = cpu_baseline(recipe, degree, layers, rtol, scale * 8, policy, problem,
                                            inherit=args.inherit)
    if args.workload == "cube_129_p2" and not args.no_batch:
        # the many-instance pattern in the same run: 32 cubes of uneven size,
        # 4 right-hand sides each, all solved together
        log("many-instance solve (cube_batch_32x4)")
        bt = run_batch("cube_batch_32x4", 2, 1)
        line["many_instance"] = {
            "workload": "cube_batch_32x4", "metric": bt["metric"], "value": bt["value"], "unit": "DOF/s",
            "ms_per_batch": bt["ms_per_step"], "batches_timed": 2,
            "instances": bt["config"]["instances"], "rhs_per_instance": bt["config"]["rhs_per_instance"],
            "dofs_total": bt["config"]["dofs_total"], "iterations_min_max": bt["config"]["iterations_min_max"],
            "worst_true_rel_residual": bt["config"]["worst_true_rel_residual"],
            "setup_s": bt["config"]["setup_s"], "unblocked_dofs_per_s": bt["unblocked_dofs_per_s"],
            "one_by_one_fp64_dofs_per_s": bt["one_by_one_fp64"]["dofs_per_s"],
            "speedup_vs_one_by_one_fp64": bt["speedup_vs_one_by_one_fp64"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
