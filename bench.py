"""Benchmark: unknowns solved per second to 1e-10 relative residual on one MI355X.

One step = the whole hot path on one synthetic problem already resident in
HBM: face transmissibilities, coarse graining and coarsest factorisation
(mscg_set_permeability), then the recursive multi-scale PCG solve
(mscg_solve).  Prints one JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload smooth1024|layered128|channel1024]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
PEAK_FP64_CU_TFLOPS = 78.6 / 256  # MI355X FP64 vector peak per CU (256 CUs)

# HBM bytes per launch on the smooth1024 FP64 workload: rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE,
# over `bench.py --kernels-only 10`; FETCH_SIZE scaled by 1.9993 (what the counter reads for a plain
# copy of known size), WRITE_SIZE by 1.0.  Taken for the kernels as they stand; a kernel change
# invalidates its figure.
PMC_TRAFFIC_SMOOTH1024 = {"small_2x2": 417049, "smooth_pre": 36879673, "smooth_post": 64656465,
                          "spmv": 33818263}

WORKLOADS = {
    # 2-D, the paper's base-case contrast (1e6) at the 1024^2 size
    "smooth1024": dict(desc="2-D 5-point FV -div(k grad p)=f, 1024x1024 (1,048,576 unknowns); log10 k ~ U[-3,3] "
                            "i.i.d. then 3x3 box-smoothed (contrast 1e6); Dirichlet p=0/1 on x, no-flow on y; "
                            "f ~ N(0,1); tol 1e-10; levels 1024,256,64,16 (dense FP64 coarsest)",
                       make="smooth", opt={}),
    "layered128": dict(desc="3-D 7-point FV, 128^3 (2,097,152 unknowns); 16 layers of log10 kx = log10 ky ~ "
                            "U[-3,3], kz = kx/100; Dirichlet on the x faces; f ~ N(0,1); tol 1e-10; "
                            "aspect-ratio-aware plan with axis weights (1, 1, 0.01): levels 128^3, 32x32x128, "
                            "8x8x128, 8x8x32, 8^3; piecewise-constant extension", make="layered",
                       opt={"semi_coarsen": 1, "axis_weight": (1.0, 1.0, 0.01), "interp": 1}),
    "layered128_uniform": dict(desc="the same 128^3 layered problem with every axis coarsened together (128^3, "
                                    "32^3, 8^3) and piecewise-constant extension", make="layered",
                               opt={"interp": 1}),
    "channel1024": dict(desc="2-D, 1024x1024, 8x8-cell blocks of log10 k ~ U[-4.5,4.5] plus 5 channels "
                             "(contrast 1e9); tol 1e-10; piecewise-constant extension", make="channel",
                        opt={"interp": 1}),
}


def make_problem(kind, seed=0):
    from paper_math_9809043_amd import synth
    if kind == "smooth":
        return synth.smoothed_lognormal_2d(seed, 1024, lo=-3.0, hi=3.0, tol=1e-10, name="smooth1024")
    if kind == "layered":
        return synth.layered_128(seed)
    if kind == "channel":
        return synth.channel_1024(seed)
    raise ValueError(kind)


def run_gpu(P, opt, steps, warmup, time_small=False):
    import torch
    from paper_math_9809043_amd import mscg
    dev = torch.device("cuda:0")
    grid = mscg.Grid(dim=P.dim, n=P.n, bc_type=P.bc_type, bc_value=P.bc_value, length=P.length)
    prob = mscg.Problem(grid, mscg.Options(**opt), device=dev)
    kx = torch.tensor(P.kx, device=dev)
    ky = torch.tensor(P.ky, device=dev)
    kz = torch.tensor(P.kz, device=dev) if P.dim == 3 else None
    f = torch.tensor(P.f, device=dev)
    p = torch.zeros(P.N, dtype=torch.float64, device=dev)

    def step():
        prob.set_permeability(kx, ky, kz)
        return prob.solve(f, p, P.tol)

    for _ in range(warmup):
        st = step()
    torch.cuda.synchronize()
    if time_small:
        prob.enable_kernel_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    stats = []
    for _ in range(steps):
        stats.append(step())
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall_ms = (t1 - t0) * 1e3 / steps
    solve_ms = sum(s.solve_ms for s in stats) / steps
    st = stats[-1]
    if time_small:
        prob.small_timing = prob.small_level_timing()
        prob.enable_kernel_timing(False)
    return prob, st, wall_ms, solve_ms, p


def run_kernels_only(reps):
    """The finest-level grid-wide kernels of the 1024^2 workload after one real solve, each
    launched `reps` times back to back, and two plain copies of known size (64 MiB and
    1 GiB of FP64) that calibrate the profiler's memory counters."""
    import torch
    from paper_math_9809043_amd import mscg
    P = make_problem("smooth")
    prob, st, _, _, _ = run_gpu(P, {}, 1, 0)
    out = {}
    for kid, name in ((mscg.KERNEL_SMOOTH_PRE, "smooth_pre"), (mscg.KERNEL_SMOOTH_POST, "smooth_post"),
                      (mscg.KERNEL_SPMV, "spmv")):
        us, nbytes = prob.time_kernel(kid, 0, reps=reps)
        out[name] = {"avg_us": round(us, 3), "alg_bytes_per_launch": int(nbytes)}
    for mib in (64, 1024):
        n = mib * (1 << 20) // 8
        a = torch.rand(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(reps):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        out[f"copy_{mib}MiB"] = {"bytes_read": n * 8, "bytes_written": n * 8}
    print(json.dumps({"kernels_only": out, "outer_iters": st.outer_iters}), flush=True)


def run_scaling(sides, mgcg=True):
    """Time against N (the paper's scaling study, Section 4): the config-1 generator (log10 k ~
    U[-1,1], 3x3 box mean) on n x n grids, tol 1e-10, set-up + solve per step, FP64 and mixed,
    plus Tatebe's preconditioner in FP64 for comparison."""
    import math
    from paper_math_9809043_amd import mscg, synth
    rows = []
    for n in sides:
        P = synth.smoothed_lognormal_2d(0, n, lo=-1.0, hi=1.0, tol=1e-10, name=f"c1_{n}")
        steps, warm = (3, 1) if n <= 2048 else (2, 1)
        row = {"side": n, "unknowns": P.N}
        variants = [("fp64", {}), ("mixed", {"precision": mscg.MIXED})]
        if mgcg:
            variants.append(("mgcg_fp64", {"cycle": mscg.CYCLE_MGCG}))
        for label, opt in variants:
            _, st, wall, solve, _ = run_gpu(P, opt, steps, warm)
            row[label] = {"ms_per_step": round(wall, 3), "solve_ms": round(solve, 3),
                          "unknowns_per_s": round(P.N / (wall * 1e-3), 1), "ns_per_unknown": round(wall * 1e6 / P.N, 3),
                          "outer_iters": st.outer_iters, "level_iters": st.level_iters, "status": st.status,
                          "rel_residual_true": st.rel_residual_true}
        print(f"[bench] scaling {n}^2: fp64 {row['fp64']['ms_per_step']:.2f} ms (outer {row['fp64']['outer_iters']}), "
              f"mixed {row['mixed']['ms_per_step']:.2f} ms"
              + (f", MGCG {row['mgcg_fp64']['ms_per_step']:.2f} ms (outer {row['mgcg_fp64']['outer_iters']})"
                 if mgcg else ""), flush=True)
        rows.append(row)
    # slope of log(time) against log(N) over the grids of 2^18 unknowns and more, where the
    # per-launch latency of the coarse levels no longer sets the time
    big = [r for r in rows if r["unknowns"] >= 1 << 18]
    fit = {}
    if len(big) >= 2:
        for label in [k for k in rows[0] if k not in ("side", "unknowns")]:
            xs = [math.log(r["unknowns"]) for r in big]
            ys = [math.log(r[label]["ms_per_step"]) for r in big]
            mx, my = sum(xs) / len(xs), sum(ys) / len(ys)
            fit[label] = round(sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sum((x - mx) ** 2 for x in xs), 3)
    return {"workload": "2-D 5-point FV, n x n, log10 k ~ U[-1,1] i.i.d. then 3x3 box-smoothed, Dirichlet p=0/1 on x, "
                        "f ~ N(0,1), tol 1e-10, seed 0; set-up + solve per step",
            "rows": rows, "time_exponent_vs_N_from_2^18": fit}


def run_serving(count):
    """Serving stream: sides U{64,128,256,512}, contrast 1e6, tol 1e-8, mixed precision.
    Saturation throughput from a burst, then Poisson arrivals at 0.7x that rate."""
    from paper_math_9809043_amd import mscg, serve, synth
    opts = mscg.Options(precision=mscg.MIXED)
    srv = serve.Server(slots=8, budget_bytes=16 << 30, options=opts, tol=1e-8)
    warm = [synth.Request(i, 0.0, side, 10 + i) for i, side in enumerate((64, 128, 256, 512) * 8)]
    srv.run(warm)  # creates every slot's resident hierarchies
    burst = synth.request_stream(min(512, count), rate_per_s=1e9, arrival_seed=11, first_seed=50000)
    sat = srv.run(burst).summary()["solves_per_s"]
    rate = 0.7 * sat
    reqs = synth.request_stream(count, rate_per_s=rate, arrival_seed=7, first_seed=1000)
    print(f"[bench] serving: saturation {sat:.1f} solves/s, replaying {count} requests at {rate:.1f}/s", flush=True)
    rep = srv.run(reqs)
    s = rep.summary()
    s.update({"arrival_rate_per_s": round(rate, 2), "saturation_solves_per_s": sat, "slots": srv.nslots,
              "budget_bytes": srv.budget, "precision": "mixed", "tol": 1e-8,
              "workload": f"{count} 2-D requests, side ~ U{{64,128,256,512}}, smoothed log-normal contrast 1e6, "
                          "Poisson arrivals"})
    print(f"[bench] serving: {s['solves_per_s']} solves/s p50 {s['p50_ms']} ms p99 {s['p99_ms']} ms "
          f"ok {s['ok']}/{s['requests']}", flush=True)
    return s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="smooth1024", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-scaling", action="store_true")
    ap.add_argument("--cycle", default="recursive", choices=["recursive", "mgcg", "poly"],
                    help="preconditioner of the main workload: the paper's recursive method (default), "
                         "Tatebe's multigrid preconditioner (eq. 2.9) or the polynomial one")
    ap.add_argument("--kernels-only", type=int, default=0, metavar="REPS",
                    help="only launch the finest-level kernels and two calibration copies REPS times each "
                         "(for memory-counter profiles); prints their timings")
    ap.add_argument("--scaling-sides", default="32,64,128,256,512,1024,2048,4096")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (one process, one MI355X).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_math_9809043_amd import mscg

    if args.kernels_only > 0:
        run_kernels_only(args.kernels_only)
        return

    W = dict(WORKLOADS[args.workload])
    cycle = {"recursive": mscg.CYCLE_RECURSIVE, "mgcg": mscg.CYCLE_MGCG, "poly": mscg.CYCLE_POLY}[args.cycle]
    if cycle != mscg.CYCLE_RECURSIVE:
        W["opt"] = dict(W["opt"], cycle=cycle, max_outer_iters=5000)
        W["desc"] = W["desc"] + {mscg.CYCLE_MGCG: "; Tatebe's multigrid preconditioner (eq. 2.9)",
                                 mscg.CYCLE_POLY: "; polynomial preconditioner (Section 2.1)"}[cycle]
    P = make_problem(W["make"])
    print(f"[bench] workload {args.workload}: {P.N} unknowns, steps {args.steps}, warmup {args.warmup}", flush=True)
    # the one-workgroup last-level solver (the dominant kernel) runs in the recursive method only
    two_d_deep = P.dim == 2 and W["make"] != "layered" and cycle == mscg.CYCLE_RECURSIVE
    prob, st, wall_ms, solve_ms, p = run_gpu(P, W["opt"], args.steps, args.warmup)
    print(f"[bench] fp64: {wall_ms:.2f} ms/step (solve {solve_ms:.2f} ms) outer {st.outer_iters} "
          f"levels {st.level_iters} res {st.rel_residual_true:.2e} status {st.status}", flush=True)
    if two_d_deep:
        # the same timed steps again with HIP events around the dominant kernel's
        # launches (the event records add host time, so `value` comes from the pass above)
        prob_t, _, wall_t, _, _ = run_gpu(P, W["opt"], args.steps, args.warmup, time_small=True)
        prob.small_timing = prob_t.small_timing
        print(f"[bench] fp64 with launch events: {wall_t:.2f} ms/step", flush=True)

    # Dominant kernel by time: the one-workgroup solver of the last inner level
    # (64^2 PCG with the 16^2 coarsest solve), timed with HIP events around each
    # of its launches inside the timed steps.  It runs on one CU by design, so
    # its roofline is one CU's FP64 vector peak.
    roofline = None
    if two_d_deep:
        t = prob.small_timing
        avg_us = t["total_ms"] * 1e3 / max(t["launches"], 1)
        achieved = t["flops"] / (t["total_ms"] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": "k_small_2x2<double>: inner PCG of the last inner level "
                    "with its dense coarsest solve, one workgroup", "achieved": round(achieved, 5),
                    "peak": round(PEAK_FP64_CU_TFLOPS, 5), "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_CU_TFLOPS, 4),
                    "traffic": PMC_TRAFFIC_SMOOTH1024["small_2x2"] if args.workload == "smooth1024" else None,
                    "avg_us": round(avg_us, 3), "launches": t["launches"],
                    "iterations": t["iterations"], "alg_flops_per_launch": round(t["flops"] / max(t["launches"], 1), 1),
                    "share_of_step": round(t["total_ms"] / (wall_ms * args.steps), 4),
                    "peak_basis": "FP64 vector peak of one CU: 78.6 TFLOP/s / 256 CUs (a one-workgroup kernel "
                                  "occupies one CU)"}
    if roofline:
        print(f"[bench] dominant kernel k_small_2x2: {roofline['avg_us']:.1f} us/launch over {roofline['launches']} "
              f"launches, {roofline['achieved'] * 1e3:.1f} GFLOP/s = {roofline['frac']:.3f} of one CU's FP64 peak, "
              f"{roofline['share_of_step']:.2f} of the step", flush=True)
    # grid-wide kernels against HBM: the finest-level smoothers and SpMV
    hbm = []
    kernels = [(mscg.KERNEL_SPMV, "k_spmv_dot<double> (finest level)", "spmv")]
    if P.dim == 2:
        kernels = [(mscg.KERNEL_SMOOTH_PRE, "k_smooth_tile<double, pre> (finest level, 9 half sweeps)", "smooth_pre"),
                   (mscg.KERNEL_SMOOTH_POST, "k_prolong_2d<double> + k_smooth_tile<double, post> (finest level, "
                                             "prolongation, then 9 half sweeps)", "smooth_post")] + kernels
    for kid, name, key in kernels:
        us, nbytes = prob.time_kernel(kid, 0, reps=50)
        gbs = nbytes / (us * 1e-6) / 1e9
        hbm.append({"kernel": name, "avg_us": round(us, 3), "alg_bytes_per_launch": int(nbytes),
                    "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                    "traffic": PMC_TRAFFIC_SMOOTH1024[key] if args.workload == "smooth1024" else None})
    # whole solve against HBM: algorithmic bytes per level iteration and unknown
    # (fused smoothers, SpMV and CG vectors, FP64) times the executed iterations
    per_unk = 193.0 if P.dim == 2 else 216.0
    # level visits: CG iterations per level for the recursive method; with Tatebe's
    # preconditioner every coarser level is passed once per outer iteration
    visits = st.level_iters if cycle == mscg.CYCLE_RECURSIVE else [st.level_iters[0]] + list(st.level_calls[1:])
    unk_iters = sum(it * n for it, n in zip(visits, [x * y * z for x, y, z in st.level_n[:st.n_levels]]))
    solve_bytes = per_unk * unk_iters
    solve_gbs = solve_bytes / (solve_ms * 1e-3) / 1e9
    solve_roof = {"alg_bytes": solve_bytes, "achieved": round(solve_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                  "frac": round(solve_gbs / PEAK_HBM_GBS, 4), "bytes_per_unknown_iteration": per_unk}

    mixed = None
    if not args.no_mixed:
        opt = dict(W["opt"])
        opt["precision"] = mscg.MIXED
        _, mst, mwall, msolve, _ = run_gpu(P, opt, args.steps, args.warmup)
        mixed = {"value": round(P.N / (mwall * 1e-3), 1), "ms_per_step": round(mwall, 3),
                 "solve_ms": round(msolve, 3), "outer_iters": mst.outer_iters, "level_iters": mst.level_iters,
                 "rel_residual_true": mst.rel_residual_true, "status": mst.status,
                 "speedup_vs_fp64": round(wall_ms / mwall, 3)}
        print(f"[bench] mixed: {mwall:.2f} ms/step outer {mst.outer_iters} res {mst.rel_residual_true:.2e}",
              flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.solve(P, cycle=cycle, max_outer=5000,
                           **({"interp": W["opt"]["interp"]} if "interp" in W["opt"] else {}))
        t1 = time.perf_counter()
        cpu = {"value": round(P.N / (t1 - t0), 1), "unit": "unknowns/s", "cores": 1, "kind": "oracle",
               "sample": f"one full set-up + solve of the same {args.workload} problem by the serial FP64 C "
                         f"oracle ({t1 - t0:.1f} s, {ref.outer_iters} outer iterations)"}
        import numpy as np
        x = p.cpu().numpy()
        cpu["gpu_rel_err_vs_oracle"] = float(np.linalg.norm(x - ref.p) / np.linalg.norm(ref.p))
        print(f"[bench] oracle: {t1 - t0:.2f} s", flush=True)

    serving = None
    if not args.no_serve:
        serving = run_serving(args.serve_requests)

    extra = {}
    if not args.no_3d and not args.workload.startswith("layered128"):
        P3 = make_problem("layered")
        for key in ("layered128", "layered128_uniform"):
            W3 = WORKLOADS[key]
            _, st3, wall3, solve3, _ = run_gpu(P3, W3["opt"], 2, 1)
            opt3 = dict(W3["opt"])
            opt3["precision"] = mscg.MIXED
            _, st3m, wall3m, solve3m, _ = run_gpu(P3, opt3, 2, 1)
            extra[key] = {"workload": W3["desc"], "fp64": {"value": round(P3.N / (wall3 * 1e-3), 1),
                          "ms_per_step": round(wall3, 3), "outer_iters": st3.outer_iters,
                          "level_iters": st3.level_iters, "rel_residual_true": st3.rel_residual_true},
                          "mixed": {"value": round(P3.N / (wall3m * 1e-3), 1), "ms_per_step": round(wall3m, 3),
                                    "outer_iters": st3m.outer_iters, "level_iters": st3m.level_iters,
                                    "rel_residual_true": st3m.rel_residual_true}}
            print(f"[bench] {key}: fp64 {wall3:.1f} ms (outer {st3.outer_iters}, levels {st3.level_iters}), "
                  f"mixed {wall3m:.1f} ms (outer {st3m.outer_iters})", flush=True)

    if not args.no_3d and args.workload == "smooth1024":
        # ablation: the modified Jacobi splitting (P = 2D) on the same problem
        optj = dict(W["opt"])
        optj["splitting"] = mscg.SPLIT_JACOBI
        _, stj, wallj, solvej, _ = run_gpu(P, optj, 2, 1)
        extra["smooth1024_jacobi"] = {"workload": W["desc"] + "; modified Jacobi splitting P = 2D on every level "
                                      "(host-driven inner levels)", "fp64": {"value": round(P.N / (wallj * 1e-3), 1),
                                      "ms_per_step": round(wallj, 3), "outer_iters": stj.outer_iters,
                                      "level_iters": stj.level_iters, "rel_residual_true": stj.rel_residual_true}}
        print(f"[bench] smooth1024 modified Jacobi: fp64 {wallj:.1f} ms (outer {stj.outer_iters}, levels "
              f"{stj.level_iters})", flush=True)

    if not args.no_3d and args.workload == "smooth1024":
        # comparison: Tatebe's multigrid preconditioner (eq. 2.9, one pass down and up
        # the same hierarchy per outer iteration, no inner PCG) on the same problem
        res = {}
        for label, prec in (("fp64", mscg.FP64), ("mixed", mscg.MIXED)):
            optg = dict(W["opt"])
            optg.update(cycle=mscg.CYCLE_MGCG, precision=prec)
            _, stg, wallg, solveg, _ = run_gpu(P, optg, 5, 1)
            res[label] = {"value": round(P.N / (wallg * 1e-3), 1), "ms_per_step": round(wallg, 3),
                          "solve_ms": round(solveg, 3), "outer_iters": stg.outer_iters,
                          "level_calls": stg.level_calls, "rel_residual_true": stg.rel_residual_true}
            print(f"[bench] smooth1024 MGCG {label}: {wallg:.2f} ms/step (outer {stg.outer_iters}) res "
                  f"{stg.rel_residual_true:.2e}", flush=True)
        extra["smooth1024_mgcg"] = dict({"workload": W["desc"] + "; Tatebe's multigrid preconditioner (eq. 2.9) "
                                         "in place of the inner PCGs"}, **res)

    if not args.no_3d and args.workload == "smooth1024":
        # a grid the integer factor cannot divide: 1001^2 coarsened by 3.98 per level, the level
        # sizes of the paper's Table 1 (1001, 252, 63, 16, 4), with fractional overlaps
        from paper_math_9809043_amd import synth
        Pf = synth.smoothed_lognormal_2d(0, 1001, lo=-3.0, hi=3.0, tol=1e-10, name="smooth1001")
        res = {}
        for label, prec in (("fp64", mscg.FP64), ("mixed", mscg.MIXED)):
            _, stf, wallf, solvef, _ = run_gpu(Pf, {"frac_scale": 3.98, "min_coarse_side": 4, "precision": prec}, 3, 1)
            res[label] = {"value": round(Pf.N / (wallf * 1e-3), 1), "ms_per_step": round(wallf, 3),
                          "outer_iters": stf.outer_iters, "level_n": [list(d) for d in stf.level_n],
                          "level_iters": stf.level_iters, "rel_residual_true": stf.rel_residual_true}
            print(f"[bench] smooth1001 factor 3.98 {label}: {wallf:.2f} ms/step (outer {stf.outer_iters}, levels "
                  f"{stf.level_iters})", flush=True)
        extra["smooth1001_frac3.98"] = dict({"workload": "2-D, 1001x1001, log10 k ~ U[-3,3] then 3x3 box mean, tol "
                                             "1e-10; non-integer factor 3.98 (levels 1001, 252, 63, 16, 4)"}, **res)
        # the paper's scale-factor study (Section 4): the same problem coarsened by other factors
        sweep = []
        for fs in (2.5, 3.0, 3.5, 3.98, 5.0):
            _, sts, walls, _, _ = run_gpu(Pf, {"frac_scale": fs, "min_coarse_side": 4}, 2, 1)
            sweep.append({"factor": fs, "ms_per_step": round(walls, 3), "ns_per_unknown": round(walls * 1e6 / Pf.N, 2),
                          "outer_iters": sts.outer_iters, "level_n": [d[0] for d in sts.level_n],
                          "level_iters": sts.level_iters, "status": sts.status})
            print(f"[bench] smooth1001 factor {fs}: {walls:.2f} ms/step, levels {[d[0] for d in sts.level_n]}, "
                  f"iterations {sts.level_iters}", flush=True)
        extra["smooth1001_scale_factor_sweep"] = {"workload": "the same 1001^2 problem, FP64, factor per level",
                                                  "rows": sweep}

    scaling = None
    if not args.no_scaling:
        scaling = run_scaling([int(v) for v in args.scaling_sides.split(",") if v])

    value = P.N / (wall_ms * 1e-3)
    line = {
        "metric": "unknowns solved/s to 1e-10 resid (set-up + solve), FP64 plain method; mixed alongside"
                  + ("" if cycle == mscg.CYCLE_RECURSIVE else f" ({args.cycle} preconditioner, not the paper's method)"),
        "value": round(value, 1), "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": W["desc"], "unknowns": P.N, "outer_iters": st.outer_iters,
                   "level_iters": st.level_iters, "rel_residual_true": st.rel_residual_true,
                   "solve_only_ms": round(solve_ms, 3)},
        "mixed": mixed,
        "roofline": roofline,
        "hbm_kernels": hbm,
        "solve_hbm_roofline": solve_roof,
        "cpu_baseline": cpu,
        "serving": serving,
        "extra_workloads": extra,
        "time_vs_N": scaling,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
