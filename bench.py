"""IBMI benchmark on one MI355X: sweeps of the p = 16384 squared-exponential workload.

A step is one IBMI sweep of the whole hot path: the block update of eq. (IBMI) for all 32
sets (panel GEMM W H[I^c,I^c] scattered into H, split-K diagonal product and H[I,I]
finalisation) followed by the ||I - A H||_F check with its host read-back.  The FP64 form is
the headline value; the low-precision update forms (FP32, split-bfloat16 bf16x3 and bf16x6,
all in the correction form) are timed the same way and reported beside it, each with its
speedup per sweep and the roofline of its update product.  Plan time (block
factors, once per solve) is reported separately.  Inputs are synthetic: 16384 seeded
uniform points in the unit square sorted by x, SE kernel with length scale 0.05 plus a
1e-3 nugget, FP64, resident in HBM before timing starts.

Prints ONE JSON line.  `--full-solve` additionally runs complete solves to a relative error
of 1e-10, certified by the bound from ||H (I - A H)||_F, and reports s/solve per form.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PANEL_KERNEL = "gemm_kernel<double, 96, 64, 16, 2, 2, 1, 2, true>"
# Update product of each low-precision form: (dense matrix-core peak of the instruction type
# used, matrix-core products executed per FP32-level product, instruction type, kernel).
UPDATE_KERNELS = {
    "fp32": (157.3, 1, "f32",
             "gemm_kernel<float, 96, 128, 32, 2, 2, 5, 4, true> (R[I,:] - A[I,:] D)"),
    "bf16x3": (2500.0, 3, "bf16",
               "split_gemm_kernel<192, 256, 32, 2, 4, 2, true> (R[I,:] - A[I,:] D)"),
    "bf16x6": (2500.0, 6, "bf16",
               "split_gemm_kernel<192, 128, 32, 3, 2, 3, true> (R[I,:] - A[I,:] D)"),
}


def measured_traffic(kernel: str):
    """HBM bytes per panel launch from the committed rocprofv3 PMC summary, if it was taken
    on the same kernel instantiation the bench runs; None otherwise."""
    import re
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "panel_gemm_p16384_hbm_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    k = re.search(r"^kernel:\s*(.+)$", text, re.M)
    if not m or not k or k.group(1).strip() != kernel:
        return None
    return float(m.group(1))


def cpu_baseline(A, ranges, n_sets):
    """The oracle, untouched, on a bounded sample of the same workload: the factors and the
    eq. (IBMI) updates of the first n_sets sets of the first sweep from H = I."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = len(os.sched_getaffinity(0))
    p = A.shape[0]
    H = np.eye(p)
    t0 = time.perf_counter()
    flops = 0.0
    for s, e in ranges[:n_sets]:
        bp = oracle.block_factors(A, s, e)
        oracle.block_update(H, bp)
        b, c = e - s, p - (e - s)
        flops += b ** 3 + 2.0 * b * b * c + 2.0 * b * c * c + 2.0 * b * b * c
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"plan + eq. (IBMI) update of the first {n_sets} of {len(ranges)} sets of "
                      f"sweep 1 from H = I at p={p} (FP64 NumPy/OpenBLAS), {dt:.1f} s"}


def batched_bench(ib, torch):
    """256 Wishart matrices (p log-uniform in [128, 2048]), b = 128, overlap 16, tol 1e-8,
    solved as one batch: cached/autotuned tile shapes, then a timed solve."""
    import workloads
    from paper_2502_06377_amd import tuning
    from paper_2502_06377_amd.flops import sweep_flops
    log("[batched] generating 256 matrices")
    mats = workloads.config4_batch()
    dev = []
    for a in mats:
        p = a.shape[0]
        ld = (p + 7) // 8 * 8
        t = torch.zeros((p, ld), dtype=torch.float64, device="cuda:0")
        t[:, :p] = torch.from_numpy(a)
        dev.append(t[:, :p])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = ib.BatchPlan(dev, block_rows=128, overlap=16, tol=1e-8, max_sweeps=500)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    tune = tuning.tuned(batch)
    log(f"[batched] tuning {tune}")
    batch.solve()  # warm-up (builds the graph for these buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = batch.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flops = sum(sweep_flops(a.shape[0], ib.ibmi_partition(a.shape[0], 128, 16)) * o.sweeps
                for a, o in zip(mats, outs))
    batch.close()
    return {"matrices": len(mats), "s_per_batch": round(dt, 4), "plan_s": round(plan_s, 4),
            "solves_per_s": round(len(mats) / dt, 2), "tflops": round(flops / dt / 1e12, 3),
            "sweeps_max": max(o.sweeps for o in outs),
            "sweeps_mean": round(sum(o.sweeps for o in outs) / len(outs), 2),
            "all_converged": all(o.converged for o in outs), "tile_cfg": list(tune["cfg"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--p", type=int, default=16384)
    ap.add_argument("--full-solve", action="store_true")
    ap.add_argument("--max-sweeps", type=int, default=3000)
    ap.add_argument("--full-solve-forms", default="fp64,fp32,bf16x3",
                    help="comma-separated forms for --full-solve")
    ap.add_argument("--full-solve-tols", default="1e-9,1e-10",
                    help="certified relative-error targets for --full-solve, loosest first")
    ap.add_argument("--batched", action="store_true",
                    help="also time the batched form on 256 matrices, p log-uniform in [128, 2048]")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed-forms", default="fp32,bf16x3,bf16x6",
                    help="low-precision update forms timed beside the FP64 form")
    ap.add_argument("--cpu-sets", type=int, default=24)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_2502_06377_amd as ib
    from paper_2502_06377_amd.flops import plan_flops, sweep_flops

    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 8}), flush=True)
        return

    p, block_rows, overlap, nugget = args.p, 576, 64, 1e-3
    log(f"generating workload p={p}")
    A_host = workloads.config3_matrix(p=p)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(A_host).to(dev)
    H = torch.empty((p, p), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def run_form(prec):
        log(f"[{prec}] plan")
        t0 = time.perf_counter()
        plan = ib.Plan(A, block_rows=block_rows, overlap=overlap, precision=prec,
                       stop="rel_bound", lambda_min=nugget, tol=1e-10, max_sweeps=500)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        ranges = plan.blocks
        ib.ibmi_init_h(plan.handle, H)
        log(f"[{prec}] warmup {args.warmup} sweeps (K={len(ranges)})")
        for i in range(args.warmup):
            ib.ibmi_sweep(plan.handle, H, i == 0)
        ib.ibmi_set_profiling(plan.handle, True)
        ib.ibmi_kernel_times(plan.handle)  # reset
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            hist.append(ib.ibmi_sweep(plan.handle, H, args.warmup == 0 and i == 0))
            log(f"[{prec}] sweep {args.warmup + i + 1}: ||I-AH||_F = {hist[-1]:.3e}")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = ib.ibmi_kernel_times(plan.handle)
        ib.ibmi_set_profiling(plan.handle, False)
        return plan, ranges, plan_s, dt, kt, hist

    def kernels_json(kt):
        return {c: {"ms_per_launch": round(v[0] / max(v[1], 1), 4), "launches": v[1],
                    "tflops": round(v[2] / (v[0] * 1e-3) / 1e12, 3) if v[0] > 0 else None}
                for c, v in kt.items()}

    panel_cfg_default = "IBMI_CFG_PANEL" not in os.environ
    plan, ranges, plan_s, dt, kt, hist = run_form("fp64")
    K = len(ranges)
    f_sweep = sweep_flops(p, ranges)
    f_plan = plan_flops(p, ranges)
    ms_step = dt / args.steps * 1e3
    tflops = f_sweep * args.steps / dt / 1e12
    panel_ms, panel_n, panel_fl = kt["panel"]
    achieved = panel_fl / (panel_ms * 1e-3) / 1e12 if panel_ms > 0 else 0.0
    peak = 78.6
    rate = (hist[-1] / hist[0]) ** (1.0 / max(len(hist) - 1, 1)) if len(hist) > 1 else None
    out = {
        "metric": "IBMI TFLOP/s + s/solve at p=16384 to 1e-10 (mixed vs FP64); p99 latency",
        "value": round(tflops, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "se_2d_p16384_k32_fp64", "p": p, "block_rows": block_rows,
                   "overlap": overlap, "n_sets": K, "form": "fp64", "step": "one sweep + residual"},
        "sweeps_per_s": round(1e3 / ms_step, 4),
        "plan_s": round(plan_s, 4),
        "plan_tflops": round(f_plan / plan_s / 1e12, 3),
        "kernels": kernels_json(kt),
        "roofline": {"kernel": PANEL_KERNEL + " (W H[I^c,I^c] scattered into H)",
                     "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": measured_traffic(PANEL_KERNEL) if panel_cfg_default else None,
                     "traffic_unit": "bytes per launch"},
        "residual_rate_per_sweep": round(rate, 5) if rate else None,
    }
    plan.close()
    forms = [] if args.no_mixed else [f for f in args.mixed_forms.split(",") if f]
    for form in forms:
        mplan, _, mplan_s, mdt, mkt, mhist = run_form(form)
        mms = mdt / args.steps * 1e3
        peak_m, mult, mfma_type, kname = UPDATE_KERNELS[form]
        u_ms, u_n, u_fl = mkt["panel"]
        u_ach = mult * u_fl / (u_ms * 1e-3) / 1e12 if u_ms > 0 else 0.0
        out[f"{form}_update_form"] = {
            "ms_per_step": round(mms, 3), "sweeps_per_s": round(1e3 / mms, 4),
            "ibmi_tflops_equiv": round(f_sweep / (mms * 1e-3) / 1e12, 3),
            "speedup_vs_fp64": round(ms_step / mms, 3), "plan_s": round(mplan_s, 4),
            "kernels": kernels_json(mkt),
            "max_rel_residual_gap_vs_fp64": round(max(abs(a - b) / b for a, b in zip(mhist, hist)), 6),
            "roofline": {"kernel": kname, "bound": "mfma", "mfma_dtype": mfma_type,
                         "achieved": round(u_ach, 3), "peak": peak_m, "unit": "TFLOP/s",
                         "frac": round(u_ach / peak_m, 4), "mfma_products_per_fp32_product": mult,
                         "traffic": None},
        }
        mplan.close()
    plan = None
    if args.full_solve:
        # Certified relative error (REL_HR bound) targets, loosest first; each later target
        # resumes from the H of the previous one (init "given"), so one pass records the time
        # to every target.  At this workload the FP64 floor of the bound is near 5e-10.
        out["full_solve"] = {}
        forms = [f for f in args.full_solve_forms.split(",") if f]
        tols = sorted((float(t) for t in args.full_solve_tols.split(",") if t), reverse=True)
        for prec in forms:
            stages = []
            done = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for j, tol in enumerate(tols):
                log(f"[{prec}] solve to a certified relative error of {tol:g} (H R bound)")
                fplan = ib.Plan(A, block_rows=block_rows, overlap=overlap, precision=prec,
                                stop="rel_hr", tol=tol, max_sweeps=max(args.max_sweeps - done, 1),
                                init="identity" if j == 0 else "given")

                def progress(r, res, sv, prec=prec, off=done):
                    if (r + off) % 50 == 0:
                        log(f"[{prec}] sweep {r + off}: ||I-AH||_F = {res:.3e}, bound {sv:.3e}")
                    return False

                sol = fplan.solve(H, progress=progress)
                torch.cuda.synchronize()
                fplan.close()
                done += sol.sweeps
                stages.append({"tol": tol, "s_cumulative": round(time.perf_counter() - t0, 2),
                               "sweeps_cumulative": done, "converged": sol.converged,
                               "floor_limited": sol.floor_limited, "bound": sol.stop_value,
                               "residual": sol.residual, "bound_evaluations": sol.evaluations})
                log(f"[{prec}] tol {tol:g}: {done} sweeps, {stages[-1]['s_cumulative']} s, "
                    f"converged {sol.converged}, bound {sol.stop_value:.2e}")
                if not sol.converged or done >= args.max_sweeps:
                    break
            if prec == "fp64" and len(forms) > 1:
                H64 = H.clone()
            elif prec != "fp64" and "fp64" in forms:
                diff = float(torch.linalg.norm(H - H64) / torch.linalg.norm(H64))
                out["full_solve"][f"{prec}_vs_fp64_rel_fro"] = diff
            out["full_solve"][prec] = stages
    del H, A
    torch.cuda.empty_cache()
    if args.batched:
        out["batched_form"] = batched_bench(ib, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(A_host, ranges, args.cpu_sets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
