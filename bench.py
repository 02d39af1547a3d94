"""Benchmark: PCG control solves/s on one MI355X for the 3D n=2047 configuration.

One step = one complete control solve (operator and preconditioner symbols built on the
GPU, then the low-rank PCG to its stopping rule; result left in device memory) in mixed
precision.  The same solve in FP64 is timed beside it, both are compared with the exact
control on a 31^3 sub-grid (oracle O1, restricted evaluation), and the CPU oracle is
timed on a bounded sample of its work.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "PCG control solves/s, 3D n=2047 (mixed vs FP64 tensor), rel err vs FP64 oracle"
PEAK = {"fp32_vector_tflops": 157.3, "fp64_vector_tflops": 78.6, "hbm_gbs": 8000.0}

# Solver settings per precision (documented in the design doc)
SETTINGS = {
    "mixed": dict(prec=1, eps=2e-5, tau=2e-5, cap=64, op_terms=28, pre_terms=12),
    "fp64": dict(prec=0, eps=2e-7, tau=2e-7, cap=96, op_terms=36, pre_terms=12),
}
STRIDE = 64  # sub-grid i = 64 p - 1 for the error against the exact control


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_solver(ctx, p, sk_by_q, s, steps, warmup, profile):
    import torch
    import paper_1809_01971_amd as tp
    X = tp.Tensor(3, p.n, s["cap"], s["prec"])
    q = s["cap"] + 16
    sk = sk_by_q[q]

    def one():
        op, pre, errs = ctx.symbol_build(3, p.n, p.alpha, p.c_neg, p.c_pos, prec=s["prec"],
                                         op_terms=s["op_terms"], pre_terms=s["pre_terms"])
        st, info = ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=s["tau"], kmax=100,
                                 trunc_tol=s["eps"], cap=s["cap"], sketch=sk)
        op.free()
        pre.free()
        info["sym_err"] = errs
        return info

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
    t0 = time.perf_counter()
    infos = [one() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read() if profile else None
    if profile:
        ctx.profile(False)
    return X, dt, infos, prof


def oracle_restricted(p, rows, slabs, workers):
    from concurrent.futures import ProcessPoolExecutor
    from oracle import exact
    chunks = [slabs[i::workers] for i in range(workers)]
    with ProcessPoolExecutor(workers) as ex:
        futs = [ex.submit(exact.solve_cp_restricted_slabs, p.weights, p.factors, p.alpha, p.c_neg, p.c_pos,
                          rows, c) for c in chunks if len(c)]
        return np.sum([f.result() for f in futs], axis=0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs a single control problem per GPU and has no "
              "multi-GPU path (see DESIGN.md, 'Sharding'); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors

    p = workloads.cfg3()
    ctx = tp.Context(0, workspace_bytes=24 << 30)
    qs = sorted({s["cap"] + 16 for s in SETTINGS.values()})
    sk_by_q = {q: sketch_tensors(workloads.sketch_matrices(p.n, 3, q)) for q in qs}
    rows = [workloads.restriction_rows(p.n, STRIDE)] * 3

    log("bench: mixed warmup=%d steps=%d" % (args.warmup, args.steps))
    Xm, dtm, infm, prof = run_solver(ctx, p, sk_by_q, SETTINGS["mixed"], args.steps, args.warmup, True)
    um = ctx.eval_grid(Xm, rows)
    fsteps = args.fp64_steps if args.fp64_steps is not None else max(1, args.steps // 2)
    log("bench: fp64 steps=%d" % fsteps)
    Xd, dtd, infd, _ = run_solver(ctx, p, sk_by_q, SETTINGS["fp64"], fsteps, 1, False)
    ud = ctx.eval_grid(Xd, rows)

    golden = os.path.join(ROOT, "tests", "golden", "cfg3_restricted_s64.npy")
    uo = np.load(golden) if os.path.exists(golden) else None

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    value = args.steps / dtm
    ms = 1000.0 * dtm / args.steps

    # roofline of the dominant kernel class in the timed region
    peaks = {"gemm_f64": ("alu", PEAK["fp64_vector_tflops"], "TFLOP/s"),
             "gemm_f32": ("alu", PEAK["fp32_vector_tflops"], "TFLOP/s"),
             "gemm_f32_f64": ("alu", PEAK["fp32_vector_tflops"], "TFLOP/s"),
             "gemm_f64_f32": ("alu", PEAK["fp64_vector_tflops"], "TFLOP/s"),
             "dst_f64": ("hbm", PEAK["hbm_gbs"], "GB/s"), "dst_f32": ("hbm", PEAK["hbm_gbs"], "GB/s"),
             "syev": ("alu", PEAK["fp64_vector_tflops"], "TFLOP/s")}
    dom = max(prof, key=lambda k: prof[k]["ms"])
    pd = prof[dom]
    bound, peak, unit = peaks[dom]
    if unit == "TFLOP/s":
        achieved = pd["flops"] / (pd["ms"] * 1e-3) / 1e12 if pd["ms"] > 0 else 0.0
        per_launch = pd["flops"] / max(pd["launches"], 1)
    else:
        achieved = pd["bytes"] / (pd["ms"] * 1e-3) / 1e9 if pd["ms"] > 0 else 0.0
        per_launch = pd["bytes"] / max(pd["launches"], 1)
    roofline = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                "traffic": None, "kernel": dom, "launches_per_step": pd["launches"] / args.steps,
                "avg_launch_us": 1000.0 * pd["ms"] / max(pd["launches"], 1),
                "algorithmic_per_launch": per_launch}
    breakdown = {k: {"ms_per_step": v["ms"] / args.steps, "launches_per_step": v["launches"] / args.steps}
                 for k, v in prof.items() if v["launches"] > 0}

    cpu = None
    if not args.no_cpu:
        import threadpoolctl
        workers = min(16, os.cpu_count() or 1)
        sample = list(range(0, p.n, 8))          # 1/8 of the first-index slabs
        log("bench: cpu oracle sample (%d slabs of %d, %d workers)" % (len(sample), p.n, workers))
        with threadpoolctl.threadpool_limits(1):
            t0 = time.perf_counter()
            oracle_restricted(p, rows, sample, workers)
            tc = time.perf_counter() - t0
        full_s = tc * p.n / len(sample)
        cpu = {"value": 1.0 / full_s, "unit": "solves/s", "cores": workers, "kind": "oracle",
               "sample": "exact spectral solve (restricted evaluation on the 31^3 sub-grid i=64p-1) over %d of "
                         "%d first-index slabs, %.1fs, scaled to a full solve" % (len(sample), p.n, tc)}

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cfg3: 3D n=2047, alpha=1/2, beta=1, gamma=1e-2, rank-8 rhs z/(1+k)",
                   "mixed": SETTINGS["mixed"], "fp64": SETTINGS["fp64"]},
        "fp64_solves_per_s": fsteps / dtd,
        "speedup_mixed_over_fp64": value / (fsteps / dtd),
        "rel_err_mixed_vs_fp64_tensor": rel(um, ud),
        "rel_err_mixed_vs_oracle": rel(um, uo) if uo is not None else None,
        "rel_err_fp64_vs_oracle": rel(ud, uo) if uo is not None else None,
        "iters_mixed": infm[-1]["iters"], "ranks_mixed": infm[-1]["rank"],
        "iters_fp64": infd[-1]["iters"], "ranks_fp64": infd[-1]["rank"],
        "symbol_err_mixed": infm[-1]["sym_err"][0], "precond_err": infm[-1]["sym_err"][1],
        "roofline": roofline, "kernel_breakdown": breakdown, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
