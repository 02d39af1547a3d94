"""Benchmark: PCG control solves/s on one MI355X for the 3D n=2047 configuration.

One step = one complete control solve (operator and preconditioner symbols built on the GPU, then
the low-rank PCG to its stopping rule; result left in device memory) in mixed precision.  Beside it:
the same solve in FP64, both with the paper's sinc-quadrature operator symbol, the spectral-domain
variant, the mixed solve with split-BF16 products in its FP32 contractions, concurrent independent
solves, and the per-solve time over grid sizes n = 1023..32767.  The
results are compared with the exact control by Parseval's identity over sampled first-index spectral
slabs of the 2047^3 grid (oracle O1), and that oracle is timed on the host cores as the CPU baseline.
The timed steps run without per-launch events; a second pass of the same steps records HIP events
around every launch, one class per kernel, for the per-kernel roofline fractions.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--fp64-steps F] [--no-sweep]
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "PCG control solves/s, 3D n=2047 (mixed vs FP64 tensor), rel err vs FP64 oracle"
PEAK = {"fp32_tflops": 157.3, "fp64_tflops": 78.6, "hbm_gbs": 8000.0}

# Solver settings per precision: one PCG iteration on every right-hand side of the workload's shape
# tried (mixed: cap 56, sketch 64; FP64 near its 1e-6 target).  The sinc legs use the paper's rule
# for the operator symbol: M = 50 (k = -50..50) in mixed precision, k = -120..35 in FP64.
SETTINGS = {
    "mixed": dict(prec=1, eps=3e-5, tau=1.2e-4, cap=56, q=64, op_terms=28, pre_terms=28),
    "fp64": dict(prec=0, eps=1.5e-7, tau=6e-7, cap=96, q=112, op_terms=36, pre_terms=36),
    "sinc_mixed": dict(prec=1, eps=3e-5, tau=1.2e-4, cap=56, q=64, pre_terms=28, sinc=(50, 50)),
    "sinc_fp64": dict(prec=0, eps=1.5e-7, tau=6e-7, cap=96, q=112, pre_terms=36, sinc=(120, 35)),
}
ERR_SLAB_STRIDE = 4   # exact error over every 4th first-index spectral slab (unbiased sample)
# HBM bytes per launch of the kernel classes, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs each scaled
# by the reading of a 256 MiB device copy; valid only for the sources and mixed settings they were
# taken with, identified by traffic_key() (SHA-256 prefix of csrc/kernels.hip, csrc/api.hip and the
# settings' JSON); null otherwise.
TRAFFIC = {"src": "82c1495f1da07055",
           "bytes_per_launch": {"gemm_f32": 27932824, "gemm_f32_split64": 35192331, "gemm_f64": 3408414,
                                "gemm_f32_f64": 3839517, "gemm_f64_f32": 3269687, "gemm_reduce": 6569913,
                                "psd_tri": 378717, "psd_eig": 444146, "chol": 436723, "ns_isqrt": 189394,
                                "dst_f32": 3054783}}

# kernel classes of tp_profile_read: the kernel, its bound and the peak it is priced against (the
# contractions run on the FP32 / FP64 matrix cores, whose dense peaks on MI355X equal the vector
# peaks; the eigensolvers and Cholesky are FP64 ALU work)
CLASSES = {
    "gemm_f64": ("k_gemm_mfma<double, double, double, double>", "mfma", PEAK["fp64_tflops"], "TFLOP/s"),
    "gemm_f32": ("k_gemm_mfma<float, float, float, float>", "mfma", PEAK["fp32_tflops"], "TFLOP/s"),
    "gemm_f32_f64": ("k_gemm_mfma<float, float, double, double>", "mfma", PEAK["fp64_tflops"], "TFLOP/s"),
    "gemm_f64_f32": ("k_gemm_mfma<double, double, float, double>", "mfma", PEAK["fp64_tflops"], "TFLOP/s"),
    "gemm_f32_split64": ("k_gemm_mfma<float, float, double, float>", "mfma", PEAK["fp32_tflops"], "TFLOP/s"),
    "gemm_reduce": ("k_gemm_reduce", "hbm", PEAK["hbm_gbs"], "GB/s"),
    "dst_f64": ("k_dst1<double, double, ...>", "hbm", PEAK["hbm_gbs"], "GB/s"),
    "dst_f32": ("k_dst1<float, double, ...>", "hbm", PEAK["hbm_gbs"], "GB/s"),
    "syev": ("k_syev", "alu", PEAK["fp64_tflops"], "TFLOP/s"),
    "chol": ("k_pchol", "alu", PEAK["fp64_tflops"], "TFLOP/s"),
    "psd_eig": ("k_psd_eig", "alu", PEAK["fp64_tflops"], "TFLOP/s"),
    "psd_tri": ("k_psd_tri", "alu", PEAK["fp64_tflops"], "TFLOP/s"),
    "ns_isqrt": ("k_ns_isqrt", "alu", PEAK["fp64_tflops"], "TFLOP/s"),
}


def traffic_key():
    import hashlib
    data = b""
    for f in ("kernels.hip", "api.hip"):
        with open(os.path.join(ROOT, "paper_1809_01971_amd", "csrc", f), "rb") as fh:
            data += fh.read()
    data += json.dumps(SETTINGS["mixed"], sort_keys=True).encode()
    return hashlib.sha256(data).hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_solver(ctx, p, sk_by_q, s, steps, warmup, profile, spectral=False):
    import torch
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import TP_SYM_SINC
    X = tp.Tensor(3, p.n, s["cap"], s["prec"])
    sk = sk_by_q[(p.n, s["q"])]
    rhs = tp.Rhs(p.weights, p.factors)  # the input is in HBM before the timed steps
    if "sinc" in s:
        kw = dict(method=TP_SYM_SINC, sinc_kl=s["sinc"][0], sinc_kr=s["sinc"][1])
    else:
        kw = dict(op_terms=s["op_terms"])

    def one():
        op, pre, errs = ctx.symbol_build(3, p.n, p.alpha, p.c_neg, p.c_pos, prec=s["prec"],
                                         pre_terms=s["pre_terms"], **kw)
        st, info = ctx.pcg_solve(op, pre, rhs, None, X, tau=s["tau"], kmax=100,
                                 trunc_tol=s["eps"], cap=s["cap"], sketch=sk, spectral_domain=spectral)
        info["sym_err"] = errs
        info["sym_rank"] = op.info()[0]
        op.free()
        pre.free()
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


def kernel_classes(prof, steps):
    """Per kernel class: time and launches per step, algorithmic work per launch, achieved rate and
    its fraction of the class's peak (HIP-event time of the profiled pass)."""
    out = {}
    for k, v in prof.items():
        if v["launches"] <= 0:
            continue
        kern, bound, peak, unit = CLASSES[k]
        sec = v["ms"] * 1e-3
        if unit == "TFLOP/s":
            ach = v["flops"] / sec / 1e12 if sec > 0 else 0.0
            per_launch = v["flops"] / v["launches"]
        else:
            ach = v["bytes"] / sec / 1e9 if sec > 0 else 0.0
            per_launch = v["bytes"] / v["launches"]
        out[k] = {"kernel": kern, "bound": bound, "ms_per_step": v["ms"] / steps,
                  "launches_per_step": v["launches"] / steps,
                  "avg_launch_us": 1000.0 * v["ms"] / v["launches"], "algorithmic_per_launch": per_launch,
                  "algorithmic_bytes_per_launch": v["bytes"] / v["launches"],
                  "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak}
    return out


def _err_part(args):
    from threadpoolctl import threadpool_limits
    from oracle import exact
    p, tensors, slabs = args
    out = []
    with threadpool_limits(limits=1):
        for core, fs in tensors:
            out.append(exact.tucker_error_slabs(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos, core, fs, slabs))
    return out


def oracle_errors(p, tensors, slabs, workers):
    """Exact spectral errors of the GPU results over the given slabs (oracle O1 by Parseval)."""
    from concurrent.futures import ProcessPoolExecutor
    chunks = [slabs[i::workers] for i in range(workers)]
    with ProcessPoolExecutor(workers) as ex:
        parts = list(ex.map(_err_part, [(p, tensors, c) for c in chunks if len(c)]))
    res = []
    for t in range(len(tensors)):
        e2 = sum(pt[t][0] for pt in parts)
        u2 = sum(pt[t][1] for pt in parts)
        res.append(float(np.sqrt(e2 / u2)))
    return res


def host_info():
    """Host cores usable by this process, the CPU model and the numerical library versions."""
    import scipy
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model, "numpy": np.__version__,
            "scipy": scipy.__version__, "python": platform.python_version()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--sinc-steps", type=int, default=None,
                    help="timed steps of each sinc-symbol leg (default: --steps // 2; 0 skips them)")
    ap.add_argument("--batch-steps", type=int, default=8,
                    help="timed calls of the concurrent leg: 16 independent problems of the workload's "
                         "shape on 8 streams per call (0 skips it)")
    ap.add_argument("--spectral-steps", type=int, default=None,
                    help="timed steps of the spectral-domain variant (default: --steps; 0 skips it)")
    ap.add_argument("--split-steps", type=int, default=None,
                    help="timed steps of the split-BF16 variant of the mixed solve (default: --steps; 0 skips it)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the grid-size sweep n = 1023..32767")
    ap.add_argument("--cpu-workers", type=int, default=None,
                    help="host processes of the oracle (default: the usable CPUs, at most 16)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 256 MiB on the device (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs each control problem on one GPU and has no "
              "multi-GPU path (independent problems shard across GPUs without communication); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors

    p = workloads.cfg3()
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = tp.Context(0, workspace_bytes=24 << 30)
    qs = sorted({s["q"] for s in SETTINGS.values()})
    sk_by_q = {(p.n, q): sketch_tensors(workloads.sketch_matrices(p.n, 3, q)) for q in qs}

    log("bench: mixed warmup=%d steps=%d" % (args.warmup, args.steps))
    Xm, dtm, infm, _ = run_solver(ctx, p, sk_by_q, SETTINGS["mixed"], args.steps, args.warmup, False)
    log("bench: mixed profiled pass steps=%d" % args.steps)
    _, dtp, _, prof = run_solver(ctx, p, sk_by_q, SETTINGS["mixed"], args.steps, 0, True)
    fsteps = args.fp64_steps if args.fp64_steps is not None else max(1, args.steps // 2)
    prof_d, dtdp = None, None
    if fsteps > 0:
        log("bench: fp64 steps=%d (+ profiled pass)" % fsteps)
        Xd, dtd, infd, _ = run_solver(ctx, p, sk_by_q, SETTINGS["fp64"], fsteps, 1, False)
        _, dtdp, _, prof_d = run_solver(ctx, p, sk_by_q, SETTINGS["fp64"], fsteps, 0, True)
        parts_d = Xd.numpy_parts()
    else:
        dtd, infd, parts_d = None, [{"iters": None, "rank": None}], None
    parts_m = Xm.numpy_parts()

    sinc = {}
    sc_steps = args.sinc_steps if args.sinc_steps is not None else max(1, args.steps // 2)
    sinc_parts = {}
    if sc_steps > 0:
        for leg in ("sinc_mixed", "sinc_fp64"):
            n_steps = sc_steps if leg == "sinc_mixed" else max(1, sc_steps // 2)
            log("bench: %s steps=%d" % (leg, n_steps))
            Xs, dts, infs, _ = run_solver(ctx, p, sk_by_q, SETTINGS[leg], n_steps, 1, False)
            sinc_parts[leg] = Xs.numpy_parts()
            kl, kr = SETTINGS[leg]["sinc"]
            sinc[leg] = {"solves_per_s": n_steps / dts, "ms_per_step": 1000.0 * dts / n_steps,
                         "sinc_nodes": kl + kr + 1, "k_range": [-kl, kr], "symbol_rank": infs[-1]["sym_rank"],
                         "symbol_err": infs[-1]["sym_err"][0], "iters": infs[-1]["iters"],
                         "ranks": infs[-1]["rank"], "status": infs[-1]["status"]}

    ssteps = args.spectral_steps if args.spectral_steps is not None else args.steps
    spectral = None
    if ssteps > 0:
        # the same mixed solve with the iteration kept in sine coordinates (transforms only on B in
        # and X out); compared with the stated path's result on a stride-16 sub-grid
        log("bench: mixed spectral-domain steps=%d" % ssteps)
        Xs, dts, infs, _ = run_solver(ctx, p, sk_by_q, SETTINGS["mixed"], ssteps, 1, False, spectral=True)
        rows = [np.arange(0, p.n, 16)] * 3
        a, b = ctx.eval_grid(Xs, rows), ctx.eval_grid(Xm, rows)
        spectral = {"solves_per_s": ssteps / dts, "ms_per_step": 1000.0 * dts / ssteps,
                    "iters": infs[-1]["iters"], "ranks": infs[-1]["rank"],
                    "rel_diff_vs_stated_path": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                    "note": "outside the paper: PCG in DST coordinates, same settings"}

    bsteps = args.split_steps if args.split_steps is not None else args.steps
    split, split_parts = None, None
    if bsteps > 0:
        # the same mixed solve with split-BF16 products (hi hi' + hi lo' + lo hi' on the BF16 matrix
        # cores, FP32 accumulation) in its FP32 contractions: tp_gemm_mode(2); its FP32 contraction
        # class timed in a profiled pass as in the headline
        log("bench: mixed split-BF16 steps=%d (+ profiled pass)" % bsteps)
        try:
            ctx.gemm_mode(2)
            Xb, dtbs, infb, _ = run_solver(ctx, p, sk_by_q, SETTINGS["mixed"], bsteps, 1, False)
            _, _, _, prof_b = run_solver(ctx, p, sk_by_q, SETTINGS["mixed"], bsteps, 0, True)
        finally:
            ctx.gemm_mode(1)
        split_parts = Xb.numpy_parts()
        cb = kernel_classes(prof_b, bsteps)["gemm_f32"]
        split = {"solves_per_s": bsteps / dtbs, "ms_per_step": 1000.0 * dtbs / bsteps,
                 "iters": infb[-1]["iters"], "ranks": infb[-1]["rank"], "status": infb[-1]["status"],
                 "gemm_f32_launches_per_step": cb["launches_per_step"], "gemm_f32_avg_launch_us": cb["avg_launch_us"],
                 "gemm_f32_tflops": cb["achieved"],
                 "note": "tp_gemm_mode(2): the FP32 contractions with FP32 results take split-BF16 products "
                         "accumulated in FP32; gemm_f32_tflops counts the FP32 product's 2 M N K flops"}

    batched = None
    if args.batch_steps > 0:
        # independent control problems of the same shape (16 right-hand sides, seeds 2 and up: the
        # first is the workload itself) solved concurrently by tp_pcg_solve_batched on 8 streams
        from paper_1809_01971_amd._tp import batch_solve
        probs = [workloads.cfg3(seed=2 + i) for i in range(16)]
        log("bench: batched 16 problems x %d calls" % args.batch_steps)

        rhs = [tp.Rhs(q.weights, q.factors) for q in probs]

        def one_batch():
            return batch_solve(ctx, probs, lambda _: SETTINGS["mixed"], sk_by_q, streams=8, rhs=rhs,
                               workspace_per_stream=4 << 30)
        one_batch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            outs, res = one_batch()
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        rows = [np.arange(0, p.n, 16)] * 3
        a, b = ctx.eval_grid(outs[0], rows), ctx.eval_grid(Xm, rows)
        batched = {"problems": 16, "streams": 8, "solves_per_s": 16 * args.batch_steps / dtb,
                   "ms_per_call": 1000.0 * dtb / args.batch_steps,
                   "iters": sorted({r["iters"] for r in res}), "statuses": sorted({r["status"] for r in res}),
                   "rel_diff_first_vs_single": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                   "note": "16 independent n=2047 control problems (rhs seeds 2-17) per call, concurrent; one operator, so the 16 share one symbol build"}
        del outs

    sweep = None
    if not args.no_sweep:
        # per-solve time of the mixed solve over grid sizes (Gaussian-bump right-hand side of rank 10,
        # alpha = 0.3, gamma = 1e-3, cap 40, tolerance 1e-5); the operator sum grows with the spectrum
        sweep = {"note": "mixed solve, rank-10 Gaussian-bump rhs, alpha=0.3, gamma=1e-3, eps=1e-5, cap 40",
                 "n": [], "ms_per_solve": [], "iters": [], "ranks": [], "err_est": []}
        for n in (1023, 2047, 4095, 8191, 16383, 32767):
            pn = workloads.cfg5(n=n)
            s = dict(prec=1, eps=1e-5, tau=4e-5, cap=40, q=56, op_terms=40 if n > 4095 else 32, pre_terms=28)
            sk_by_q[(n, 56)] = sketch_tensors(workloads.sketch_matrices(n, 3, 56))
            steps = 3
            log("bench: sweep n=%d steps=%d" % (n, steps))
            _, dtw, infw, _ = run_solver(ctx, pn, sk_by_q, s, steps, 1, False)
            sweep["n"].append(n)
            sweep["ms_per_solve"].append(1000.0 * dtw / steps)
            sweep["iters"].append(infw[-1]["iters"])
            sweep["ranks"].append(infw[-1]["rank"])
            sweep["err_est"].append(infw[-1]["err_est"])
            del sk_by_q[(n, 56)]

    value = args.steps / dtm
    ms = 1000.0 * dtm / args.steps

    classes = kernel_classes(prof, args.steps)
    if TRAFFIC["src"] and traffic_key() == TRAFFIC["src"]:
        for k, v in classes.items():
            v["hbm_bytes_per_launch"] = TRAFFIC["bytes_per_launch"].get(k)
    classes_d = kernel_classes(prof_d, fsteps) if prof_d else None
    dom = max(classes, key=lambda k: classes[k]["ms_per_step"])
    cd = classes[dom]
    traffic = None
    if TRAFFIC["src"] and traffic_key() == TRAFFIC["src"]:
        traffic = TRAFFIC["bytes_per_launch"].get(dom)
    roofline = {"bound": cd["bound"], "achieved": cd["achieved"], "peak": cd["peak"], "unit": cd["unit"],
                "frac": cd["frac"], "traffic": traffic, "kernel": cd["kernel"], "class": dom,
                "launches_per_step": cd["launches_per_step"], "avg_launch_us": cd["avg_launch_us"],
                "algorithmic_per_launch": cd["algorithmic_per_launch"],
                "algorithmic_bytes_per_launch": cd["algorithmic_bytes_per_launch"],
                "measured_over": "a second pass of the same %d steps with HIP events around every launch "
                                 "on the context stream (%.2f ms per step with the events)" % (
                                     args.steps, 1000.0 * dtp / args.steps)}
    work = {"gflop_per_step": sum(v["flops"] for v in prof.values()) / args.steps / 1e9,
            "algorithmic_mb_per_step": sum(v["bytes"] for v in prof.values()) / args.steps / 1e6,
            "kernel_ms_per_step": sum(v["ms"] for v in prof.values()) / args.steps}

    cpu = None
    errs = [None, None]
    sinc_errs = {}
    if not args.no_cpu:
        hinfo = host_info()
        workers = args.cpu_workers or min(16, hinfo["usable_cpus"])
        sample = list(range(0, p.n, ERR_SLAB_STRIDE))
        log("bench: oracle over %d of %d spectral slabs, %d workers" % (len(sample), p.n, workers))
        t0 = time.perf_counter()
        errs = oracle_errors(p, [parts_m], sample, workers)
        tc = time.perf_counter() - t0
        errs += oracle_errors(p, [parts_d], sample, workers) if parts_d else [None]
        if split_parts:
            split["rel_err_vs_oracle"] = oracle_errors(p, [split_parts], sample, workers)[0]
            split["rel_err_note"] = "Parseval over every %dth spectral slab, as the headline" % ERR_SLAB_STRIDE
        if sinc_parts:
            sub = list(range(0, p.n, 4 * ERR_SLAB_STRIDE))
            names = sorted(sinc_parts)
            vals = oracle_errors(p, [sinc_parts[k] for k in names], sub, workers)
            sinc_errs = dict(zip(names, vals))
        full_s = tc * p.n / len(sample)
        cpu = dict(hinfo)
        cpu.update({"value": 1.0 / full_s, "unit": "solves/s", "cores": workers, "kind": "oracle",
                    "sample": "oracle O1 in the sine basis (exact spectral solve fhat / s(rho), slab by slab, "
                              "and the error sum against the GPU result; the two inverse transforms of a "
                              "physical-space solve are not done) over %d of %d first-index slabs (every "
                              "%dth), %.1f s on %d processes, scaled to all slabs" % (
                                  len(sample), p.n, ERR_SLAB_STRIDE, tc, workers)})
    for k, v in sinc.items():
        v["rel_err_vs_oracle"] = sinc_errs.get(k)
        v["rel_err_note"] = "Parseval over every %dth spectral slab" % (4 * ERR_SLAB_STRIDE)

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D n=2047, alpha=1/2, beta=1, gamma=1e-2, rank-8 rhs z/(1+k)",
                   "mixed": SETTINGS["mixed"], "fp64": SETTINGS["fp64"]},
        "fp64_solves_per_s": fsteps / dtd if dtd else None,
        "speedup_mixed_over_fp64": value / (fsteps / dtd) if dtd else None,
        "rel_err_mixed_vs_oracle": errs[0],
        "rel_err_fp64_vs_oracle": errs[1],
        "rel_err_note": "||X-u||/||u|| by Parseval over every %dth spectral slab of the 2047^3 grid" % ERR_SLAB_STRIDE,
        "iters_mixed": infm[-1]["iters"], "ranks_mixed": infm[-1]["rank"], "status_mixed": infm[-1]["status"],
        "iters_fp64": infd[-1]["iters"], "ranks_fp64": infd[-1]["rank"], "status_fp64": infd[-1].get("status"),
        "symbol_err_mixed": infm[-1]["sym_err"][0], "precond_err": infm[-1]["sym_err"][1],
        "sinc_symbol": sinc or None,
        "spectral_domain_mixed": spectral,
        "split_bf16_mixed": split,
        "batched_mixed": batched,
        "grid_sweep_mixed": sweep,
        "roofline": roofline, "kernel_classes_mixed": classes, "kernel_classes_fp64": classes_d,
        "fp64_profiled_ms_per_step": 1000.0 * dtdp / fsteps if dtdp else None,
        "work": work, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
