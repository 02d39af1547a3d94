"""Batched independent solves (a sample of the 256-problem batch) and large grids (n up to 32767)
on the GPU, checked against the exact oracle O1 or, where O1 cannot reach, against what holds at any
size: the single-sine-mode closed form and agreement of the mixed and FP64 tensor solves."""
import numpy as np
import pytest

import workloads
from oracle import exact, tensor
from tests.gpu_helpers import global_rel_error, log, rel

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-4


def _mixed(p, cap=40):
    return dict(prec=1, eps=1e-5, tau=4e-5, cap=cap, op_terms=28, pre_terms=28)


def _batch(p):
    # the rank cap follows the tolerance: alpha near 0.8 needs Tucker ranks up to ~70 at 1e-5
    return _mixed(p, cap=80)


@pytest.fixture(scope="module")
def ctx():
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=8 << 30)
    yield c
    c.close()


def _single(ctx, p, s, sk):
    import paper_1809_01971_amd as tp
    op, pre, errs = ctx.symbol_build(p.d, p.n, p.alpha, p.c_neg, p.c_pos, prec=s["prec"],
                                     op_terms=s["op_terms"], pre_terms=s["pre_terms"])
    X = tp.Tensor(p.d, p.n, s["cap"], s["prec"])
    st, info = ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=s["tau"], kmax=100, trunc_tol=s["eps"],
                             cap=s["cap"], sketch=sk)
    op.free()
    pre.free()
    info["sym_err"] = errs
    return X, info


def test_batched_sample_against_oracle(ctx):
    """The first 12 problems of the batch (n in {127, 255, 511, 1023}, alpha in [0.1, 0.9], gamma in
    [1e-4, 1e-1], rank 1-12), solved together on 4 streams with tolerance 1e-5 and a rank cap large
    enough for it: every result within 1e-4 of the exact control (Parseval over every 4th spectral
    slab, an unbiased sample of the whole-grid error), and two of them equal to the same problem
    solved alone."""
    from paper_1809_01971_amd._tp import batch_solve, sketch_tensors
    probs = workloads.cfg4()[:12]
    sks = {n: sketch_tensors(workloads.sketch_matrices(n, 3, 96)) for n in sorted({p.n for p in probs})}
    log("batch of %d, n = %s" % (len(probs), [p.n for p in probs]))
    outs, res = batch_solve(ctx, probs, _batch, sks, streams=4, workspace_per_stream=2 << 30)
    for p, X, r in zip(probs, outs, res):
        core, fs = X.numpy_parts()
        err = global_rel_error(p, core, fs, stride=4)
        log("  %s n=%d alpha=%.2f gamma=%.1e rank=%d: err %.2e %s" % (p.name, p.n, p.alpha, p.c_pos, len(p.weights),
                                                                   err, r))
        assert r["status"] in (0, 4)
        assert err < MIXED_TOL
    for i in (0, 5):
        p = probs[i]
        X, info = _single(ctx, p, _batch(p), sks[p.n])
        rows = [np.arange(0, p.n, 5)] * 3
        d = rel(ctx.eval_grid(X, rows), ctx.eval_grid(outs[i], rows))
        log("  single vs batched %s: %.2e" % (p.name, d))
        assert d < 1e-10


def test_sine_mode_n32767_mixed(ctx):
    """Largest grid of the mixed path: a single sine mode is solved exactly by the closed form.
    The spectrum spans rho_max/rho_min = 4.4e8 here; the operator's exponential sum needs 40 terms
    for 3e-6 (28 terms give 2.5e-4, which the solution error follows one to one)."""
    from paper_1809_01971_amd._tp import sketch_tensors
    n, ks = 32767, (5, 1, 3000)
    p = workloads.sine_mode_problem(n, 3, ks, 0.3, 1.0, 1e-3)
    s = dict(prec=1, eps=1e-6, tau=4e-5, cap=8, op_terms=40, pre_terms=28)
    X, info = _single(ctx, p, s, sketch_tensors(workloads.sketch_matrices(n, 3, 16)))
    fac = exact.single_mode_factor((n,) * 3, ks, 0.3, 1.0, 1e-3)
    rows = [np.arange(0, n, 1021)] * 3
    err = rel(ctx.eval_grid(X, rows), fac * tensor.cp_full(p.weights, [f[r] for f, r in zip(p.factors, rows)]))
    log("sine mode n=%d: err %.2e info %s" % (n, err, info))
    assert info["sym_err"][0] < 1e-5
    assert err < MIXED_TOL


def test_bumps_n16383_mixed_vs_fp64(ctx):
    """The Gaussian-bump right-hand side at n = 16383: the mixed and FP64
    tensor solves agree to 1e-4 on a sampled 128^3 sub-grid, and the FP64 solve's error estimate is
    below its tolerance.  Exponential sums: 36 terms (5e-6) mixed, 48 (7e-8) FP64."""
    from paper_1809_01971_amd._tp import sketch_tensors
    p = workloads.cfg5(n=16383)
    sk = sketch_tensors(workloads.sketch_matrices(p.n, 3, 56))
    Xm, im = _single(ctx, p, dict(_mixed(p), op_terms=36), sk)
    sk64 = sketch_tensors(workloads.sketch_matrices(p.n, 3, 76))
    Xd, idd = _single(ctx, p, dict(prec=0, eps=1e-7, tau=4e-7, cap=60, op_terms=48, pre_terms=36), sk64)
    rows = [np.arange(0, p.n, 128)] * 3
    d = rel(ctx.eval_grid(Xm, rows), ctx.eval_grid(Xd, rows))
    log("bumps n=%d: mixed vs fp64 %.2e; mixed %s; fp64 %s" % (p.n, d, im, idd))
    assert im["status"] in (0, 4) and idd["status"] in (0, 4)
    assert d < MIXED_TOL
    assert idd["err_est"] < 4e-7


def test_batched_calls_reuse_their_workers(ctx):
    """Two batched calls in one context, with 2 and then 4 streams (the workers of the first call
    are kept and two are added; each worker's symbols live in its workspace and are released after
    every problem): every result equals the one of the first call."""
    from paper_1809_01971_amd._tp import batch_solve, sketch_tensors
    probs = workloads.cfg4()[:6]
    sks = {n: sketch_tensors(workloads.sketch_matrices(n, 3, 96)) for n in sorted({p.n for p in probs})}
    outs2, res2 = batch_solve(ctx, probs, _batch, sks, streams=2, workspace_per_stream=2 << 30)
    outs4, res4 = batch_solve(ctx, probs, _batch, sks, streams=4, workspace_per_stream=2 << 30)
    for p, a, b, ra, rb in zip(probs, outs2, outs4, res2, res4):
        rows = [np.arange(0, p.n, 7)] * 3
        d = rel(ctx.eval_grid(b, rows), ctx.eval_grid(a, rows))
        log("  %s: %s / %s diff %.1e" % (p.name, ra, rb, d))
        assert ra["iters"] == rb["iters"] and d < 1e-12
