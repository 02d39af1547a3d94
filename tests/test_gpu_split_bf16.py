"""Split-BF16 products for the FP32 contractions (tp_gemm_mode(2)): each FP32 operand x is split
into hi = bf16(x) and lo = bf16(x - hi), and a product is hi hi' + hi lo' + lo hi' on the BF16
matrix cores, accumulated in FP32, so each product carries a relative error of at most about
3 * 2^-16 (typically far less) instead of 2^-24.  Checked against the oracle at the contraction
(symbol product) and at the benchmark workload's full solve, where the mixed tolerance of 1e-4
applies."""
import numpy as np
import pytest

import workloads
from oracle import exact, tensor
from tests.gpu_helpers import global_rel_error, log, rel

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-4     # relative error vs the exact control, mixed precision
SPLIT_EPS = 2.0 ** -16  # unit of the split products' relative error (at most about 3 of it per product)


@pytest.fixture(scope="module")
def ctx():
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=8 << 30)
    yield c
    c.gemm_mode(1)
    c.close()


@pytest.mark.parametrize("d,n,alpha", [(3, 31, 0.5), (2, 63, 0.25), (3, 63, 0.75), (3, 255, 0.5)])
def test_split_bf16_symbol_product(ctx, d, n, alpha):
    """y = F(s (.) F x) for a low-rank x with the split-BF16 contractions, against the exact symbol
    on the full grid and against the same product with FP32 matrix-core contractions.  The split
    adds at most about 3 * 2^-16 per product to the FP32 path's rounding; the bound allows 4 * 2^-16
    of relative error in the result beside the symbol fit error and the truncation tolerance."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    log("split-bf16 apply d=%d n=%d alpha=%g" % (d, n, alpha))
    cn, cp = 1.0, 1e-2
    op, pre, (eo, ep) = ctx.symbol_build(d, n, alpha, cn, cp, prec=1, op_terms=32, pre_terms=12)
    rng = np.random.default_rng(n + d)
    F = [rng.standard_normal((n, 3)) for _ in range(d)]
    w = np.ones(3)
    X = tp.Tensor(d, n, 64, 1)
    Y1, Y2 = tp.Tensor(d, n, 64, 1), tp.Tensor(d, n, 64, 1)
    ctx.from_cp(w, F, X)
    sk = sketch_tensors(workloads.sketch_matrices(n, d, min(100, n)))
    tol = 1e-5
    rows = [np.arange(n)] * d if n < 255 else [np.arange(0, n, 3)] * d
    try:
        ctx.gemm_mode(1)
        ctx.apply(op, X, Y1, tol, 64, sk, allow_erank=True)
        ctx.gemm_mode(2)
        ctx.apply(op, X, Y2, tol, 64, sk, allow_erank=True)
        g1, g2 = ctx.eval_grid(Y1, rows), ctx.eval_grid(Y2, rows)
        ctx.apply(pre, X, Y2, tol, 64, sk, allow_erank=True)
        gp = ctx.eval_grid(Y2, rows)
    finally:
        ctx.gemm_mode(1)
    f = tensor.cp_full(w, F)
    sub = np.ix_(*rows)
    ref = exact.apply_full(f, alpha, cn, cp)[sub]
    err, d12 = rel(g2, ref), rel(g2, g1)
    errp = rel(gp, exact.solve_full(f, alpha, cn, cp)[sub])
    log("  err %.2e (FP32 path %.2e, sym %.2e), split vs FP32 %.2e, pre err %.2e" % (err, rel(g1, ref), eo, d12, errp))
    assert err <= eo + 3 * tol + 4 * SPLIT_EPS
    assert d12 <= 3 * tol + 4 * SPLIT_EPS
    assert errp <= ep + 3 * tol + 4 * SPLIT_EPS


def test_split_bf16_n2047_solve_against_oracle(ctx):
    """The benchmark workload (3D n = 2047, alpha = 1/2, rank-8 right-hand side) with the
    split-BF16 contractions and the benchmark's mixed settings: the relative error against the exact
    control, by Parseval over every 8th spectral slab of the 2047^3 grid, within the mixed
    tolerance; a second solve gives the same result bit for bit (the split and the accumulation
    order are fixed)."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    p = workloads.cfg3()
    log("split-bf16 cfg3 n=2047")
    sk = sketch_tensors(workloads.sketch_matrices(p.n, 3, 64))
    rows = [np.arange(0, p.n, 64)] * 3
    out = []
    try:
        ctx.gemm_mode(2)
        for _ in range(2):
            op, pre, errs = ctx.symbol_build(3, p.n, p.alpha, p.c_neg, p.c_pos, prec=1, op_terms=28, pre_terms=28)
            X = tp.Tensor(3, p.n, 56, 1)
            st, info = ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=1.2e-4, kmax=100, trunc_tol=3e-5,
                                     cap=56, sketch=sk)
            out.append((X, st, info, ctx.eval_grid(X, rows)))
    finally:
        ctx.gemm_mode(1)
    X, st, info, g = out[0]
    core, fs = X.numpy_parts()
    err = global_rel_error(p, core, fs, stride=8)
    log("  err %.2e info %s" % (err, info))
    assert info["status"] in (0, 4)
    assert info["iters"] <= 5
    assert err < MIXED_TOL
    assert np.array_equal(g, out[1][3])


def test_gemm_mode_rejects_unknown_modes(ctx):
    from paper_1809_01971_amd._tp import TPError
    with pytest.raises(TPError):
        ctx.gemm_mode(3)
    with pytest.raises(TPError):
        ctx.gemm_mode(-1)
