"""Kernel-level parity of the HIP library against the CPU oracle (single steps of the path)."""
import numpy as np
import pytest

import workloads
from oracle import exact, spectral, tensor
from tests.gpu_helpers import log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=1 << 30)
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 3, 63, 2047, 32767])
def test_lambda(ctx, n):
    log("lambda n=%d" % n)
    got = ctx.lam(n).cpu().numpy()
    np.testing.assert_allclose(got, spectral.eigenvalues(n), rtol=1e-13)


@pytest.mark.parametrize("n,cols", [(1, 3), (3, 5), (7, 1), (63, 37), (255, 300), (1023, 7), (2047, 65), (4095, 3)])
@pytest.mark.parametrize("prec", [0, 1])
def test_dst_matches_definition(ctx, n, cols, prec):
    import torch
    log("dst n=%d cols=%d prec=%d" % (n, cols, prec))
    x = np.random.default_rng(n + cols).standard_normal((n, cols))
    dt = torch.float64 if prec == 0 else torch.float32
    xt = torch.as_tensor(x, dtype=dt, device="cuda")
    got = ctx.dst(xt).double().cpu().numpy()
    ref = spectral.dst(x.astype(np.float32).astype(np.float64) if prec else x)
    # FP64: rounding grows like eps log2(N); FP32 columns are transformed in FP64 arithmetic, so
    # only their rounding to FP32 remains
    lg = np.log2(n + 1)
    tol = 4e-14 * lg if prec == 0 else 3e-7
    assert rel(got, ref) < tol
    # F is an involution
    back = ctx.dst(torch.as_tensor(got, dtype=dt, device="cuda")).double().cpu().numpy()
    assert rel(back, x) < 2 * tol


def test_dst_large_fp32(ctx):
    import torch
    n = 32767
    log("dst n=%d fp32" % n)
    x = np.random.default_rng(1).standard_normal((n, 2))
    got = ctx.dst(torch.as_tensor(x, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    import scipy.fft as sfft
    ref = sfft.dst(x.astype(np.float32).astype(np.float64), type=1, norm="ortho", axis=0)
    log("  rel %.2e" % rel(got, ref))
    assert rel(got, ref) < 3e-7


@pytest.mark.parametrize("n,k", [(2047, 1), (2047, 190), (8191, 1), (16383, 1500), (16383, 16383), (32767, 1),
                                 (32767, 3000), (32767, 30000), (32767, 32767)])
def test_dst_single_mode_fp32(ctx, n, k):
    """A single sine mode maps to one spike and back (F is orthonormal and its own inverse).  Modes at
    either end of the spectrum are the ill-conditioned case of the FFT-based DST-I: its
    pre-processing adds a sin(pi j/N)-weighted symmetric part to an antisymmetric one, which FP32
    arithmetic resolves only to about eps N / pi (7e-5 for the first mode at N = 32768).  FP32 columns
    are therefore transformed in FP64 arithmetic, and only the rounding of input and output to FP32
    remains."""
    import torch
    x = np.sin(k * np.pi * np.arange(1, n + 1) / (n + 1.0))[:, None]
    got = ctx.dst(torch.as_tensor(x, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    ref = spectral.dst(x.astype(np.float32).astype(np.float64))
    e1 = rel(got, ref)
    back = ctx.dst(torch.as_tensor(got, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    e2 = rel(back, x)
    log("dst single mode n=%d k=%d fp32: %.2e, round trip %.2e" % (n, k, e1, e2))
    assert e1 < 3e-7 and e2 < 6e-7


@pytest.mark.parametrize("K", [1, 2, 17, 64, 100, 128, 129, 200, 256])
def test_syev_matches_numpy(ctx, K):
    import torch
    log("syev K=%d" % K)
    rng = np.random.default_rng(K)
    A = rng.standard_normal((3, K, K))
    A = A + A.transpose(0, 2, 1)
    A[1] = A[1] @ A[1].T           # PSD with spread spectrum
    if K > 4:
        A[2, :, :] = 0.0
        Q = np.linalg.qr(rng.standard_normal((K, 4)))[0]
        A[2] = (Q * [5.0, 1.0, 1e-3, 1e-9]) @ Q.T   # rank 4, rest zero
    w, V = ctx.syev(torch.as_tensor(A, device="cuda"))
    w, V = w.cpu().numpy(), V.cpu().numpy()
    for b in range(3):
        ref = np.sort(np.linalg.eigvalsh(A[b]))[::-1]
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(w[b] - ref).max() <= 1e-12 * scale
        assert np.all(np.diff(w[b]) <= 1e-12 * scale)
        rec = (V[b] * w[b]) @ V[b].T
        assert np.abs(rec - A[b]).max() <= 1e-11 * scale
        assert np.abs(V[b].T @ V[b] - np.eye(K)).max() <= 1e-11


@pytest.mark.parametrize("d,n,alpha,cn,cp", [(3, 255, 0.5, 1.0, 1e-2), (3, 2047, 0.5, 1.0, 1e-2),
                                             (2, 63, 0.5, 1.0, 1e-2), (3, 255, 0.25, 1.0, 1e-3),
                                             (3, 127, 0.9, 1.0, 1e-1), (3, 63, 1.0, 1.0, 1e-2)])
def test_symbol_matches_exact_power(ctx, d, n, alpha, cn, cp):
    log("symbol d=%d n=%d alpha=%g" % (d, n, alpha))
    op, pre, (eo, ep) = ctx.symbol_build(d, n, alpha, cn, cp, op_terms=32, pre_terms=12)
    rng = np.random.default_rng(n)
    idx = rng.integers(0, n, size=(20000, d))
    idx[:4] = [[0] * d, [n - 1] * d, [0] * (d - 1) + [n - 1], [n // 2] * d]
    lam = spectral.eigenvalues(n)
    rho = lam[idx].sum(axis=1)
    s = spectral.symbol(rho, alpha, cn, cp)
    so = op.eval(idx)
    sp = pre.eval(idx)
    err_op = np.abs(so / s - 1).max()
    err_pre = np.abs(sp * s - 1).max()
    log("  op err %.2e (reported %.2e) pre err %.2e (reported %.2e)" % (err_op, eo, err_pre, ep))
    assert err_op <= 1.05 * eo + 1e-13
    assert err_pre <= 1.05 * ep + 1e-13
    assert eo < 2e-5
    assert ep < 5e-2
    assert sp.min() > 0
    # alpha = 1: c_pos rho is kept exact as one more (tau = 0) term
    assert op.info()[0] == d * (32 + (alpha == 1.0))


def test_symbol_sinc_rule_matches_power(ctx):
    n, d, alpha = 255, 3, 0.5
    log("symbol sinc n=%d" % n)
    op, pre, (eo, ep) = ctx.symbol_build(d, n, alpha, 1.0, 1e-2, method=1, sinc_kl=120, sinc_kr=40, sinc_h=0.45)
    idx = np.random.default_rng(3).integers(0, n, size=(5000, d))
    rho = spectral.eigenvalues(n)[idx].sum(axis=1)
    s = spectral.symbol(rho, alpha, 1.0, 1e-2)
    err = np.abs(op.eval(idx) / s - 1).max()
    assert err <= 1.05 * eo + 1e-13
    assert eo < 1e-5


@pytest.mark.parametrize("d,n,R", [(3, 15, 4), (2, 31, 6), (3, 31, 1)])
@pytest.mark.parametrize("prec", [0, 1])
def test_from_cp_and_eval_grid(ctx, d, n, R, prec):
    import paper_1809_01971_amd as tp
    log("from_cp d=%d n=%d R=%d prec=%d" % (d, n, R, prec))
    rng = np.random.default_rng(d * n + R)
    F = [rng.standard_normal((n, R)) for _ in range(d)]
    w = rng.standard_normal(R)
    X = tp.Tensor(d, n, 16, prec)
    ctx.from_cp(w, F, X)
    full = ctx.eval_grid(X, [np.arange(n)] * d)
    ref = tensor.cp_full(w, F)
    assert rel(full, ref) < (1e-13 if prec == 0 else 2e-6)
    assert X.rank == [min(R, n)] * d
    # sub-grid evaluation agrees with the restriction
    rows = [np.arange(0, n, 3)] * d
    sub = ctx.eval_grid(X, rows)
    assert rel(sub, ref[np.ix_(*rows)]) < (1e-13 if prec == 0 else 2e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_inner_products(ctx, prec):
    import paper_1809_01971_amd as tp
    n, d = 31, 3
    log("inner prec=%d" % prec)
    rng = np.random.default_rng(11)
    Fa = [rng.standard_normal((n, 3)) for _ in range(d)]
    Fb = [rng.standard_normal((n, 5)) for _ in range(d)]
    wa, wb = rng.standard_normal(3), rng.standard_normal(5)
    A, B = tp.Tensor(d, n, 16, prec), tp.Tensor(d, n, 16, prec)
    ctx.from_cp(wa, Fa, A)
    ctx.from_cp(wb, Fb, B)
    ref = tensor.inner(tensor.cp_full(wa, Fa), tensor.cp_full(wb, Fb))
    scale = np.linalg.norm(tensor.cp_full(wa, Fa)) * np.linalg.norm(tensor.cp_full(wb, Fb))
    assert abs(ctx.inner(A, B) - ref) <= (1e-13 if prec == 0 else 1e-6) * scale


@pytest.mark.parametrize("mfma", [1, 0])
@pytest.mark.parametrize("prec", [0, 1])
def test_inner_products_both_gemm_modes(ctx, mfma, prec):
    """The matrix-core and the FMA contraction tiles give the same Gram inner products."""
    import paper_1809_01971_amd as tp
    log("inner gemm mode mfma=%d prec=%d" % (mfma, prec))
    ctx.gemm_mode(bool(mfma))
    try:
        n, d = 255, 3
        rng = np.random.default_rng(12)
        Fa = [rng.standard_normal((n, 40)) for _ in range(d)]
        Fb = [rng.standard_normal((n, 33)) for _ in range(d)]
        wa, wb = rng.standard_normal(40), rng.standard_normal(33)
        A, B = tp.Tensor(d, n, 64, prec), tp.Tensor(d, n, 64, prec)
        ctx.from_cp(wa, Fa, A)
        ctx.from_cp(wb, Fb, B)
        G = np.ones((40, 33))
        for a_, b_ in zip(Fa, Fb):
            G = G * (a_.T @ b_)
        ref = wa @ G @ wb
        scale = np.sqrt((wa @ (np.prod([f.T @ f for f in Fa], axis=0)) @ wa) * (wb @ (np.prod([f.T @ f for f in Fb], axis=0)) @ wb))
        assert abs(ctx.inner(A, B) - ref) <= (1e-12 if prec == 0 else 1e-5) * scale
    finally:
        ctx.gemm_mode(True)


@pytest.mark.parametrize("eps", [1e-2, 1e-5, 1e-7])
@pytest.mark.parametrize("prec", [0, 1])
def test_truncate_sum_hosvd_bound(ctx, eps, prec):
    """HOSVD bound ||T - T_r|| <= eps ||T||.  Mode spectra come from FP64 Gram matrices, which
    resolve singular values down to about 1e-8 of the largest, so eps stays above that floor."""
    import paper_1809_01971_amd as tp
    if prec == 1 and eps < 1e-6:
        pytest.skip("below FP32 resolution")
    n, d = 31, 3
    log("truncate eps=%g prec=%d" % (eps, prec))
    rng = np.random.default_rng(5)
    # two tensors whose sum has decaying mode spectra
    F1 = [rng.standard_normal((n, 6)) * (0.3 ** np.arange(6)) for _ in range(d)]
    F2 = [rng.standard_normal((n, 6)) * (0.2 ** np.arange(6)) for _ in range(d)]
    w1, w2 = np.ones(6), np.ones(6)
    A, B, Y = tp.Tensor(d, n, 32, prec), tp.Tensor(d, n, 32, prec), tp.Tensor(d, n, 32, prec)
    ctx.from_cp(w1, F1, A)
    ctx.from_cp(w2, F2, B)
    ctx.truncate([1.0, -0.7], [A, B], Y, eps, 32)
    full_ref = tensor.cp_full(w1, F1) - 0.7 * tensor.cp_full(w2, F2)
    got = ctx.eval_grid(Y, [np.arange(n)] * d)
    err = rel(got, full_ref)
    _, _, ranks = tensor.hosvd_truncate(full_ref, eps)
    log("  err %.2e ranks %s oracle ranks %s" % (err, Y.rank, ranks))
    assert err <= eps * 1.01 + (0 if prec == 0 else 2e-6)
    assert all(abs(a - b) <= 1 for a, b in zip(Y.rank, ranks))
    # in-place: Y = trunc(Y + A)
    ctx.truncate([1.0, 1.0], [Y, A], Y, eps, 32)
    got2 = ctx.eval_grid(Y, [np.arange(n)] * d)
    assert rel(got2, full_ref + tensor.cp_full(w1, F1)) <= 2.5 * eps + (0 if prec == 0 else 4e-6)


@pytest.mark.parametrize("a,c,e", [(40, 56, 56), (4, 63, 63), (70, 26, 26), (20, 76, 40)])
def test_truncate_large_rank_sums_fp64(ctx, a, c, e):
    """FP64 sums X1 + X2 with X1 = A + C and X2 = -A + D (canonical ranks a, c, e): the stacked
    factors have a + c + a + e = 134..192 columns per mode and a joint span of a + c + e (the
    orthonormalisation's pivoted Cholesky of orders above 128, rank-deficient), while the sum is
    exactly C + D.  Truncated at eps = 1e-12, the result is C + D (checked on every 5th grid index
    per mode) with mode ranks c + e."""
    import paper_1809_01971_amd as tp
    n, d = 255, 3
    log("truncate large ranks a=%d c=%d e=%d" % (a, c, e))
    rng = np.random.default_rng(a + 7 * c + 13 * e)
    FA = [rng.standard_normal((n, a)) for _ in range(d)]
    FC = [rng.standard_normal((n, c)) for _ in range(d)]
    FD = [rng.standard_normal((n, e)) for _ in range(d)]
    wA, wC, wD = rng.standard_normal(a), rng.standard_normal(c), rng.standard_normal(e)
    X1, X2, Y = tp.Tensor(d, n, 128, 0), tp.Tensor(d, n, 128, 0), tp.Tensor(d, n, 128, 0)
    ctx.from_cp(np.concatenate([wA, wC]), [np.hstack([FA[m], FC[m]]) for m in range(d)], X1)
    ctx.from_cp(np.concatenate([-wA, wD]), [np.hstack([FA[m], FD[m]]) for m in range(d)], X2)
    assert list(X1.rank) == [a + c] * d and list(X2.rank) == [a + e] * d
    ctx.truncate([1.0, 1.0], [X1, X2], Y, 1e-12, 128)
    rows = np.arange(0, n, 5)
    got = ctx.eval_grid(Y, [rows] * d)
    ref = tensor.cp_full(wC, [f[rows] for f in FC]) + tensor.cp_full(wD, [f[rows] for f in FD])
    err = rel(got, ref)
    log("  err %.2e ranks %s" % (err, Y.rank))
    assert err <= 1e-10
    assert list(Y.rank) == [c + e] * d


@pytest.mark.parametrize("d,n,alpha", [(3, 31, 0.5), (2, 63, 0.25), (3, 63, 0.75)])
@pytest.mark.parametrize("prec", [0, 1])
def test_apply_matches_spectral_product(ctx, d, n, alpha, prec):
    """y = F(s (.) F x) for a low-rank x, against the exact symbol on the full grid."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    log("apply d=%d n=%d alpha=%g prec=%d" % (d, n, alpha, prec))
    cn, cp = 1.0, 1e-2
    op, pre, (eo, ep) = ctx.symbol_build(d, n, alpha, cn, cp, prec=prec, op_terms=32, pre_terms=12)
    rng = np.random.default_rng(n)
    F = [rng.standard_normal((n, 3)) for _ in range(d)]
    w = np.ones(3)
    X, Y = tp.Tensor(d, n, 64, prec), tp.Tensor(d, n, 64, prec)
    ctx.from_cp(w, F, X)
    q = min(100, n)
    sk = sketch_tensors(workloads.sketch_matrices(n, d, q))
    tol = 1e-7 if prec == 0 else 1e-5
    ctx.apply(op, X, Y, tol, 64, sk, allow_erank=True)
    f = tensor.cp_full(w, F)
    ref = exact.apply_full(f, alpha, cn, cp)
    got = ctx.eval_grid(Y, [np.arange(n)] * d)
    err = rel(got, ref)
    log("  apply err %.2e (sym %.2e) ranks %s" % (err, eo, Y.rank))
    assert err <= eo + 3 * tol + (0 if prec == 0 else 1e-5)
    # preconditioner product against 1/s
    ctx.apply(pre, X, Y, tol, 64, sk, allow_erank=True)
    refp = exact.solve_full(f, alpha, cn, cp)
    errp = rel(ctx.eval_grid(Y, [np.arange(n)] * d), refp)
    assert errp <= ep + 3 * tol + (0 if prec == 0 else 1e-5)


@pytest.mark.parametrize("d,n", [(3, 31), (2, 63)])
@pytest.mark.parametrize("prec", [0, 1])
def test_apply_sum_and_structured_inner(ctx, d, n, prec):
    """R - a F(s (.) F P) truncated as one sum, and <P, F(s (.) F P)> without truncation."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    log("apply_sum d=%d n=%d prec=%d" % (d, n, prec))
    alpha, cn, cp = 0.5, 1.0, 1e-2
    op, pre, (eo, ep) = ctx.symbol_build(d, n, alpha, cn, cp, prec=prec, op_terms=32, pre_terms=12)
    rng = np.random.default_rng(3 * n + d)
    F1 = [rng.standard_normal((n, 3)) for _ in range(d)]
    F2 = [rng.standard_normal((n, 2)) for _ in range(d)]
    w1, w2 = np.ones(3), np.ones(2)
    R, P, Y = tp.Tensor(d, n, 64, prec), tp.Tensor(d, n, 64, prec), tp.Tensor(d, n, 64, prec)
    ctx.from_cp(w1, F1, R)
    ctx.from_cp(w2, F2, P)
    sk = sketch_tensors(workloads.sketch_matrices(n, d, n))
    tol = 1e-7 if prec == 0 else 1e-5
    a = 0.37
    ctx.apply_sum([None, op], [R, P], [1.0, -a], Y, tol, 64, sk, allow_erank=True)
    r_full, p_full = tensor.cp_full(w1, F1), tensor.cp_full(w2, F2)
    ap = exact.apply_full(p_full, alpha, cn, cp)
    ref = r_full - a * ap
    got = ctx.eval_grid(Y, [np.arange(n)] * d)
    err = rel(got, ref)
    log("  err %.2e" % err)
    assert err <= (a * np.linalg.norm(ap) / np.linalg.norm(ref)) * eo + 3 * tol + (0 if prec == 0 else 1e-5)
    ps = ctx.inner_sym(P, op, P)
    ps_ref = tensor.inner(p_full, ap)
    assert abs(ps - ps_ref) <= (eo + (1e-12 if prec == 0 else 2e-6)) * abs(ps_ref)
