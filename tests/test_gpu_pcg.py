"""End-to-end parity of the GPU PCG control solve against the exact oracle O1."""
import numpy as np
import pytest

import workloads
from oracle import exact, spectral, tensor
from tests.gpu_helpers import global_rel_error, log, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-6     # relative error vs the exact control, FP64 mode
MIXED_TOL = 1e-4    # relative error vs the exact control, mixed precision


@pytest.fixture(scope="module")
def ctx():
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=8 << 30)
    yield c
    c.close()


def solve(ctx, p, prec, eps, tau, cap=64, q=None, op_terms=32, pre_terms=28, spectral=False):
    """The sketch width is the cap plus an oversampling of 16 columns.  tau is compared with the
    error estimate ||Z||/||X||, whose floor is about 2-3 times the truncation tolerance eps."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    op, pre, errs = ctx.symbol_build(p.d, p.n, p.alpha, p.c_neg, p.c_pos, prec=prec, op_terms=op_terms,
                                     pre_terms=pre_terms)
    q = q or min(cap + 16, 192)
    sk = sketch_tensors(workloads.sketch_matrices(p.n, p.d, q))
    X = tp.Tensor(p.d, p.n, cap, prec)
    st, info = ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=tau, kmax=100, trunc_tol=eps, cap=cap,
                             sketch=sk, true_residual=True, spectral_domain=spectral)
    info["sym_err"] = errs
    return X, st, info


def test_cfg1_2d_fp64_against_full_grid_and_brute_force(ctx):
    """The 2D workload (n = 63) in FP64 against the full-grid O1 and the dense brute force
    (3969 x 3969 Kronecker-sum matrix, numpy eigh, no sine transform)."""
    p = workloads.cfg1()
    log("cfg1 fp64")
    X, st, info = solve(ctx, p, 0, eps=1e-8, tau=4e-8, op_terms=40, pre_terms=36)
    f = tensor.cp_full(p.weights, p.factors)
    u = exact.solve_full(f, p.alpha, p.c_neg, p.c_pos)
    ub = exact.brute_force(f, p.alpha, p.c_neg, p.c_pos)
    got = ctx.eval_grid(X, [np.arange(p.n)] * 2)
    err, errb = rel(got, u), rel(got, ub)
    log("  cfg1 err %.2e (brute force %.2e) info %s" % (err, errb, info))
    assert err < FP64_TOL and errb < FP64_TOL
    assert info["iters"] <= 20


def test_stall_keeps_best_iterate(ctx):
    """tau far below the FP32 floor: the solve must stop on its own (estimate grown 8-fold
    over its minimum) well before kmax, report TP_ENOCONV and return its best iterate."""
    from paper_1809_01971_amd._tp import TP_ENOCONV
    p = workloads.sine_mode_problem(2047, 2, (1, 2), 0.5, 1.0, 1e-2)
    log("stall: sine mode n=2047 mixed, tau=1e-9")
    X, st, info = solve(ctx, p, 1, eps=1e-6, tau=1e-9, cap=8, q=16)
    fac = exact.single_mode_factor((p.n,) * 2, (1, 2), 0.5, 1.0, 1e-2)
    rows = [np.arange(0, p.n, 31)] * 2
    err = rel(ctx.eval_grid(X, rows), fac * tensor.cp_full(p.weights, [f[r] for f, r in zip(p.factors, rows)]))
    log("  err %.2e info %s" % (err, info))
    assert st == TP_ENOCONV and info["status"] == TP_ENOCONV
    assert info["iters"] < 100
    assert err < MIXED_TOL
    assert info["err_est"] < 1e-4


def test_cfg1_2d_mixed(ctx):
    p = workloads.cfg1()
    log("cfg1 mixed")
    X, st, info = solve(ctx, p, 1, eps=1e-6, tau=4e-6)
    u = exact.solve_full(tensor.cp_full(p.weights, p.factors), p.alpha, p.c_neg, p.c_pos)
    err = rel(ctx.eval_grid(X, [np.arange(p.n)] * 2), u)
    log("  cfg1 mixed err %.2e info %s" % (err, info))
    assert err < MIXED_TOL


@pytest.mark.parametrize("n,ks", [(63, (3, 5)), (2047, (1, 2)), (2047, (700, 3))])
@pytest.mark.parametrize("prec", [0, 1])
def test_single_sine_mode_closed_form(ctx, n, ks, prec):
    d = len(ks)
    p = workloads.sine_mode_problem(n, d, ks, 0.5, 1.0, 1e-2)
    log("sine mode n=%d ks=%s prec=%d" % (n, ks, prec))
    # mixed: the estimate ||Z||/||X|| bottoms out near 1e-5 at n=2047 (FP32 rounding of the
    # operator product, amplified by s_max/s_min), so tau sits above that floor
    X, st, info = solve(ctx, p, prec, eps=1e-8 if prec == 0 else 1e-6, tau=4e-8 if prec == 0 else 4e-5, cap=8, q=16)
    assert info["status"] in (0, 4)  # converged (4: an intermediate sum met the rank cap 8)
    fac = exact.single_mode_factor((n,) * d, ks, 0.5, 1.0, 1e-2)
    rows = [np.arange(0, n, max(1, n // 64))] * d
    got = ctx.eval_grid(X, rows)
    ref = fac * tensor.cp_full(p.weights, [f[r] for f, r in zip(p.factors, rows)])
    err = rel(got, ref)
    log("  err %.2e info %s" % (err, info))
    assert err < (FP64_TOL if prec == 0 else MIXED_TOL)


@pytest.mark.parametrize("alpha,gamma", [(0.5, 1e-2), (0.25, 1e-1), (0.75, 1e-3)])
def test_cfg2_type_n63_fp64(ctx, alpha, gamma):
    p = workloads.cfg2(alpha=alpha, gamma=gamma, n=63)
    log("cfg2-type n=63 alpha=%g gamma=%g" % (alpha, gamma))
    X, st, info = solve(ctx, p, 0, eps=1e-7, tau=4e-7, pre_terms=36)
    u = exact.solve_full(tensor.cp_full(p.weights, p.factors), p.alpha, p.c_neg, p.c_pos)
    err = rel(ctx.eval_grid(X, [np.arange(p.n)] * 3), u)
    log("  err %.2e info %s" % (err, info))
    assert err < FP64_TOL


@pytest.mark.parametrize("alpha,gamma", [(0.25, 1e-1), (0.25, 1e-3), (0.5, 1e-1), (0.5, 1e-3), (0.75, 1e-1),
                                         (0.75, 1e-3)])
def test_cfg2_n255_fp64(ctx, alpha, gamma):
    """All six problems of the n = 255 configuration, FP64, the rank cap raised to what the tolerance
    needs (96), against the full-grid O1."""
    p = workloads.cfg2(alpha=alpha, gamma=gamma)
    log("cfg2 n=255 alpha=%g gamma=%g" % (alpha, gamma))
    assert p.n == 255
    X, st, info = solve(ctx, p, 0, eps=2e-7, tau=8e-7, cap=96, op_terms=36, pre_terms=36)
    u = exact.solve_full(tensor.cp_full(p.weights, p.factors), p.alpha, p.c_neg, p.c_pos)
    err = rel(ctx.eval_grid(X, [np.arange(p.n)] * 3), u)
    log("  err %.2e info %s" % (err, info))
    assert err < FP64_TOL


@pytest.mark.parametrize("alpha,gamma", [(0.5, 1e-1), (0.25, 1e-3)])
def test_cfg2_n255_mixed(ctx, alpha, gamma):
    p = workloads.cfg2(alpha=alpha, gamma=gamma)
    log("cfg2 mixed n=255 alpha=%g gamma=%g" % (alpha, gamma))
    X, st, info = solve(ctx, p, 1, eps=2e-5, tau=8e-5, cap=64, op_terms=28, pre_terms=28)
    u = exact.solve_full(tensor.cp_full(p.weights, p.factors), p.alpha, p.c_neg, p.c_pos)
    err = rel(ctx.eval_grid(X, [np.arange(p.n)] * 3), u)
    log("  err %.2e info %s" % (err, info))
    assert err < MIXED_TOL


@pytest.mark.parametrize("prec", [1, 0])
def test_cfg3_n2047_global_error(ctx, prec):
    """The benchmark workload at full size: exact relative error over all 2047^3 points by
    Parseval (oracle.exact.tucker_error_slabs over every spectral slab)."""
    p = workloads.cfg3()
    log("cfg3 n=2047 prec=%d" % prec)
    if prec == 1:
        X, st, info = solve(ctx, p, 1, eps=3e-5, tau=1.2e-4, cap=56, q=64, op_terms=28, pre_terms=28)
        tol = MIXED_TOL
    else:
        X, st, info = solve(ctx, p, 0, eps=1.5e-7, tau=6e-7, cap=96, q=112, op_terms=36, pre_terms=36)
        tol = FP64_TOL
    core, fs = X.numpy_parts()
    err = global_rel_error(p, core, fs)
    log("  global err %.2e info %s" % (err, info))
    assert info["iters"] <= 5
    assert err < tol


@pytest.mark.parametrize("prec", [0, 1])
def test_cfg3_n2047_printed_recursion(ctx, prec):
    """Algorithm alg:pcg as printed, on the benchmark workload: the recursive residual
    R = trunc(R - a trunc(fun(P))) and the stop on ||R|| / ||B|| <= tau; the error against the exact
    control by Parseval over every 8th spectral slab of the 2047^3 grid."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import TP_STOP_RESIDUAL, sketch_tensors
    p = workloads.cfg3()
    log("cfg3 printed recursion prec=%d" % prec)
    if prec == 1:
        eps, tau, cap, q, K, tol = 3e-5, 1e-4, 56, 64, 28, MIXED_TOL
    else:
        eps, tau, cap, q, K, tol = 1.5e-7, 1e-6, 96, 112, 36, FP64_TOL
    op, pre, errs = ctx.symbol_build(3, p.n, p.alpha, p.c_neg, p.c_pos, prec=prec, op_terms=K, pre_terms=K)
    sk = sketch_tensors(workloads.sketch_matrices(p.n, 3, q))
    X = tp.Tensor(3, p.n, cap, prec)
    st, info = ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=tau, kmax=100, trunc_tol=eps, cap=cap,
                             sketch=sk, stop_rule=TP_STOP_RESIDUAL, recursive_residual=True)
    core, fs = X.numpy_parts()
    err = global_rel_error(p, core, fs, stride=8)
    log("  err %.2e info %s" % (err, info))
    assert info["status"] in (0, 4)
    assert err < tol


@pytest.mark.parametrize("prec", [0, 1])
def test_state_recovery_and_cost(ctx, prec):
    """y = beta A^-alpha u (eqn:State) and J(y,u) = 1/2||y - y_Omega||^2 + gamma/2 ||u||^2 from the
    GPU control, against the exact state and cost of the exact control."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    n, beta, gamma, alpha = 63, 2.0, 1e-2, 0.5
    p = workloads.cfg2(alpha=alpha, gamma=gamma, n=n)
    p.c_neg, p.c_pos = beta, gamma / beta          # paper form of eqn:forControl
    log("state/cost prec=%d" % prec)
    eps = 1e-7 if prec == 0 else 1e-5
    X, st, info = solve(ctx, p, prec, eps=eps, tau=4 * eps, pre_terms=36 if prec == 0 else 28)
    state, serr = ctx.state_symbol_build(3, n, alpha, beta, prec=prec, terms=36 if prec == 0 else 28)
    sk = sketch_tensors(workloads.sketch_matrices(n, 3, 63))
    Y = tp.Tensor(3, n, 64, prec)
    ctx.apply(state, X, Y, eps, 64, sk, allow_erank=True)
    f = tensor.cp_full(p.weights, p.factors)
    u = exact.solve_full(f, alpha, p.c_neg, p.c_pos)
    y = exact.state_full(u, alpha, beta)
    err_y = rel(ctx.eval_grid(Y, [np.arange(n)] * 3), y)
    B = tp.Tensor(3, n, 64, prec)
    ctx.from_cp(p.weights, p.factors, B)
    J = 0.5 * (ctx.inner(Y, Y) - 2 * ctx.inner(Y, B) + ctx.inner(B, B)) + 0.5 * gamma * ctx.inner(X, X)
    J_ref = exact.cost_functional(y, u, f, gamma)
    log("  state err %.2e (sym %.1e)  J %.10e ref %.10e" % (err_y, serr, J, J_ref))
    tol = FP64_TOL if prec == 0 else MIXED_TOL
    assert err_y < tol
    assert abs(J - J_ref) <= tol * abs(J_ref)


@pytest.mark.parametrize("prec", [1, 0])
def test_cfg3_n2047_spectral_domain(ctx, prec):
    """The benchmark workload with the iteration in sine coordinates (spectral_domain): the same
    error bound against the oracle (Parseval over every 8th spectral slab of the 2047^3 grid), and
    the result equal to the standard path's up to the truncation tolerance (the two differ only in
    rounding and in where the transforms sit)."""
    p = workloads.cfg3()
    log("cfg3 spectral domain prec=%d" % prec)
    kw = (dict(eps=3e-5, tau=1.2e-4, cap=56, q=64, op_terms=28, pre_terms=28) if prec == 1 else
          dict(eps=1.5e-7, tau=6e-7, cap=96, q=112, op_terms=36, pre_terms=36))
    Xs, st, info = solve(ctx, p, prec, spectral=True, **kw)
    X0, st0, info0 = solve(ctx, p, prec, **kw)
    core, fs = Xs.numpy_parts()
    err = global_rel_error(p, core, fs, stride=8)   # every 8th spectral slab
    rows = [np.arange(0, p.n, 64)] * 3
    d = rel(ctx.eval_grid(Xs, rows), ctx.eval_grid(X0, rows))
    log("  global err %.2e, vs standard path %.2e; info %s / %s" % (err, d, info, info0))
    assert info["iters"] == info0["iters"]
    assert err < (MIXED_TOL if prec == 1 else FP64_TOL)
    assert d < (3 * kw["eps"])
    assert abs(info["true_rel_res"] - info0["true_rel_res"]) <= 0.05 * info0["true_rel_res"] + 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_spectral_domain_2d_against_oracle(ctx, prec):
    p = workloads.cfg1()
    log("cfg1 spectral domain prec=%d" % prec)
    X, st, info = solve(ctx, p, prec, eps=1e-8 if prec == 0 else 1e-6, tau=4e-8 if prec == 0 else 4e-6,
                        op_terms=40 if prec == 0 else 32, pre_terms=36, spectral=True)
    u = exact.solve_full(tensor.cp_full(p.weights, p.factors), p.alpha, p.c_neg, p.c_pos)
    err = rel(ctx.eval_grid(X, [np.arange(p.n)] * 2), u)
    log("  err %.2e info %s" % (err, info))
    assert err < (FP64_TOL if prec == 0 else MIXED_TOL)


@pytest.mark.parametrize("seed", [4, 10, 12])
def test_cfg3_shape_other_right_hand_sides(ctx, seed):
    """The benchmark's mixed settings on other right-hand sides of the same shape (the three of
    seeds 3-17 that are hardest for them): one PCG iteration and the error within 1e-4
    (Parseval over every 16th spectral slab)."""
    p = workloads.cfg3(seed=seed)
    log("cfg3 shape seed=%d mixed" % seed)
    X, st, info = solve(ctx, p, 1, eps=3e-5, tau=1.2e-4, cap=56, q=64, op_terms=28, pre_terms=28)
    core, fs = X.numpy_parts()
    err = global_rel_error(p, core, fs, stride=16)
    log("  err %.2e info %s" % (err, info))
    assert info["iters"] == 1
    assert err < MIXED_TOL
