"""Edge cases of the GPU path through the C ABI: grids of different size per mode, a zero
right-hand side, indices outside the grid, the largest rank cap and sketch width, and argument
checks on a live context (every rejection happens on the host, before device work)."""
import numpy as np
import pytest

import workloads
from oracle import exact, spectral, tensor
from tests.gpu_helpers import log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=4 << 30)
    yield c
    c.close()


def _solve(ctx, ns, F, w, prec, eps, tau, cap, q, alpha=0.5, cn=1.0, cp=1e-2, op_terms=40, pre_terms=28):
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    d = len(ns)
    op, pre, errs = ctx.symbol_build(d, ns, alpha, cn, cp, prec=prec, op_terms=op_terms, pre_terms=pre_terms)
    X = tp.Tensor(d, ns, cap, prec)
    sk = sketch_tensors(workloads.sketch_matrices(ns, d, q))
    st, info = ctx.pcg_solve(op, pre, w, F, X, tau=tau, kmax=100, trunc_tol=eps, cap=cap, sketch=sk)
    return X, info


@pytest.mark.parametrize("ns,prec", [((31, 63, 127), 0), ((127, 255), 0), ((255, 15, 63), 1), ((1, 7, 3), 0)])
def test_grids_of_different_size_per_mode(ctx, ns, prec):
    """Each mode its own n (its own eigenvalues, sine transform length and factor height), the
    smallest grids (n = 1, 3) included: the whole grid against O1."""
    d = len(ns)
    rng = np.random.default_rng(31)
    F = [rng.standard_normal((n, 2)) for n in ns]
    w = np.ones(2)
    log("grid %s prec=%d" % (ns, prec))
    eps, tau = (1e-9, 3e-8) if prec == 0 else (1e-5, 4e-5)
    X, info = _solve(ctx, ns, F, w, prec, eps, tau, cap=48, q=64)
    u = exact.solve_full(tensor.cp_full(w, F), 0.5, 1.0, 1e-2)
    err = rel(ctx.eval_grid(X, [np.arange(n) for n in ns]), u)
    log("  err %.2e info %s" % (err, info))
    assert info["status"] in (0, 4)
    assert all(r <= min(n, 48) for r, n in zip(info["rank"], ns))
    assert err < (1e-6 if prec == 0 else 1e-4)


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_right_hand_side(ctx, prec):
    """b = 0: the solve returns X = 0 (all ranks 0) without iterating, and evaluates to zeros."""
    n, d = 63, 3
    F = [np.zeros((n, 1)) for _ in range(d)]
    X, info = _solve(ctx, (n,) * d, F, np.zeros(1), prec, 1e-6, 4e-6, cap=16, q=32)
    log("zero rhs prec=%d: %s" % (prec, info))
    assert info["status"] == 0 and info["iters"] == 0 and info["rank"] == [0, 0, 0]
    assert np.all(ctx.eval_grid(X, [np.arange(0, n, 7)] * d) == 0.0)


def test_indices_outside_the_grid_give_nan(ctx):
    """tp_eval_grid and tp_symbol_eval bound every index they read with: points with an index
    outside [0, n) are NaN, the others are unchanged."""
    n, d = 63, 3
    rng = np.random.default_rng(32)
    F = [rng.standard_normal((n, 1)) for _ in range(d)]
    X, info = _solve(ctx, (n,) * d, F, np.ones(1), 0, 1e-9, 3e-8, cap=32, q=48)
    rows = [np.array([0, 5, n, -1]), np.array([1, 2]), np.array([3])]
    v = ctx.eval_grid(X, rows)
    ref = ctx.eval_grid(X, [np.array([0, 5]), np.array([1, 2]), np.array([3])])
    assert np.all(np.isnan(v[2:])) and np.array_equal(v[:2], ref)
    op, pre, _ = ctx.symbol_build(d, n, 0.5, 1.0, 1e-2, prec=0, op_terms=32, pre_terms=12)
    pre_r, _ = ctx.symbol_build(d, n, 0.5, 1.0, 1e-2, prec=0, op_terms=32, pre_terms=28, pre_rank=3)[1:]
    idx = np.array([[0, 0, 0], [n, 0, 0], [0, -1, 0], [0, 0, n + 5], [n - 1, n - 1, n - 1]])
    for sym in (op, pre, pre_r):
        s = sym.eval(idx)
        assert np.all(np.isnan(s[1:4])) and np.all(np.isfinite(s[[0, 4]]))
    lam = spectral.eigenvalues(n)
    rho = lam[[0, n - 1]] * 3
    so = op.eval(idx[[0, 4]])
    assert np.abs(so / spectral.symbol(rho, 0.5, 1.0, 1e-2) - 1).max() < 1e-4


def test_largest_cap_and_sketch(ctx):
    """cap = 128 (the largest Tucker rank) with the widest sketch q = 192 on a 2D problem whose
    solution needs more than 128 ranks at eps = 1e-8 (16 Gaussian terms): the ranks stop at the
    cap, the iteration stops at the floor the cap sets (TP_ENOCONV with the best iterate), and the
    error estimate it reports is the true error."""
    n = 511
    rng = np.random.default_rng(33)
    F = [rng.standard_normal((n, 16)) for _ in range(2)]
    w = np.ones(16)
    X, info = _solve(ctx, (n, n), F, w, 0, 1e-8, 4e-8, cap=128, q=192)
    u = exact.solve_full(tensor.cp_full(w, F), 0.5, 1.0, 1e-2)
    err = rel(ctx.eval_grid(X, [np.arange(n)] * 2), u)
    log("cap 128 / q 192: err %.2e info %s" % (err, info))
    assert info["status"] in (0, 3, 4) and max(info["rank"]) <= 128
    if info["status"] == 0:
        assert err < 1e-6
    else:
        assert err < 1e-4 and 0.5 < err / info["err_est"] < 2.0


def test_invalid_arguments_on_a_live_context(ctx):
    """Each invalid request raises with a message; the context keeps working afterwards."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    n, d = 63, 3
    bad_symbols = [dict(alpha=1.5), dict(alpha=0.0), dict(c_neg=-1.0), dict(c_neg=0.0, c_pos=0.0), dict(beta=1.5),
                   dict(c0=-1.0), dict(pre_rank=17), dict(pre_terms=65), dict(op_terms=1),
                   dict(directional=True, beta=0.5), dict(method=1, c0=1.0), dict(n=100), dict(n=0)]
    for bad in bad_symbols:
        kw = dict(n=n, alpha=0.5, c_neg=1.0, c_pos=1e-2)
        kw.update(bad)
        with pytest.raises(tp.TPError) as e:
            ctx.symbol_build(d, kw.pop("n"), kw.pop("alpha"), kw.pop("c_neg"), kw.pop("c_pos"), prec=0, **kw)
        assert e.value.status == tp.TP_EINVAL, bad
    op, pre, _ = ctx.symbol_build(d, n, 0.5, 1.0, 1e-2, prec=0, op_terms=32, pre_terms=12)
    F = [np.ones((n, 1))] * d
    X = tp.Tensor(d, n, 16, 0)
    sk = sketch_tensors(workloads.sketch_matrices(n, d, 32))
    base = dict(tau=1e-6, kmax=100, trunc_tol=1e-8, cap=16, sketch=sk)
    bad_solves = [(op, pre, X, dict(cap=17)), (op, pre, X, dict(cap=0)), (op, pre, X, dict(tau=0.0)),
                  (op, pre, X, dict(kmax=0)), (op, pre, X, dict(stop_rule=2)), (pre, op, X, {}),
                  (op, pre, X, dict(sketch=sketch_tensors(workloads.sketch_matrices(n, d, 1)))),
                  (op, pre, tp.Tensor(d, n, 16, 1), {}), (op, pre, tp.Tensor(d, 127, 16, 0), {})]
    for o, p_, x, bad in bad_solves:
        kw = dict(base)
        kw.update(bad)
        with pytest.raises(tp.TPError) as e:
            ctx.pcg_solve(o, p_, np.ones(1), F, x, allow=(), **kw)
        assert e.value.status == tp.TP_EINVAL, bad
    st, info = ctx.pcg_solve(op, pre, np.ones(1), F, X, **base)
    assert info["status"] in (0, 4)


WS_CASES = [  # (d, n, alpha, settings, symbol extras)
    (3, 2047, 0.5, dict(prec=1, eps=3e-5, tau=1.2e-4, cap=56, q=64, op_terms=28, pre_terms=28), {}),
    (3, 1023, 0.5, dict(prec=0, eps=1.5e-7, tau=6e-7, cap=96, q=112, op_terms=36, pre_terms=36), {}),
    (2, 2047, 0.5, dict(prec=0, eps=1e-9, tau=3e-8, cap=128, q=144, op_terms=40, pre_terms=36), {"pre_rank": 8}),
    (3, 255, 0.1, dict(prec=0, eps=1e-9, tau=3e-8, cap=64, q=80, op_terms=40, pre_terms=28), {"directional": 1}),
]


@pytest.mark.parametrize("case", range(len(WS_CASES)))
def test_workspace_query_covers_the_peak(ctx, case):
    """tp_workspace_query bounds the workspace a symbol build and a solve use (measured high-water
    mark of the context).  It is a worst case with every rank at the cap: where the ranks reach it
    (the benchmark's right-hand side, case 0) it overshoots the peak by less than 8x."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors, workspace_query
    d, n, alpha, s, extra = WS_CASES[case]
    if case == 0:
        p = workloads.cfg3()
        F, w = p.factors, p.weights
    else:
        rng = np.random.default_rng(40 + case)
        F = [rng.standard_normal((n, 4)) / (1.0 + np.arange(n))[:, None] for _ in range(d)]
        w = np.ones(4)
    query = workspace_query(d, n, alpha, s, len(w), **extra)
    big = tp.Context(0, workspace_bytes=max(query, 8 << 30))
    try:
        big.workspace_peak(reset=True)
        kw = dict(extra)
        if "directional" in kw:
            kw["directional"] = True
        op, pre, _ = big.symbol_build(d, n, alpha, 1.0, 1e-2, prec=s["prec"], op_terms=s["op_terms"],
                                      pre_terms=s["pre_terms"], **kw)
        X = tp.Tensor(d, n, s["cap"], s["prec"])
        sk = sketch_tensors(workloads.sketch_matrices(n, d, s["q"]))
        st, info = big.pcg_solve(op, pre, w, F, X, tau=s["tau"], kmax=100, trunc_tol=s["eps"], cap=s["cap"],
                                 sketch=sk)
        peak = big.workspace_peak()
    finally:
        big.close()
    log("workspace case %d: peak %.1f MiB, query %.1f MiB (%.2fx) info %s" % (case, peak / 2**20, query / 2**20,
                                                                          query / peak, info))
    assert peak <= query
    if case == 0:
        assert max(info["rank"]) >= 0.85 * s["cap"] and query <= 8 * peak


def test_solve_in_a_workspace_of_the_queried_size():
    """A context whose workspace is exactly the queried size runs the benchmark's mixed solve."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors, workspace_query
    d, n, alpha, s, _ = WS_CASES[0]
    p = workloads.cfg3()
    q = workspace_query(d, n, alpha, s, len(p.weights))
    c = tp.Context(0, workspace_bytes=q)
    try:
        op, pre, _ = c.symbol_build(d, n, alpha, p.c_neg, p.c_pos, prec=1, op_terms=28, pre_terms=28)
        X = tp.Tensor(d, n, s["cap"], 1)
        st, info = c.pcg_solve(op, pre, p.weights, p.factors, X, tau=s["tau"], kmax=100, trunc_tol=s["eps"],
                               cap=s["cap"], sketch=sketch_tensors(workloads.sketch_matrices(n, d, s["q"])))
    finally:
        c.close()
    log("solve in %.1f MiB: %s" % (q / 2**20, info))
    assert info["status"] in (0, 4) and info["iters"] == 1


@pytest.mark.parametrize("spectral", [False, True])
def test_warm_start(ctx, spectral):
    """X^(0) given (Algorithm alg:pcg's initial guess): from a coarse solution (eps 1e-3) the FP64
    solve reaches O1's solution to 1e-6, and from its own result it stops after one step."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    p = workloads.cfg2(alpha=0.5, gamma=1e-1, n=63)
    op, pre, _ = ctx.symbol_build(3, 63, p.alpha, p.c_neg, p.c_pos, prec=0, op_terms=40, pre_terms=36)
    sk = sketch_tensors(workloads.sketch_matrices(63, 3, 64))
    X = tp.Tensor(3, 63, 48, 0)
    ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=4e-3, kmax=100, trunc_tol=1e-3, cap=48, sketch=sk,
                  spectral_domain=spectral)
    coarse = ctx.eval_grid(X, [np.arange(63)] * 3)
    u = exact.solve_full(tensor.cp_full(p.weights, p.factors), p.alpha, p.c_neg, p.c_pos)
    st, info = ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=4e-8, kmax=100, trunc_tol=1e-8, cap=48,
                             sketch=sk, warm_start=True, spectral_domain=spectral)
    fine = ctx.eval_grid(X, [np.arange(63)] * 3)
    log("warm start spectral=%s: coarse err %.2e, warm err %.2e, %s" % (spectral, rel(coarse, u), rel(fine, u), info))
    assert rel(coarse, u) > 1e-5 and rel(fine, u) < 1e-6
    st, info2 = ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=4e-8, kmax=100, trunc_tol=1e-8, cap=48,
                              sketch=sk, warm_start=True, spectral_domain=spectral)
    assert info2["iters"] <= 1 and rel(ctx.eval_grid(X, [np.arange(63)] * 3), u) < 1e-6
    X.s.rank[0] = 49  # a guess with a rank above the cap is rejected before any device work
    with pytest.raises(tp.TPError):
        ctx.pcg_solve(op, pre, p.weights, p.factors, X, tau=4e-8, kmax=100, trunc_tol=1e-8, cap=48, sketch=sk,
                      warm_start=True, allow=())


def test_symbol_blocks_reused_and_symbol_outlives_its_context():
    """tp_symbol_free hands a symbol's device blocks back to the context that built it: rebuilding
    the same symbols reuses them and gives bitwise the same symbol values and the same solve; a
    build of another size takes new blocks; a symbol freed after its context was destroyed still
    releases its blocks."""
    import paper_1809_01971_amd as tp
    c = tp.Context(0, workspace_bytes=1 << 30)
    ns = (63, 63, 63)
    rng = np.random.default_rng(5)
    idx = rng.integers(0, 63, size=(4096, 3))
    F = [rng.standard_normal((63, 2)) for _ in ns]
    w = np.ones(2)
    vals, xs = [], []
    for _ in range(3):
        op, pre, _ = c.symbol_build(3, ns, 0.5, 1.0, 1e-2, prec=1, op_terms=28, pre_terms=28)
        vals.append((op.eval(idx), pre.eval(idx)))
        X, _ = _solve_with(c, op, pre, ns, F, w)
        core, fac = X.numpy_parts()
        xs.append(tensor.tucker_full(core, fac))
        op.free()
        pre.free()
    for v, x in zip(vals[1:], xs[1:]):
        assert np.array_equal(v[0], vals[0][0]) and np.array_equal(v[1], vals[0][1])
        assert np.array_equal(x, xs[0])
    big, bigpre, _ = c.symbol_build(3, (127, 127, 127), 0.5, 1.0, 1e-2, prec=1, op_terms=28, pre_terms=28)
    small, smallpre, _ = c.symbol_build(3, ns, 0.5, 1.0, 1e-2, prec=1, op_terms=28, pre_terms=28)
    assert np.array_equal(small.eval(idx), vals[0][0])
    c.close()
    for s in (big, bigpre, small, smallpre):
        s.free()


def _solve_with(ctx, op, pre, ns, F, w):
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import sketch_tensors
    X = tp.Tensor(3, ns, 32, 1)
    sk = sketch_tensors(workloads.sketch_matrices(ns, 3, 40))
    st, info = ctx.pcg_solve(op, pre, w, F, X, tau=1e-4, kmax=100, trunc_tol=3e-5, cap=32, sketch=sk)
    return X, info


def test_device_resident_rhs_matches_host_arrays(ctx):
    """A right-hand side copied to the device once (`Rhs`) gives bitwise the same solution as one
    passed as host arrays, in a single solve and in a batch."""
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import batch_solve, sketch_tensors
    ns = (63, 63, 63)
    rng = np.random.default_rng(9)
    F = [rng.standard_normal((63, 3)) for _ in ns]
    w = rng.standard_normal(3)
    op, pre, _ = ctx.symbol_build(3, ns, 0.5, 1.0, 1e-2, prec=1, op_terms=28, pre_terms=28)
    sk = sketch_tensors(workloads.sketch_matrices(ns, 3, 40))
    parts = []
    for rhs in ((w, F), (tp.Rhs(w, F), None)):
        X = tp.Tensor(3, ns, 32, 1)
        ctx.pcg_solve(op, pre, rhs[0], rhs[1], X, tau=1e-4, kmax=100, trunc_tol=3e-5, cap=32, sketch=sk)
        core, fac = X.numpy_parts()
        parts.append(tensor.tucker_full(core, fac))
    assert np.array_equal(parts[0], parts[1])
    p = workloads.cfg3(seed=3)
    p.n = 63
    p.factors = [f[:63] for f in p.factors]
    s = dict(prec=1, eps=3e-5, tau=1e-4, cap=32, q=40, op_terms=28, pre_terms=28)
    skb = {(63, 40): sketch_tensors(workloads.sketch_matrices(63, 3, 40))}
    full = []
    for rhs in (None, [tp.Rhs(p.weights, p.factors)]):
        outs, res = batch_solve(ctx, [p], lambda _: s, skb, streams=1, workspace_per_stream=1 << 30, rhs=rhs)
        core, fac = outs[0].numpy_parts()
        full.append(tensor.tucker_full(core, fac))
    assert np.array_equal(full[0], full[1])


def test_batch_problems_sharing_a_descriptor(ctx):
    """Problems of a batch with equal descriptors share one symbol build: every result equals the
    single solve of the same problem bitwise, next to a problem with another descriptor."""
    import dataclasses
    import paper_1809_01971_amd as tp
    from paper_1809_01971_amd._tp import batch_solve, sketch_tensors
    n = 63
    probs = []
    for seed, alpha in ((3, 0.5), (4, 0.5), (5, 0.3), (6, 0.5)):
        p = workloads.cfg3(seed=seed)
        probs.append(dataclasses.replace(p, n=n, alpha=alpha, factors=[f[:n] for f in p.factors]))
    s = dict(prec=1, eps=3e-5, tau=1e-4, cap=32, q=40, op_terms=28, pre_terms=28)
    sk = {(n, 40): sketch_tensors(workloads.sketch_matrices(n, 3, 40))}
    outs, res = batch_solve(ctx, probs, lambda _: s, sk, streams=2, workspace_per_stream=1 << 30)
    for p, X in zip(probs, outs):
        op, pre, _ = ctx.symbol_build(3, n, p.alpha, p.c_neg, p.c_pos, prec=1, op_terms=28, pre_terms=28)
        Y = tp.Tensor(3, n, 32, 1)
        ctx.pcg_solve(op, pre, p.weights, p.factors, Y, tau=1e-4, kmax=100, trunc_tol=3e-5, cap=32,
                      sketch=sk[(n, 40)])
        a = tensor.tucker_full(*X.numpy_parts())
        b = tensor.tucker_full(*Y.numpy_parts())
        assert np.array_equal(a, b)
