"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types an oracle formula: each compares an oracle routine with an
independent route (a library eigensolver, a dense brute force, a closed form,
a 50-digit evaluation, an error bound, an exact rank)."""
import math
import os

import numpy as np
import pytest
import scipy.fft as sfft
import scipy.linalg as sla

import workloads
from oracle import exact, expfit, lowrank_pcg, sinc, spectral, tensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


# ---------------------------------------------------------------- spectra (Sec. 3.2)
@pytest.mark.parametrize("n", [1, 2, 7, 63, 255])
def test_eigenvalues_match_tridiagonal_eigensolver(n):
    h = 1.0 / (n + 1)
    ev = sla.eigh_tridiagonal(np.full(n, 2.0 / h**2), np.full(n - 1, -1.0 / h**2),
                              eigvals_only=True) if n > 1 else np.array([2.0 / h**2])
    lam = spectral.eigenvalues(n)
    np.testing.assert_allclose(lam, np.sort(ev), rtol=1e-12, atol=1e-13 * lam.max() * n)


@pytest.mark.parametrize("n", [7, 31, 63])
def test_dst_matrix_diagonalises_laplacian(n):
    F = spectral.dst_matrix(n)
    np.testing.assert_allclose(F @ F, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(F, F.T, atol=0)
    D = F @ spectral.laplacian_1d(n) @ F
    np.testing.assert_allclose(np.diag(D), spectral.eigenvalues(n), rtol=1e-12)
    off = D - np.diag(np.diag(D))
    assert np.abs(off).max() < 1e-10 * spectral.eigenvalues(n).max()


@pytest.mark.parametrize("n", [1, 15, 63, 127])
def test_dst_definition_matches_library_dst(n):
    x = np.random.default_rng(n).standard_normal((n, 3))
    np.testing.assert_allclose(spectral.dst(x), sfft.dst(x, type=1, norm="ortho", axis=0),
                               atol=1e-12)


def test_worked_single_mode_values_golden():
    g = _golden("cfg1_sine_mode.txt")
    lam = spectral.eigenvalues(63)
    assert lam[2] == pytest.approx(g["lambda_3"], rel=1e-14)
    assert lam[4] == pytest.approx(g["lambda_5"], rel=1e-14)
    rho = lam[2] + lam[4]
    assert rho == pytest.approx(g["rho"], rel=1e-14)
    assert spectral.symbol(rho, 0.5, 1.0, 1e-2) == pytest.approx(g["s_paper"], rel=1e-13)
    assert spectral.symbol(rho, 0.5, 1e-2, 1.0) == pytest.approx(g["s_literal"], rel=1e-13)


def test_single_mode_solution_closed_form_2d():
    """f = sin(3 pi x) sin(5 pi y) is an eigenvector of A: u = f / s exactly."""
    g = _golden("cfg1_sine_mode.txt")
    p = workloads.sine_mode_problem(63, 2, (3, 5), 0.5, 1.0, 1e-2)
    f = tensor.cp_full(p.weights, p.factors)
    u = exact.solve_full(f, p.alpha, p.c_neg, p.c_pos)
    np.testing.assert_allclose(u, g["u_over_f_paper"] * f, atol=1e-12)
    u2 = exact.solve_full(f, 0.5, 1e-2, 1.0)
    np.testing.assert_allclose(u2, g["u_over_f_literal"] * f, atol=1e-13)


@pytest.mark.parametrize("ns,ks", [((2047, 2047, 2047), (1, 2, 3)), ((255, 255, 255), (17, 200, 5))])
def test_single_mode_factor_any_n(ns, ks):
    """The closed form at large n is checked against the 1D eigen-relation directly."""
    fac = exact.single_mode_factor(ns, ks, 0.5, 1.0, 1e-2)
    rho = 0.0
    for n, k in zip(ns, ks):
        v = exact.sine_mode(n, k)
        Av = spectral.laplacian_1d(n) @ v if n <= 300 else None
        lam = spectral.eigenvalues(n)[k - 1]
        if Av is not None:
            np.testing.assert_allclose(Av, lam * v, atol=1e-7 * lam)
        rho += lam
    assert fac == pytest.approx(1.0 / (rho ** -0.5 + 1e-2 * rho ** 0.5), rel=1e-14)


# ---------------------------------------------------------------- O1 vs brute force
@pytest.mark.parametrize("d,n,alpha,cn,cp", [(3, 7, 0.5, 1.0, 1e-2), (3, 11, 0.25, 1.0, 1e-3),
                                             (2, 31, 0.75, 1.0, 1e-1), (2, 15, 1.0, 1.0, 1e-2),
                                             (3, 5, 0.1, 1e-2, 1.0)])
def test_full_solve_equals_dense_brute_force(d, n, alpha, cn, cp):
    f = np.random.default_rng(n * d).standard_normal((n,) * d)
    u = exact.solve_full(f, alpha, cn, cp)
    ub = exact.brute_force(f, alpha, cn, cp)
    assert np.linalg.norm(u - ub) <= 1e-11 * np.linalg.norm(ub)
    # and it inverts apply_full
    np.testing.assert_allclose(exact.apply_full(u, alpha, cn, cp), f, atol=1e-10)


def test_full_solve_symmetric_and_linear():
    rng = np.random.default_rng(5)
    f, g = rng.standard_normal((2, 15, 15, 15))
    uf = exact.solve_full(f, 0.5, 1.0, 1e-2)
    ug = exact.solve_full(g, 0.5, 1.0, 1e-2)
    assert abs(np.sum(uf * g) - np.sum(f * ug)) < 1e-12 * np.linalg.norm(uf) * np.linalg.norm(g)
    np.testing.assert_allclose(exact.solve_full(2 * f - g, 0.5, 1.0, 1e-2), 2 * uf - ug, atol=1e-12)


def test_restricted_solve_equals_full_solve():
    p = workloads.cfg2(alpha=0.5, gamma=1e-2, n=63)
    f = tensor.cp_full(p.weights, p.factors)
    u = exact.solve_full(f, p.alpha, p.c_neg, p.c_pos)
    rows = [workloads.restriction_rows(63, 8)] * 3
    ur = exact.solve_cp_restricted(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos, rows)
    np.testing.assert_allclose(ur, u[np.ix_(*rows)], atol=1e-12 * np.abs(u).max())
    half = exact.solve_cp_restricted_slabs(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos,
                                           rows, range(0, 63, 2))
    rest = exact.solve_cp_restricted_slabs(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos,
                                           rows, range(1, 63, 2))
    np.testing.assert_allclose(half + rest, ur, atol=1e-12 * np.abs(u).max())


# ---------------------------------------------------------------- sinc (Sec. 2, Sec. 4.2)
@pytest.mark.parametrize("mu", [0.25, 0.5, 0.75, 1.5])
def test_sinc_expsum_converges_to_power(mu):
    """Direct rho^-mu against the sinc sum on a dense log grid; the error must fall
    as the rule is refined (hh = c pi / sqrt(M), M growing)."""
    B = 1.7e6
    rho = np.exp(np.linspace(0, np.log(B), 3000))
    errs = []
    for M in (20, 60, 160):
        hh = sinc.paper_step(M, 1.6)
        t, c = sinc.laplace_nodes(mu, int(3 * M), M, hh)
        errs.append(np.max(np.abs(sinc.expsum(rho, t, c) * rho**mu - 1)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-5


def test_sinc_weights_integrate_gamma_density():
    """sum_k c_k exp(-t_k) ~ 1 (rho = 1) and sum_k c_k t_k exp(-t_k rho) ~ mu rho^-(mu+1)."""
    t, c = sinc.laplace_nodes(0.5, 800, 300, 0.12)
    assert sinc.expsum(1.0, t, c) == pytest.approx(1.0, rel=1e-9)
    rho = 7.0
    assert float(np.sum(c * t * np.exp(-t * rho))) == pytest.approx(0.5 * rho ** -1.5, rel=1e-8)


@pytest.mark.parametrize("alpha,cn,cp", [(0.5, 1.0, 1e-2), (0.25, 1.0, 1e-1), (1.0, 1.0, 1e-2)])
def test_sinc_g_times_rho_is_symbol(alpha, cn, cp):
    """Lemma 4.1 reading: rho * g(rho) = s(rho) on the attained rho range."""
    n, d = 255, 3
    lam = spectral.eigenvalues(n)
    rho0 = d * lam[0]
    tau, w = sinc.g_nodes(alpha, cn, cp, rho0, 800, 300, 0.12)
    rho = np.exp(np.linspace(np.log(rho0), np.log(d * lam[-1]), 2000))
    s = spectral.symbol(rho, alpha, cn, cp)
    assert np.max(np.abs(rho * sinc.expsum(rho, tau, w) / s - 1)) < 1e-12


# ---------------------------------------------------------------- expfit
@pytest.mark.parametrize("K,tol", [(24, 2e-4), (32, 5e-6)])
def test_expfit_power_accuracy(K, tol):
    B = 1.7e6
    t = expfit.geometric_exponents(B, K, -1.0, 2.25)
    f = lambda y: y ** -0.5
    w = expfit.fit_weights(f, t, B, 1500)
    err = expfit.max_rel_error(f, t, w, B)
    assert err < tol
    # the fit beats the sinc rule with the same number of terms
    hh = sinc.paper_step(K, 1.0)
    ts, cs = sinc.laplace_nodes(0.5, K - 8, 7, hh)
    y = expfit.log_samples(B, 5000)
    assert np.max(np.abs(sinc.expsum(y, ts, cs) * y**0.5 - 1)) > err


def test_expfit_preconditioner_positive_and_close():
    n, d, alpha, cn, cp = 255, 3, 0.5, 1.0, 1e-2
    lam = spectral.eigenvalues(n)
    rho0 = d * lam[0]
    B = lam[-1] / lam[0]
    s = lambda y: spectral.symbol(rho0 * y, alpha, cn, cp)
    t = expfit.geometric_exponents(B, 12, -2.75, 0.5)
    w = expfit.fit_weights(lambda y: 1.0 / s(y), t, B, 1500)
    rho = spectral.rho_grid((n, n, n))[::8, ::8, ::8] / rho0
    p = sinc.expsum(rho, t, w)
    assert p.min() > 0
    assert np.max(np.abs(p * s(rho) - 1)) < 5e-3


# ---------------------------------------------------------------- tensor formats (Sec. 5)
def test_laplacian_core_has_exact_tucker_rank_2_and_cp_rank_3():
    """g(i,j,k) = lambda_i + lambda_j + lambda_k has canonical rank 3 and every mode
    unfolding has rank 2 (span{lambda, 1}) (Sec. 4.1)."""
    lam = spectral.eigenvalues(31)
    G = spectral.rho_grid((31, 31, 31))
    one = np.ones(31)
    Gcp = tensor.cp_full(np.ones(3), [np.column_stack([lam, one, one]),
                                      np.column_stack([one, lam, one]),
                                      np.column_stack([one, one, lam])])
    np.testing.assert_allclose(Gcp, G, rtol=1e-14)
    core, U, ranks = tensor.hosvd_truncate(G, 1e-12)
    assert ranks == [2, 2, 2]
    assert np.linalg.norm(tensor.tucker_full(core, U) - G) < 1e-12 * np.linalg.norm(G)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_hosvd_error_bound_and_random_lowrank_recovery(eps):
    rng = np.random.default_rng(7)
    A = tensor.tucker_full(rng.standard_normal((4, 5, 3)),
                           [np.linalg.qr(rng.standard_normal((20, r)))[0] for r in (4, 5, 3)])
    T = A + 1e-9 * rng.standard_normal(A.shape)
    core, U, ranks = tensor.hosvd_truncate(T, eps)
    err = np.linalg.norm(tensor.tucker_full(core, U) - T)
    assert err <= eps * np.linalg.norm(T)
    assert ranks == [4, 5, 3]
    # a random full tensor keeps most of its rank at tight eps
    R = rng.standard_normal((9, 9, 9))
    core, U, ranks = tensor.hosvd_truncate(R, eps)
    assert np.linalg.norm(tensor.tucker_full(core, U) - R) <= eps * np.linalg.norm(R)


def test_cp_inner_product_matches_gram_formula():
    """<X,Y> = xi^T (Hadamard of per-mode Grams) eta (Sec. 5, CP algebra)."""
    rng = np.random.default_rng(3)
    Fx = [rng.standard_normal((9, 3)) for _ in range(3)]
    Fy = [rng.standard_normal((9, 4)) for _ in range(3)]
    wx, wy = rng.standard_normal(3), rng.standard_normal(4)
    G = np.ones((3, 4))
    for a, b in zip(Fx, Fy):
        G = G * (a.T @ b)
    assert tensor.inner(tensor.cp_full(wx, Fx), tensor.cp_full(wy, Fy)) == pytest.approx(wx @ G @ wy, rel=1e-12)


# ---------------------------------------------------------------- Algorithm alg:pcg step model
def test_lowrank_pcg_step_model_converges_to_exact_solution():
    n, d, alpha, cn, cp = 15, 3, 0.5, 1.0, 1e-2
    p = workloads.cfg2(alpha=alpha, gamma=cp, n=n)
    f = tensor.cp_full(p.weights, p.factors)
    u = exact.solve_full(f, alpha, cn, cp)
    s = spectral.symbol(spectral.rho_grid((n,) * d), alpha, cn, cp)
    pre = 1.0 / s * (1 + 0.05 * np.cos(np.arange(n ** d)).reshape((n,) * d))  # inexact SPD precond
    X, it, hist = lowrank_pcg.pcg(s, pre, f, eps=1e-10, tau=1e-9)
    assert it < 15
    assert np.linalg.norm(X - u) <= 1e-8 * np.linalg.norm(u)
    # an exact preconditioner converges in one step (first iterate is A_2^-1 B)
    X1, it1, _ = lowrank_pcg.pcg(s, 1.0 / s, f, eps=1e-12, tau=1e-9)
    assert it1 == 1
    assert np.linalg.norm(X1 - u) <= 1e-10 * np.linalg.norm(u)


def test_tucker_error_by_parseval_matches_full_grid():
    """The slab-wise spectral error equals the full-grid relative error of a Tucker tensor."""
    p = workloads.cfg3(n=31)
    f = tensor.cp_full(p.weights, p.factors)
    u = exact.solve_full(f, p.alpha, p.c_neg, p.c_pos)
    core, U, _ = tensor.hosvd_truncate(u, 1e-3)
    X = tensor.tucker_full(core, U)
    e2, u2 = exact.tucker_error_slabs(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos, core, U, range(31))
    assert np.sqrt(e2 / u2) == pytest.approx(np.linalg.norm(X - u) / np.linalg.norm(u), rel=1e-9)
    assert u2 == pytest.approx(np.sum(u * u), rel=1e-12)
    a, b = exact.tucker_error_slabs(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos, core, U, range(0, 31, 2))
    c2, d2 = exact.tucker_error_slabs(p.weights, p.factors, p.alpha, p.c_neg, p.c_pos, core, U, range(1, 31, 2))
    assert a + c2 == pytest.approx(e2, rel=1e-12)


# --- the preconditioning tests of Sec. 6: A^alpha x = b, (I + A^{2 alpha}) x = b, (A^alpha + A^-alpha) x = b

PRECOND_EQS = {  # name: (c_neg, c_pos, c0, beta as a multiple of alpha)
    "A^a": (0.0, 1.0, 0.0, 1.0),
    "I+A^2a": (0.0, 1.0, 1.0, 2.0),
    "A^a+A^-a": (1.0, 1.0, 0.0, 1.0),
}


@pytest.mark.parametrize("eq", sorted(PRECOND_EQS))
@pytest.mark.parametrize("alpha", [0.5, 0.1])
@pytest.mark.parametrize("shape", [(7, 9), (5, 4, 3)])
def test_general_symbol_solve_matches_brute_force(eq, alpha, shape):
    """The sine-transform solve with the general symbol equals the dense eigendecomposition route."""
    cn, cp, c0, bm = PRECOND_EQS[eq]
    f = np.random.default_rng(11).standard_normal(shape)
    u = exact.solve_full(f, alpha, cn, cp, c0, bm * alpha)
    v = exact.brute_force(f, alpha, cn, cp, c0, bm * alpha)
    assert np.linalg.norm(u - v) <= 1e-11 * np.linalg.norm(v)


@pytest.mark.parametrize("shape", [(7, 9), (5, 4, 3)])
def test_identity_plus_laplacian_without_fractional_powers(shape):
    """alpha = 1/2 in (I + A^{2 alpha}) x = b is (I + A) x = b: a plain sparse solve, no
    eigendecomposition, no sine transform."""
    f = np.random.default_rng(12).standard_normal(shape)
    A = exact.laplacian_full(shape)
    x = np.linalg.solve(np.eye(A.shape[0]) + A, f.ravel()).reshape(shape)
    u = exact.solve_full(f, 0.5, 0.0, 1.0, 1.0, 1.0)
    assert np.linalg.norm(u - x) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("shape", [(7, 9), (5, 4, 3)])
def test_half_power_applied_twice_is_the_laplacian(shape):
    """Solving A^{1/2} y = b and then A^{1/2} x = y gives A x = b (dense solve of A)."""
    f = np.random.default_rng(13).standard_normal(shape)
    y = exact.solve_full(f, 0.5, 0.0, 1.0)
    x = exact.solve_full(y, 0.5, 0.0, 1.0)
    A = exact.laplacian_full(shape)
    ref = np.linalg.solve(A, f.ravel()).reshape(shape)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


# ---------------------------------------------------------------- rank-r preconditioner (Sec. 6)
@pytest.mark.parametrize("eq", sorted(PRECOND_EQS))
@pytest.mark.parametrize("r", [1, 3, 6])
def test_rank_r_preconditioner_2d_is_the_best_rank_r_matrix(eq, r):
    """2D: the truncated HOSVD of the symmetric matrix P = 1/s(lambda_i + lambda_j) is its best
    rank-r approximation, so its Frobenius error is the tail of the eigenvalue magnitudes
    (Eckart-Young), taken here from a symmetric eigensolver rather than an SVD."""
    cn, cp, c0, bm = PRECOND_EQS[eq]
    n, alpha = 40, 0.5
    P = 1.0 / spectral.symbol(spectral.rho_grid((n, n)), alpha, cn, cp, c0, bm * alpha)
    Pr = exact.precond_rank_r((n, n), r, alpha, cn, cp, c0, bm * alpha)
    lam = np.sort(np.abs(np.linalg.eigvalsh(P)))[::-1]
    want = np.sqrt(np.sum(lam[r:] ** 2))
    assert abs(np.linalg.norm(P - Pr) - want) <= 1e-10 * np.linalg.norm(P) + 1e-6 * want
    assert np.linalg.matrix_rank(Pr, tol=1e-12 * np.linalg.norm(P)) == r
    assert np.allclose(Pr, Pr.T, atol=1e-13 * np.abs(P).max())


@pytest.mark.parametrize("r", [2, 4])
def test_rank_r_preconditioner_3d_within_hosvd_bounds(r):
    """3D: the HOSVD truncation error lies between the largest and the sum of the discarded mode
    singular-value tails (the quasi-optimality bounds of the HOSVD)."""
    ns, alpha = (12, 10, 9), 0.1
    P = 1.0 / spectral.symbol(spectral.rho_grid(ns), alpha, 1.0, 1.0, 0.0, alpha)
    Pr = exact.precond_rank_r(ns, r, alpha, 1.0, 1.0, 0.0, alpha)
    tails = []
    for l in range(3):
        M = np.moveaxis(P, l, 0).reshape(ns[l], -1)
        ev = np.sort(np.linalg.eigvalsh(M @ M.T))[::-1]
        tails.append(np.sum(np.clip(ev[r:], 0, None)))
    e2 = np.linalg.norm(P - Pr) ** 2
    assert max(tails) * (1 - 1e-9) <= e2 <= sum(tails) * (1 + 1e-9)


def test_rank_r_preconditioner_full_rank_is_exact():
    """r at least the grid size: nothing is discarded, the inverse symbol is returned."""
    ns = (6, 5, 4)
    P = 1.0 / spectral.symbol(spectral.rho_grid(ns), 0.5, 0.0, 1.0, 1.0, 1.0)
    assert np.abs(exact.precond_rank_r(ns, 6, 0.5, 0.0, 1.0, 1.0, 1.0) - P).max() <= 1e-13 * P.max()


# ------------------------------------------------- directionally fractional Laplacian (Sec. 4.1)
@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.9])
@pytest.mark.parametrize("shape", [(7, 9), (5, 4, 3)])
def test_directional_solve_matches_dense_powers(alpha, shape):
    """The sine-transform solve with rho' = sum_l lambda^alpha equals the dense route that takes
    fractional powers of each 1D matrix by its own eigendecomposition."""
    f = np.random.default_rng(13).standard_normal(shape)
    u = exact.solve_directional(f, alpha, 1.0, 0.3)
    v = exact.brute_force_directional(f, alpha, 1.0, 0.3)
    assert np.linalg.norm(u - v) <= 1e-11 * np.linalg.norm(v)


@pytest.mark.parametrize("shape", [(7, 9), (5, 4, 3)])
def test_directional_at_alpha_one_is_the_laplacian(shape):
    """alpha = 1: sum_l (-Delta_l) is the Laplacian, and the directional control equation is the
    ordinary one with alpha = 1 (checked through the dense Laplacian, no fractional power)."""
    f = np.random.default_rng(14).standard_normal(shape)
    u = exact.solve_directional(f, 1.0, 1.0, 0.3, c0=0.5)
    A = exact.laplacian_full(shape)
    N = A.shape[0]
    v = np.linalg.solve(0.5 * np.eye(N) + np.linalg.inv(A) + 0.3 * A, f.reshape(N)).reshape(shape)
    assert np.linalg.norm(u - v) <= 1e-11 * np.linalg.norm(v)


def test_directional_differs_from_the_fractional_laplacian():
    """For alpha < 1 the two operators differ (sum of powers is not the power of the sum):
    (lambda_1 + lambda_2)^alpha < lambda_1^alpha + lambda_2^alpha."""
    rp = spectral.rho_directional((5, 6), 0.5)
    r = spectral.rho_grid((5, 6)) ** 0.5
    assert np.all(r < rp)


# ---------------------------------------------------------------- golden file and its generator
def test_golden_sine_mode_file_is_what_its_generator_writes():
    """The stored worked example is the committed 50-digit script's output, byte for byte."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_cfg1_sine_mode",
                                                  os.path.join(GOLDEN, "make_cfg1_sine_mode.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(GOLDEN, "cfg1_sine_mode.txt")) as fh:
        assert fh.read() == mod.render()


# ---------------------------------------------------------------- state and cost (Sec. 3.1)
def _control_problem(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape)


@pytest.mark.parametrize("shape,alpha", [((9, 7), 0.5), ((5, 4, 6), 0.3), ((6, 6, 5), 0.8)])
def test_state_matches_dense_fractional_power(shape, alpha):
    """y = beta A^-alpha u (eqn:State) against the dense Kronecker-sum Laplacian, whose
    eigenpairs come from numpy.linalg.eigh (no sine transform)."""
    beta = 1.7
    u = _control_problem(shape, 11)
    A = exact.laplacian_full(shape)
    lam, Q = np.linalg.eigh(A)
    y_ref = ((Q * (beta * lam ** (-alpha))) @ Q.T @ u.reshape(-1)).reshape(shape)
    np.testing.assert_allclose(exact.state_full(u, alpha, beta), y_ref, rtol=1e-11,
                               atol=1e-12 * np.abs(y_ref).max())


@pytest.mark.parametrize("shape,alpha,beta,gamma", [((9, 7), 0.5, 2.0, 0.3), ((5, 4, 6), 0.3, 0.6, 1e-2),
                                                    ((6, 6, 5), 0.75, 1.5, 1e-3)])
def test_exact_control_minimises_the_cost(shape, alpha, beta, gamma):
    """The exact control u* = (beta A^-alpha + (gamma/beta) A^alpha)^-1 y_Omega (eqn:forControl) is
    the minimiser of the reduced cost j(u) = J(y(u), u) with the state y(u) = beta A^-alpha u
    (eqn:State) and J = 1/2 ||y - y_Omega||^2 + gamma/2 ||u||^2 (Sec. 3.1).  j is quadratic, so
    for every direction v and step t:  j(u* + t v) - j(u*) = t^2/2 (||y(v)||^2 + gamma ||v||^2)
    exactly (the linear term vanishes only at the minimiser).  beta != 1 separates the paper's
    form from the others: a state without beta, the cost with gamma/beta, or the coefficients
    swapped each leave a linear term and fail."""
    y_om = _control_problem(shape, 5)
    u = exact.solve_full(y_om, alpha, beta, gamma / beta)

    def j(v):
        return exact.cost_functional(exact.state_full(v, alpha, beta), v, y_om, gamma)

    j0 = j(u)
    rng = np.random.default_rng(7)
    for _ in range(4):
        v = rng.standard_normal(shape)
        yv = exact.state_full(v, alpha, beta)
        curv = float(np.sum(yv * yv)) + gamma * float(np.sum(v * v))
        for t in (1e-3, 0.1, 1.0, -0.5):
            inc = j(u + t * v) - j0
            assert inc > 0
            assert inc == pytest.approx(0.5 * t * t * curv, rel=1e-6, abs=1e-9 * abs(j0))


def test_cost_stationarity_fails_for_the_other_operator_forms():
    """Planted mistakes: the controls of the literal form (beta A^alpha + gamma A^-alpha), of the
    form without the 1/beta, and of a sign-flipped power are not minimisers of the same cost,
    so the exact identity above rejects them."""
    shape, alpha, beta, gamma = (8, 7), 0.5, 2.0, 0.3
    y_om = _control_problem(shape, 5)
    wrong = [exact.solve_full(y_om, alpha, gamma, beta),          # literal spec form
             exact.solve_full(y_om, alpha, beta, gamma),          # gamma instead of gamma/beta
             exact.solve_full(y_om, -alpha, beta, gamma / beta)]  # rho^+alpha in the state term
    v = np.random.default_rng(3).standard_normal(shape)
    yv = exact.state_full(v, alpha, beta)
    curv = float(np.sum(yv * yv)) + gamma * float(np.sum(v * v))
    for u in wrong:
        def j(w):
            return exact.cost_functional(exact.state_full(w, alpha, beta), w, y_om, gamma)
        t = 1e-2
        inc = j(u + t * v) - j(u)
        assert abs(inc - 0.5 * t * t * curv) > 1e-3 * abs(inc)
