"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds input recipes only (no arithmetic of the solver): right-hand
side factor matrices of the canonical design function y_Omega, problem
parameters, and the Gaussian test matrices that the sketched truncation takes as
an input.  All draws use numpy's PCG64 generator; factor vectors are drawn term
by term and, inside a term, mode by mode.

The paper's own design functions exist only as figures (Sec. 6), so every
workload here is synthetic, with the sizes and parameters of the configurations
below.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One control problem (c_neg A^-alpha + c_pos A^alpha) u = f, f canonical."""
    d: int
    n: int
    alpha: float
    c_neg: float
    c_pos: float
    weights: np.ndarray                      # (R,)
    factors: list = field(default_factory=list)   # d arrays (n, R), column k = term k
    name: str = ""
    c0: float = 0.0         # constant term of the symbol (preconditioning tests)
    beta: float = None      # exponent of the c_pos term; None = alpha


def grid(n):
    """Interior nodes x_i = i/(n+1), i = 1..n."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1.0)


def gaussian_factors(rng, n, d, rank):
    """Term-major draws: for each term, for each mode, n standard normals."""
    F = [np.empty((n, rank)) for _ in range(d)]
    for k in range(rank):
        for l in range(d):
            F[l][:, k] = rng.standard_normal(n)
    return F


def cfg1(seed=0, with_mode=True):
    """2D, n=63 (h=1/64), alpha=1/2, beta=1, gamma=1e-2 (paper form c_neg=1, c_pos=1e-2):
    three rank-1 N(0,1) terms plus the separable sine mode sin(3 pi x) sin(5 pi y)."""
    n, d = 63, 2
    rng = np.random.default_rng(seed)
    F = gaussian_factors(rng, n, d, 3)
    w = np.ones(3)
    if with_mode:
        x = grid(n)
        F = [np.column_stack([F[0], np.sin(3 * np.pi * x)]),
             np.column_stack([F[1], np.sin(5 * np.pi * x)])]
        w = np.ones(4)
    return Problem(d, n, 0.5, 1.0, 1e-2, w, F, "cfg1")


def sine_mode_problem(n, d, ks, alpha, c_neg, c_pos):
    """f = (x)_l sin(k_l pi x): the exact control is f / s(sum_l lambda_{k_l})."""
    x = grid(n)
    F = [np.sin(k * np.pi * x)[:, None] for k in ks]
    return Problem(d, n, alpha, c_neg, c_pos, np.ones(1), F, "sine_mode")


def cfg2(alpha=0.5, gamma=1e-1, seed=1, n=255):
    """3D, n=255, beta=1, alpha in {1/4,1/2,3/4}, gamma in {1e-1,1e-3}; rank 5 N(0,1)."""
    rng = np.random.default_rng(seed)
    F = gaussian_factors(rng, n, 3, 5)
    return Problem(3, n, alpha, 1.0, gamma, np.ones(5), F, "cfg2")


def cfg3(seed=2, n=2047):
    """3D, n=2047, alpha=1/2, beta=1, gamma=1e-2; rank 8; the entry at 0-based grid
    position k of every factor is z/(1+k), z ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    F = gaussian_factors(rng, n, 3, 8)
    scale = 1.0 / (1.0 + np.arange(n, dtype=np.float64))
    F = [f * scale[:, None] for f in F]
    return Problem(3, n, 0.5, 1.0, 1e-2, np.ones(8), F, "cfg3")


def cfg4(count=256, seed=3):
    """Batch of independent 3D problems: n ~ U{127,255,511,1023}, rank ~ U{1..12},
    alpha ~ U[0.1,0.9], beta = 1, gamma = 10^U[-4,-1]; problem draws first, then
    the factor draws problem by problem."""
    rng = np.random.default_rng(seed)
    ns = rng.choice([127, 255, 511, 1023], size=count)
    ranks = rng.integers(1, 13, size=count)
    alphas = rng.uniform(0.1, 0.9, size=count)
    gammas = 10.0 ** rng.uniform(-4, -1, size=count)
    out = []
    for i in range(count):
        F = gaussian_factors(rng, int(ns[i]), 3, int(ranks[i]))
        out.append(Problem(3, int(ns[i]), float(alphas[i]), 1.0, float(gammas[i]),
                           np.ones(int(ranks[i])), F, "cfg4[%d]" % i))
    return out


def cfg5(seed=4, n=32767):
    """3D, n=32767, alpha=0.3, beta=1, gamma=1e-3; rank 10 Gaussian bumps
    exp(-(x-c)^2/0.01) with c ~ U(0.2,0.8) drawn per (term, mode)."""
    rng = np.random.default_rng(seed)
    x = grid(n)
    F = [np.empty((n, 10)) for _ in range(3)]
    for k in range(10):
        for l in range(3):
            c = rng.uniform(0.2, 0.8)
            F[l][:, k] = np.exp(-(x - c) ** 2 / 0.01)
    return Problem(3, n, 0.3, 1.0, 1e-3, np.ones(10), F, "cfg5")


# The test operators of the preconditioning experiments (Sec. 6, eq:precond_ex1-3) as
# (c_neg, c_pos, c0, beta / alpha) of the symbol c0 + c_neg rho^-alpha + c_pos rho^beta.
PRECOND_EQS = {
    "A^a": (0.0, 1.0, 0.0, 1.0),
    "I+A^2a": (0.0, 1.0, 1.0, 2.0),
    "A^a+A^-a": (1.0, 1.0, 0.0, 1.0),
}


def precond_problem(eq, alpha, n, d, kind="ones", seed=7):
    """Right-hand side b of the preconditioning experiments.  The paper does not state it;
    kind "ones" is the constant grid function (rank 1), kind "gauss" two N(0,1) terms."""
    cn, cp, c0, bm = PRECOND_EQS[eq]
    if kind == "ones":
        F = [np.ones((n, 1)) for _ in range(d)]
        w = np.ones(1)
    else:
        F = gaussian_factors(np.random.default_rng(seed), n, d, 2)
        w = np.ones(2)
    return Problem(d, n, alpha, cn, cp, w, F, "%s alpha=%g" % (eq, alpha), c0=c0, beta=bm * alpha)


def sketch_matrices(n, d, q, seed=1000):
    """Gaussian test matrices Omega^(l) (n_l x q), one per mode, for the sketched
    range finder of the truncation (drawn once, passed to the library).  n: one size
    for every mode or a sequence of d sizes."""
    rng = np.random.default_rng(seed)
    ns = list(n) if hasattr(n, "__len__") else [n] * d
    return [rng.standard_normal((ns[l], q)) for l in range(d)]


def restriction_rows(n, stride):
    """0-based indices of the sub-grid i = stride*p (p = 1..), e.g. stride 8 maps the
    n=2047 grid onto its n=255 injection."""
    return np.arange(stride - 1, n, stride)
