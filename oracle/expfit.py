"""Weighted least-squares exponential sums (oracle; test infrastructure only).

The paper precomputes the operator and preconditioner in low Kronecker rank
(Sec. 1, Sec. 3.1 after eqn:forControl; Sec. 5: multigrid Tucker of the full
core tensor, then Tucker-to-canonical).  On the n^d grid that precompute costs
O(n^d); the reading used here keeps the cost linear in n: the symbol is a
function of rho = sum_l lambda_l only, so a short exponential sum in rho,
sum_k w_k exp(-tau_k rho), is a canonical tensor of rank K (rank d K after the
Lemma 4.1 factor rho).  The exponents are fixed on a geometric grid and the
weights solve a relative-error least-squares problem on log-spaced samples:

    min_w  sum_j ( sum_k w_k exp(-t_k y_j) / f(y_j) - 1 )^2 ,   y_j in [1, B],

with y = rho/rho0 and t_k = exp(linspace(log(1/B) + a, b, K)).  The same fit
with f = 1/s gives the preconditioner (a low Kronecker rank approximation of
A_2^-1, Sec. 1 and eqn:OptCont).
"""
import numpy as np


def geometric_exponents(B, K, a, b):
    """t_k = exp(linspace(log(1/B) + a, b, K)) for the scaled variable y in [1, B]."""
    return np.exp(np.linspace(np.log(1.0 / B) + a, b, K))


def log_samples(B, m):
    """m log-spaced sample points in [1, B]."""
    return np.exp(np.linspace(0.0, np.log(B), m))


def fit_weights(f, t, B, m):
    """Relative-error least-squares weights for sum_k w_k exp(-t_k y) ~ f(y).

    Solved through numpy's SVD least squares with cut-off 1e-15 * sigma_max."""
    y = log_samples(B, m)
    E = np.exp(-np.outer(y, t)) / f(y)[:, None]
    w, *_ = np.linalg.lstsq(E, np.ones(m), rcond=1e-15)
    return w


def max_rel_error(f, t, w, B, m=20000):
    """max over m log-spaced y in [1, B] of |sum_k w_k exp(-t_k y)/f(y) - 1|."""
    y = log_samples(B, m)
    return float(np.max(np.abs((np.exp(-np.outer(y, t)) @ w) / f(y) - 1.0)))
