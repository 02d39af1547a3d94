"""Canonical / Tucker tensors on the full grid (oracle; test infrastructure only).

Sec. 5: canonical format T = sum_k xi_k u_k^(1) (x) ... (x) u_k^(d) (eqn:CP_form),
orthogonal Tucker format T = beta x_1 V^(1) ... x_d V^(d) (eqn:Tucker_form, Tuckt),
and the HOSVD (De Lathauwer et al., cited in Sec. 5): per mode the left singular
vectors of the mode unfolding, core by projection (eqn coret).

Rank rule (the paper gives none): r_l is the least r with
sum_{i>r} sigma_{l,i}^2 <= eps^2 ||T||^2 / d, so that the HOSVD error bound
||T - T_r||^2 <= sum_l sum_{i>r_l} sigma_{l,i}^2 gives ||T - T_r|| <= eps ||T||.
"""
import numpy as np


def cp_full(weights, factors):
    """Expand sum_k xi_k (x)_l u_k^(l) to the full array (eqn:CP_form)."""
    w = np.asarray(weights, dtype=np.float64)
    T = None
    for k in range(w.shape[0]):
        t = np.asarray(factors[0][:, k], dtype=np.float64) * w[k]
        for f in factors[1:]:
            t = np.multiply.outer(t, np.asarray(f[:, k], dtype=np.float64))
        T = t if T is None else T + t
    if T is None:
        T = np.zeros(tuple(f.shape[0] for f in factors))
    return T


def mode_product(T, M, l):
    """T x_l M: contract mode l of T with the columns of M (M is m x n_l)."""
    Tl = np.moveaxis(T, l, 0)
    R = np.tensordot(M, Tl, axes=([1], [0]))
    return np.moveaxis(R, 0, l)


def tucker_full(core, factors):
    """Expand beta x_1 V^(1) ... x_d V^(d) (eqn:Tuckt)."""
    T = np.asarray(core, dtype=np.float64)
    for l, V in enumerate(factors):
        T = mode_product(T, np.asarray(V, dtype=np.float64), l)
    return T


def unfolding(T, l):
    """Mode-l unfolding: n_l x prod_{m != l} n_m."""
    return np.moveaxis(T, l, 0).reshape(T.shape[l], -1)


def inner(A, B):
    """Euclidean inner product of two full arrays (finite differences, M = I, Sec. 3.1)."""
    return float(np.sum(np.asarray(A) * np.asarray(B)))


def hosvd_ranks(T, eps, cap=None):
    """Mode singular values and the ranks chosen by the energy rule above."""
    T = np.asarray(T, dtype=np.float64)
    d = T.ndim
    tot = float(np.sum(T * T))
    ranks, svals, bases = [], [], []
    for l in range(d):
        U, s, _ = np.linalg.svd(unfolding(T, l), full_matrices=False)
        tail = np.concatenate([np.cumsum((s**2)[::-1])[::-1], [0.0]])
        r = next(r for r in range(0, len(s) + 1) if tail[r] <= eps**2 * tot / d)
        r = max(r, 1 if tot > 0 else 0)
        if cap is not None:
            r = min(r, cap)
        ranks.append(r)
        svals.append(s)
        bases.append(U[:, :r])
    return ranks, svals, bases


def hosvd_truncate(T, eps, cap=None):
    """HOSVD truncation of a full tensor: returns (core, factors, ranks)."""
    ranks, _, bases = hosvd_ranks(T, eps, cap)
    core = np.asarray(T, dtype=np.float64)
    for l, U in enumerate(bases):
        core = mode_product(core, U.T, l)
    return core, bases, ranks
