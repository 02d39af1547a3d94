"""Low-rank PCG of Algorithm alg:pcg on full-grid arrays (oracle; test infrastructure only).

The iteration follows Algorithm alg:pcg (Sec. 3.3) step for step: R0 = B - fun(X0),
Z0 = trunc(precond(R0)), P0 = Z0; then S = trunc(fun(P)), alpha_k = <R,Z>/<P,S>,
X = trunc(X + alpha_k P), R = trunc(R - alpha_k S), stop when R is small,
Z = trunc(precond(R)), beta_k = <R_new,Z_new>/<Z_old,R_old>, P = trunc(Z + beta_k P).

Here the tensors are full arrays (small n only), fun and precond multiply by a
symbol in the sine basis (eqn:Lap3DtimesX / eqn:DiagFLaplace3D) and trunc is the
HOSVD truncation of tensor.hosvd_truncate.  Readings: X0 = 0 so R0 = B untruncated;
"sufficiently small" means ||R||/||B|| <= tau; k_max = 100 (Sec. 6, tables).
"""
import numpy as np
import scipy.fft as sfft

from . import tensor


def spectral_multiply(x, sym):
    """F^(x d) diag(sym) F^(x d) x for a full array x and a full symbol array."""
    return sfft.idstn(sfft.dstn(x, type=1, norm="ortho") * sym, type=1, norm="ortho")


def _trunc(T, eps, cap):
    core, U, _ = tensor.hosvd_truncate(T, eps, cap)
    return tensor.tucker_full(core, U)


def pcg(op_sym, pre_sym, B, eps, tau, kmax=100, cap=None):
    """Returns (X, iterations, relative residual history)."""
    B = np.asarray(B, dtype=np.float64)
    nb = np.sqrt(tensor.inner(B, B))
    X = np.zeros_like(B)
    R = B.copy()
    Z = _trunc(spectral_multiply(R, pre_sym), eps, cap)
    P = Z
    rz = tensor.inner(R, Z)
    hist = []
    for k in range(kmax):
        S = _trunc(spectral_multiply(P, op_sym), eps, cap)
        a = rz / tensor.inner(P, S)
        X = _trunc(X + a * P, eps, cap)
        R = _trunc(R - a * S, eps, cap)
        res = np.sqrt(tensor.inner(R, R)) / nb
        hist.append(res)
        if res <= tau:
            return X, k + 1, hist
        Z = _trunc(spectral_multiply(R, pre_sym), eps, cap)
        rz_new = tensor.inner(R, Z)
        P = _trunc(Z + (rz_new / rz) * P, eps, cap)
        rz = rz_new
    return X, kmax, hist
