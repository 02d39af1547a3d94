"""O1: the exact discrete control u = A_2^-1 y_Omega (oracle; test infrastructure only).

The control equation eqn:forControl reads (beta A^-alpha + (gamma/beta) A^alpha) u = y_Omega,
written here as (c_neg A^-alpha + c_pos A^alpha) u = f.  A is the d-dimensional
finite-difference Dirichlet Laplacian, diagonalised by the tensor sine transform
(eqn:DiagLaplace, eqn:DiagFLaplace3D), and A^alpha is defined spectrally
(eqn:frac_Oper).  Hence

    u = F^(x d) diag(1/s(rho)) F^(x d) f ,  s(rho) = c_neg rho^-alpha + c_pos rho^alpha,

which is what every routine below evaluates, each by a different route.
"""
import numpy as np
import scipy.fft as sfft

from . import spectral, tensor


def solve_full(f, alpha, c_neg, c_pos, c0=0.0, beta=None):
    """u on the full grid: forward sine transform, divide by s(rho), inverse
    (eqn:DiagFLaplace3D / eqn:DiagFLaplace2D).  The orthonormal DST-I of scipy is
    the library step for F (it equals spectral.dst_matrix, pinned in the tests).
    c0 and beta give the general symbol of spectral.symbol."""
    f = np.asarray(f, dtype=np.float64)
    fh = sfft.dstn(f, type=1, norm="ortho")
    s = spectral.symbol(spectral.rho_grid(f.shape), alpha, c_neg, c_pos, c0, beta)
    return sfft.idstn(fh / s, type=1, norm="ortho")


def apply_full(x, alpha, c_neg, c_pos, c0=0.0, beta=None):
    """A_2 x on the full grid (the same diagonalisation, multiplying by s)."""
    x = np.asarray(x, dtype=np.float64)
    xh = sfft.dstn(x, type=1, norm="ortho")
    s = spectral.symbol(spectral.rho_grid(x.shape), alpha, c_neg, c_pos, c0, beta)
    return sfft.idstn(xh * s, type=1, norm="ortho")


def laplacian_full(ns):
    """The d-dimensional matrix A as the Kronecker sum of the 1D tridiagonal matrices
    (eqn_low_rank_lap), dense.  Only for n^d up to a few thousand."""
    N = int(np.prod(ns))
    A = np.zeros((N, N))
    for l, n in enumerate(ns):
        mats = [np.eye(m) for m in ns]
        mats[l] = spectral.laplacian_1d(n)
        K = mats[0]
        for M in mats[1:]:
            K = np.kron(K, M)
        A += K
    return A


def brute_force(f, alpha, c_neg, c_pos, c0=0.0, beta=None):
    """Dense route that uses no sine transform: A from laplacian_full, its
    eigendecomposition by numpy.linalg.eigh, c0 I + c_neg A^-alpha + c_pos A^beta from the
    eigenpairs, dense solve."""
    f = np.asarray(f, dtype=np.float64)
    ns = f.shape
    N = int(np.prod(ns))
    A = laplacian_full(ns)
    lam, Q = np.linalg.eigh(A)
    b = alpha if beta is None else beta
    A2 = (Q * (c0 + c_neg * lam ** (-alpha) + c_pos * lam**b)) @ Q.T
    return np.linalg.solve(A2, f.reshape(N)).reshape(ns)


def sine_mode(n, k):
    """Grid values sin(k pi x_i), x_i = i/(n+1): the k-th eigenvector of A_(l)."""
    x = np.arange(1, n + 1) / (n + 1.0)
    return np.sin(k * np.pi * x)


def single_mode_factor(ns, ks, alpha, c_neg, c_pos, c0=0.0, beta=None):
    """For f = (x)_l sin(k_l pi x): u = f / s(sum_l lambda_{k_l}) exactly."""
    rho = sum(spectral.eigenvalues(n)[k - 1] for n, k in zip(ns, ks))
    return 1.0 / float(spectral.symbol(rho, alpha, c_neg, c_pos, c0, beta))


def solve_cp_restricted(weights, factors, alpha, c_neg, c_pos, rows):
    """u at the sample grid points rows[0] x rows[1] x rows[2] (0-based indices)
    for a canonical right-hand side f = sum_t xi_t (x)_l f^(l)_t (eqn:CP_form).

    f-hat = (x)_l F f^(l)_t is exact (Kronecker identity), then slab by slab over the
    first spectral index i1: W = f-hat[i1] / s(lambda_i1 + lambda_j + lambda_k),
    u[R1,R2,R3] += F[R1, i1] (x) (F[R2,:] W F[R3,:]^T).  O(n^2) memory, no n^3 array."""
    w = np.asarray(weights, dtype=np.float64)
    ns = [f.shape[0] for f in factors]
    assert len(ns) == 3
    lam = [spectral.eigenvalues(n) for n in ns]
    Fh = [spectral.dst(f) for f in factors]          # F f_t per mode
    Fr = [spectral.dst_matrix(n)[np.asarray(r)] for n, r in zip(ns, rows)]
    out = np.zeros((len(rows[0]), len(rows[1]), len(rows[2])))
    rho23 = lam[1][:, None] + lam[2][None, :]
    for i1 in range(ns[0]):
        slab = (Fh[1] * (w * Fh[0][i1])) @ Fh[2].T       # f-hat[i1, :, :]
        rho = lam[0][i1] + rho23
        W = slab / (c_neg * rho ** (-alpha) + c_pos * rho**alpha)
        out += np.multiply.outer(Fr[0][:, i1], Fr[1] @ W @ Fr[2].T)
    return out


def solve_cp_restricted_slabs(weights, factors, alpha, c_neg, c_pos, rows, slabs):
    """The same sum as solve_cp_restricted restricted to the first-index slabs
    listed in `slabs` (used to time a bounded sample of the full evaluation)."""
    w = np.asarray(weights, dtype=np.float64)
    ns = [f.shape[0] for f in factors]
    lam = [spectral.eigenvalues(n) for n in ns]
    Fh = [spectral.dst(f) for f in factors]
    Fr = [spectral.dst_matrix(n)[np.asarray(r)] for n, r in zip(ns, rows)]
    out = np.zeros((len(rows[0]), len(rows[1]), len(rows[2])))
    rho23 = lam[1][:, None] + lam[2][None, :]
    for i1 in slabs:
        slab = (Fh[1] * (w * Fh[0][i1])) @ Fh[2].T
        rho = lam[0][i1] + rho23
        W = slab / (c_neg * rho ** (-alpha) + c_pos * rho**alpha)
        out += np.multiply.outer(Fr[0][:, i1], Fr[1] @ W @ Fr[2].T)
    return out


def tucker_error_slabs(weights, factors, alpha, c_neg, c_pos, core, tfactors, slabs):
    """Partial sums over first-index slabs of the spectral (Parseval) identity
    ||X - u||^2 = sum_i (Xhat_i - fhat_i / s(rho_i))^2 and ||u||^2 = sum_i (fhat_i/s(rho_i))^2,
    where u is the exact control for the canonical right-hand side (weights, factors) and
    X = core x_1 T1 x_2 T2 x_3 T3 a Tucker tensor (any factors).  F is orthogonal, so the sums over
    spectral indices equal the grid sums.  Returns (sum of squared errors, sum of squared u)."""
    w = np.asarray(weights, dtype=np.float64)
    ns = [f.shape[0] for f in factors]
    lam = [spectral.eigenvalues(n) for n in ns]
    Fh = [spectral.dst(f) for f in factors]
    Th = [spectral.dst(np.asarray(t, dtype=np.float64)) for t in tfactors]
    C = np.asarray(core, dtype=np.float64)
    rho23 = lam[1][:, None] + lam[2][None, :]
    err2 = 0.0
    u2 = 0.0
    for i1 in slabs:
        fh = (Fh[1] * (w * Fh[0][i1])) @ Fh[2].T
        rho = lam[0][i1] + rho23
        uh = fh / (c_neg * rho ** (-alpha) + c_pos * rho**alpha)
        Ca = np.tensordot(Th[0][i1], C, axes=([0], [0]))          # r2 x r3
        xh = Th[1] @ Ca @ Th[2].T
        err2 += float(np.sum((xh - uh) ** 2))
        u2 += float(np.sum(uh * uh))
    return err2, u2


def solve_directional(f, alpha, c_neg, c_pos, c0=0.0):
    """u on the full grid for the directionally fractional operator A_(alpha) = sum_l
    (-Delta_l)^alpha (Remark rem:direct_fract_Lap, eq:Laplace_1Dfract) in the control equation's
    place of A^alpha: (c0 I + c_neg A_(alpha)^-1 + c_pos A_(alpha)) u = f.  Its spectral values are
    c0 + c_neg / rho' + c_pos rho', rho' = sum_l lambda_{i_l}^alpha (the reciprocal of the core
    eq:3c1d for c0 = 0, c_neg = c_pos = 1)."""
    f = np.asarray(f, dtype=np.float64)
    fh = sfft.dstn(f, type=1, norm="ortho")
    rp = spectral.rho_directional(f.shape, alpha)
    return sfft.idstn(fh / (c0 + c_neg / rp + c_pos * rp), type=1, norm="ortho")


def brute_force_directional(f, alpha, c_neg, c_pos, c0=0.0):
    """Dense route without the sine transform: (A_l)^alpha from numpy.linalg.eigh of each 1D
    tridiagonal matrix, A_(alpha) as their Kronecker sum, then c0 I + c_neg A_(alpha)^-1 +
    c_pos A_(alpha) formed with a dense inverse and solved."""
    f = np.asarray(f, dtype=np.float64)
    ns = f.shape
    N = int(np.prod(ns))
    Ad = np.zeros((N, N))
    for l, n in enumerate(ns):
        lam, Q = np.linalg.eigh(spectral.laplacian_1d(n))
        mats = [np.eye(m) for m in ns]
        mats[l] = (Q * lam**alpha) @ Q.T
        K = mats[0]
        for M in mats[1:]:
            K = np.kron(K, M)
        Ad += K
    A2 = c0 * np.eye(N) + c_neg * np.linalg.inv(Ad) + c_pos * Ad
    return np.linalg.solve(A2, f.reshape(N)).reshape(ns)


def precond_rank_r(ns, r, alpha, c_neg, c_pos, c0=0.0, beta=None):
    """The rank-r preconditioner of the Sec. 6 iteration counts on the full grid: the inverse
    symbol 1/s(rho) (the spectral values of the operator's inverse, eqn:DiagFLaplace3D) truncated
    by the HOSVD to mode ranks <= r.  In 2D this is the rank-r SVD of the n x n matrix
    1/s(lambda_i + lambda_j) (the paper's 2D reduced SVD); in 3D the Tucker rank-r reading of
    its multigrid Tucker approximation."""
    P = 1.0 / spectral.symbol(spectral.rho_grid(ns), alpha, c_neg, c_pos, c0, beta)
    core, U, _ = tensor.hosvd_truncate(P, 0.0, cap=r)
    return tensor.tucker_full(core, U)


def state_full(u, alpha, beta):
    """State y = beta A^-alpha u (eqn:State, eqn:L_alp_state) on the full grid."""
    u = np.asarray(u, dtype=np.float64)
    uh = sfft.dstn(u, type=1, norm="ortho")
    rho = spectral.rho_grid(u.shape)
    return sfft.idstn(beta * rho ** (-alpha) * uh, type=1, norm="ortho")


def cost_functional(y, u, y_omega, gamma):
    """J(y,u) = 1/2 ||y - y_Omega||^2 + gamma/2 ||u||^2 (discrete cost of Sec. 3.1, M = I)."""
    return 0.5 * float(np.sum((y - y_omega) ** 2)) + 0.5 * gamma * float(np.sum(u * u))
