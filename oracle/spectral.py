"""1D spectra of the finite-difference Dirichlet Laplacian (oracle; test infrastructure only).

Sec. 3.2 of the paper discretises -y'' on (0,1) with homogeneous Dirichlet data on a
uniform grid and diagonalises the 1D matrix A_(l) in the sine basis
(A_(l) = F* Lambda F, eqn:eig_lap).  Readings taken here:

* A = -Delta_h is SPD: A_(l) = tridiag(-1, 2, -1) / h^2 and the eigenvalues are
  lambda_k = (4/h^2) sin^2(pi k h / 2) > 0 (the printed minus sign is that of the
  Laplacian itself, not of the SPD operator).
* n counts interior points, h = 1/(n+1), x_i = i h for i = 1..n (Sec. 4.1 uses
  h = 1/(n+1); both printed forms of lambda_k agree only for that h).
* F is the orthonormal DST-I, F_jk = sqrt(2/(n+1)) sin(pi j k/(n+1)), j,k = 1..n,
  so F = F^T = F^{-1}; factor entry j is the value at x_j.
"""
import numpy as np


def mesh_width(n):
    """h = 1/(n+1) for n interior points (Sec. 4.1)."""
    return 1.0 / (n + 1)


def eigenvalues(n):
    """lambda_k = (4/h^2) sin^2(pi k h/2), k = 1..n (eqn:eig_lap, SPD sign)."""
    h = mesh_width(n)
    k = np.arange(1, n + 1, dtype=np.float64)
    return 4.0 / h**2 * np.sin(np.pi * k * h / 2.0) ** 2


def laplacian_1d(n):
    """Dense A_(l) = tridiag(-1, 2, -1)/h^2 (Sec. 3.2, the 1D subproblem matrix)."""
    h = mesh_width(n)
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return A / h**2


def dst_matrix(n):
    """Orthonormal sine transform F_jk = sqrt(2/(n+1)) sin(pi j k/(n+1)) (Sec. 3.2)."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(j, j) / (n + 1))


def dst(x):
    """F x applied to every column of x by the plain matrix product (definition)."""
    x = np.asarray(x, dtype=np.float64)
    return dst_matrix(x.shape[0]) @ x


def rho_grid(ns):
    """rho(i_1..i_d) = sum_l lambda_{i_l}: the diagonal of Lambda in eqn:DiagLaplace,
    folded to an n_1 x ... x n_d array (Sec. 4.1, g(i_1,i_2,i_3))."""
    lams = [eigenvalues(n) for n in ns]
    d = len(ns)
    rho = np.zeros(tuple(ns))
    for l, lam in enumerate(lams):
        shape = [1] * d
        shape[l] = ns[l]
        rho = rho + lam.reshape(shape)
    return rho


def rho_directional(ns, alpha):
    """rho'(i_1..i_d) = sum_l lambda_{i_l}^alpha: the eigenvalues of the directionally fractional
    operator sum_l (-Delta_l)^alpha (Sec. 4.1, Remark rem:direct_fract_Lap, eq:Laplace_1Dfract),
    whose cores eq:3a1d-eq:3c1d are functions of this sum."""
    lams = [eigenvalues(n) ** alpha for n in ns]
    d = len(ns)
    rho = np.zeros(tuple(ns))
    for l, lam in enumerate(lams):
        shape = [1] * d
        shape[l] = ns[l]
        rho = rho + lam.reshape(shape)
    return rho


def symbol(rho, alpha, c_neg, c_pos, c0=0.0, beta=None):
    """s(rho) = c0 + c_neg rho^-alpha + c_pos rho^beta (beta = alpha unless given): the
    eigenvalues of c0 I + c_neg A^-alpha + c_pos A^beta (spectral definition eqn:frac_Oper).
    c0 = 0, beta = alpha is A_2 of eqn:forControl (c_neg = beta, c_pos = gamma/beta); the
    preconditioning tests of Sec. 6 use A^alpha (eq:precond_ex1: c_neg = c0 = 0),
    I + A^{2 alpha} (eq:precond_ex2: c0 = 1, beta = 2 alpha) and A^alpha + A^-alpha
    (eq:precond_ex3)."""
    rho = np.asarray(rho, dtype=np.float64)
    b = alpha if beta is None else beta
    return c0 + c_neg * rho ** (-alpha) + c_pos * rho**b
