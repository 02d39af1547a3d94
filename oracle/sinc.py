"""Sinc quadrature of the Laplace transform (oracle; test infrastructure only).

Sec. 2 (eqn:Laplace_transf, eqn:sinc_Laplace_tr) and Sec. 4.2
(eqn:Laplace_transf_rhom1 and the substitution that follows it):

    rho^-mu = 1/Gamma(mu) int_0^inf t^(mu-1) exp(-rho t) dt ,   rho in [1, B].

With t = phi(u) = log(1 + e^u) the integral runs over the real line and the
trapezoidal (sinc) rule with step hh at u_k = k hh gives a separable
exponential sum  rho^-mu ~ sum_k c_k exp(-t_k rho),

    t_k = phi(u_k),   c_k = hh phi(u_k)^(mu-1) phi'(u_k) / Gamma(mu),
    phi'(u) = 1/(1 + e^-u).

Readings (the printed integrand has exp(-rho log(1+e^-u)), which does not decay
as u -> +inf; the substitution t = log(1+e^u) that the text names is used):

* the range rho in [1, B] is reached by scaling with rho0 = d lambda_1:
  rho^-mu = rho0^-mu (rho/rho0)^-mu, so the factor vectors become
  exp(-(t_k/rho0) lambda_i);
* the index range is k = -kL..kR (the paper's symmetric -M..M is kL = kR = M)
  and hh = c pi / sqrt(M) is the paper's step rule; both are arguments here.

Lemma 4.1 (A^alpha = A A^(alpha-1)) is used on the whole control operator:
s(rho) = c_neg rho^-alpha + c_pos rho^alpha = rho * g(rho) with
g(rho) = c_neg rho^-(1+alpha) + c_pos rho^-(1-alpha), a sum of negative powers,
so one sinc rule on the Laplace transform of g gives g ~ sum_k w_k exp(-t_k rho)
and s has Kronecker rank d * K (rho = sum_l lambda_l is Kronecker rank d).
"""
import math

import numpy as np


def phi(u):
    """t = log(1 + e^u), computed without overflow."""
    return np.logaddexp(0.0, u)


def dphi(u):
    """phi'(u) = 1/(1 + e^-u), written as e^u/(1 + e^u) for u < 0 so that the
    relative accuracy holds far into the left tail."""
    u = np.asarray(u, dtype=np.float64)
    e = np.exp(-np.abs(u))
    return np.where(u >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def paper_step(M, c):
    """hh = c pi / sqrt(M) (Sec. 4.2, after eqn:Laplace_transf_rhom1)."""
    return c * math.pi / math.sqrt(M)


def laplace_nodes(mu, kL, kR, hh):
    """Nodes t_k and weights c_k with rho^-mu ~ sum_k c_k exp(-t_k rho), k = -kL..kR,
    for rho in [1, B] (unscaled).  eqn:sinc_Laplace_tr with hat c_k t_k^(mu-1)."""
    k = np.arange(-kL, kR + 1, dtype=np.float64)
    u = k * hh
    t = phi(u)
    c = hh * t ** (mu - 1.0) * dphi(u) / math.gamma(mu)
    return t, c


def g_nodes(alpha, c_neg, c_pos, rho0, kL, kR, hh):
    """Exponents tau_k (for the unscaled rho) and weights w_k with
    g(rho) = c_neg rho^-(1+alpha) + c_pos rho^-(1-alpha) ~ sum_k w_k exp(-tau_k rho).

    Both powers share the sinc nodes t_k = phi(u_k) of the scaled variable
    y = rho/rho0: rho^-mu = rho0^-mu y^-mu and y^-mu ~ sum c_k(mu) exp(-t_k y).
    For alpha = 1 the second power is the constant c_pos, represented exactly by
    one extra exponent tau = 0 (A^1 = A has Kronecker rank d, Lemma 4.1 remark).
    """
    t, c1 = laplace_nodes(1.0 + alpha, kL, kR, hh)
    w = c_neg * rho0 ** (-(1.0 + alpha)) * c1
    if abs(1.0 - alpha) < 1e-15:
        tau = np.concatenate([t / rho0, [0.0]])
        w = np.concatenate([w, [c_pos]])
        return tau, w
    _, c2 = laplace_nodes(1.0 - alpha, kL, kR, hh)
    w = w + c_pos * rho0 ** (-(1.0 - alpha)) * c2
    return t / rho0, w


def expsum(rho, tau, w):
    """sum_k w_k exp(-tau_k rho) at every rho (direct evaluation)."""
    rho = np.asarray(rho, dtype=np.float64)
    return np.exp(-np.multiply.outer(rho, tau)) @ w
