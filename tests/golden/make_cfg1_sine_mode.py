"""Writes cfg1_sine_mode.txt: the worked single-mode example of the 2D workload (n = 63,
h = 1/64, modes k = (3, 5)) evaluated in 50-digit arithmetic.

It uses only mpmath and the closed forms of the paper:
  lambda_k = (4/h^2) sin^2(pi k h / 2)                      (Sec. 3.2, eqn:eig_lap, SPD sign)
  s(rho) = c_neg rho^-alpha + c_pos rho^alpha, rho = lambda_3 + lambda_5   (eqn:forControl)
  u = f / s(rho) for the separable sine mode f               (eqn:DiagFLaplace2D)
No oracle or library routine enters, so the stored values pin the oracle independently.

    python tests/golden/make_cfg1_sine_mode.py      # rewrites the file next to this script
"""
import os

import mpmath as mp

mp.mp.dps = 50

HEADER = """\
# Worked single-mode example (2D, n=63, h=1/64, modes k=(3,5)).
# Source of the formulas: eqn:eig_lap (lambda_k = (4/h^2) sin^2(pi k h/2), SPD sign reading)
# and eqn:forControl (A_2 = beta A^-alpha + (gamma/beta) A^alpha); the paper prints no
# worked example, these values are the closed forms evaluated in 50-digit arithmetic
# (mpmath, tests/golden/make_cfg1_sine_mode.py) and rounded to 15 significant digits.
"""


def lam(n, k):
    h = mp.mpf(1) / (n + 1)
    return 4 / h**2 * mp.sin(mp.pi * k * h / 2) ** 2


def symbol(rho, alpha, c_neg, c_pos):
    return c_neg * rho ** (-alpha) + c_pos * rho**alpha


def values():
    n, alpha = 63, mp.mpf(1) / 2
    beta, gamma = mp.mpf(1), mp.mpf("1e-2")
    l3, l5 = lam(n, 3), lam(n, 5)
    rho = l3 + l5
    s_paper = symbol(rho, alpha, beta, gamma / beta)     # paper form
    s_literal = symbol(rho, alpha, gamma, beta)          # beta A^alpha + gamma A^-alpha
    return [("lambda_3", l3), ("lambda_5", l5), ("rho", rho), ("s_paper", s_paper),
            ("u_over_f_paper", 1 / s_paper), ("s_literal", s_literal), ("u_over_f_literal", 1 / s_literal)]


def render():
    out = [HEADER.rstrip("\n")]
    for name, v in values():
        if name == "s_literal":
            out.append("# literal operator beta A^alpha + gamma A^-alpha (c_neg=1e-2, c_pos=1)")
        if name == "lambda_3":
            out.append("# alpha=1/2, beta=1, gamma=1e-2  -> paper form c_neg=1, c_pos=1e-2")
        out.append("%s %s" % (name, mp.nstr(v, 15)))
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg1_sine_mode.txt")
    with open(path, "w") as fh:
        fh.write(render())
    print(path)
