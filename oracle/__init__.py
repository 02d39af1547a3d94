"""CPU FP64 oracle for the rank-structured PCG control solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
GPU library and its Python binding never import it, and it never imports them:
the two share no code, tables or constants.  The only module both sides read is
``workloads`` (seeded input generators, no arithmetic of the method).

Paper: Heidel, Khoromskaia, Khoromskij, Schulz, "Tensor product method for fast
solution of optimal control problems with fractional multidimensional Laplacian
in constraints" (arXiv:1809.01971).

Modules
-------
spectral   1D finite-difference Dirichlet Laplacian, its sine eigenbasis and
           eigenvalues (Sec. 3.2, eqn:eig_lap, eqn:DiagLaplace).
sinc       sinc quadrature of the Laplace transform (Sec. 2, eqn:Laplace_transf,
           eqn:sinc_Laplace_tr; Sec. 4.2, eqn:Laplace_transf_rhom1).
expfit     weighted least-squares exponential sums on fixed geometric exponents
           (the compression reading of the symbol and the preconditioner fit).
exact      O1: the exact control u = A_2^{-1} y_Omega by its spectral definition
           (eqn:frac_Oper, eqn:forControl, eqn:DiagFLaplace3D): full grid,
           restricted evaluation, dense brute force, single-mode closed form.
tensor     canonical / Tucker expansion, Euclidean inner products, HOSVD
           truncation of a full tensor (Sec. 5, eqn:CP_form, eqn:Tucker_form).
lowrank_pcg  the low-rank PCG of Algorithm alg:pcg on full-grid arrays with HOSVD
           truncation (small n only).

Every function states the passage it follows.  Nothing here is tuned for speed.
"""
