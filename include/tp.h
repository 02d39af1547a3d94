/*
 * tp.h -- C ABI of the rank-structured PCG solver for the fractional control equation
 *
 *   A_2 u = (c_neg A^-alpha + c_pos A^alpha) u = f          (eqn:forControl)
 *
 * of Heidel, Khoromskaia, Khoromskij, Schulz (arXiv:1809.01971).  A is the
 * d-dimensional (d = 2, 3) finite-difference Dirichlet Laplacian on n interior
 * points per mode (h = 1/(n+1)), diagonalised by the orthonormal sine transform
 * (eqn:DiagLaplace, eqn:DiagFLaplace3D).  The paper's coefficients are
 * c_neg = beta, c_pos = gamma/beta.
 *
 * Conventions for every entry point
 *   - Pointers marked "device" are HIP device memory owned by the caller; the
 *     library never frees them.  Pointers marked "host" are ordinary host memory.
 *   - Matrices are column-major.  A factor matrix of mode l is n[l] x cap with
 *     leading dimension n[l]; its first rank[l] columns are meaningful.
 *   - All work is ordered on the stream given to tp_create.  Calls that return
 *     host values (ranks, scalars, info) synchronise that stream.
 *   - A context is used by one host thread at a time.
 *   - Errors: every call returns a tp_status; on failure tp_last_error() gives a
 *     message (thread-local, valid until the next call on that thread).  Invalid
 *     arguments are rejected before any device work is enqueued.
 *   - The grid size n must satisfy n >= 1 and n+1 a power of two (the sine
 *     transform runs as a radix-2 FFT), n+1 <= 32768, in both precisions.
 */
#ifndef TP_H
#define TP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TP_OK = 0,
  TP_EINVAL = 1,    /* invalid argument (shape, rank, parameter, precision mismatch) */
  TP_ENOMEM = 2,    /* workspace or device allocation too small / failed */
  TP_ENOCONV = 3,   /* PCG did not reach tau; x holds its best iterate (the tables' '---') */
  TP_ERANK = 4,     /* a truncation hit the rank cap with the tolerance unmet */
  TP_EHIP = 5,      /* a HIP runtime call failed */
  TP_EINDEF = 6     /* tp_symbol_build: the preconditioner is not positive on the points it was
                     * checked on (PCG needs a positive definite one); both symbols are still
                     * returned, owned by the caller, and a solve with them may break down */
} tp_status;

typedef enum { TP_FP64 = 0, TP_MIXED = 1 } tp_precision;
typedef enum { TP_SYM_FIT = 0, TP_SYM_SINC = 1 } tp_symbol_method;

typedef struct tp_ctx tp_ctx;
typedef struct tp_symbol tp_symbol;

/* Library version (major*100 + minor). */
int tp_version(void);

/* Message for the last non-OK status on this thread. */
const char* tp_last_error(void);

/* Create a context on HIP device `device`, ordering work on `stream` (a hipStream_t,
 * NULL = default stream).  `workspace_bytes` of device memory are allocated once
 * here (0 = 2 GiB); no entry point allocates device memory afterwards except
 * tp_symbol_build (which owns its symbols) and the per-grid sine tables created
 * on first use of a grid size. */
tp_status tp_create(int device, void* stream, size_t workspace_bytes, tp_ctx** out);
tp_status tp_destroy(tp_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Tensors
 * ------------------------------------------------------------------------- */

/* Tucker tensor T = core x_1 V^(1) x_2 V^(2) (x_3 V^(3))  (eqn:Tucker_form).
 * core: device, capacity cap^d elements; holds rank[0] x rank[1] (x rank[2])
 *       column-major, packed (leading dimensions equal the ranks).
 * factor[l]: device, n[l] x cap column-major, ld n[l].
 * cap: at most 128 (the sum of two iterates is diagonalised at size <= 256).
 * prec: TP_FP64 -> double elements, TP_MIXED -> float elements (core and factors).
 * rank: host-side mode ranks; written by every call that produces the tensor.
 * Outputs written by truncation have orthonormal factors. */
typedef struct {
  int32_t d;
  int32_t n[3];
  int32_t cap;
  int32_t prec;
  int32_t rank[3];
  void* core;
  void* factor[3];
} tp_tensor;

/* Canonical tensor sum_k weight[k] (x)_l factor[l][:,k]  (eqn:CP_form), device memory,
 * always FP64 (right-hand sides enter in double). */
typedef struct {
  int32_t d;
  int32_t n[3];
  int32_t rank;
  const double* weight;      /* device, rank */
  const double* factor[3];   /* device, n[l] x rank, ld n[l] */
} tp_cp;

/* Gaussian test matrices for the sketched truncation of operator products:
 * omega[l] is device, n[l] x q, ld n[l], FP64, 2 <= q <= 192.  The random numbers are an input:
 * the library draws none. */
typedef struct {
  int32_t q;
  const double* omega[3];
} tp_sketch;

/* ---------------------------------------------------------------------------
 * Operator symbols  (Sec. 2 eqn:sinc_Laplace_tr; Sec. 4.1 Lemma 4.1; Sec. 4.2)
 * ------------------------------------------------------------------------- */

/* In the sine basis A_2 is diagonal with entries s(rho), rho = sum_l lambda_{i_l},
 * s = c0 + c_neg rho^-alpha + c_pos rho^beta (beta = alpha for the control equation;
 * c0 and beta != alpha give the test operators A^alpha, I + A^(2 alpha) and
 * A^alpha + A^-alpha of the preconditioning experiments, Sec. 6 eq:precond_ex1-3).
 * Lemma 4.1 is applied to A_2 itself: s(rho) = c0 + rho * g(rho),
 * g = c_neg rho^-(1+alpha) + c_pos rho^-(1-beta), and g is an exponential sum
 * sum_k w_k exp(-tau_k rho), so the operator symbol is a canonical tensor of rank
 * d*K (+1 for the constant c0, whose factors are all ones) in spectral coordinates.
 * For beta = 1 the term c_pos rho is kept exact as an exponential with tau = 0
 * (the d one-dimensional Laplacians), and only the c_neg part is fitted.  The
 * preconditioner is a rank-K' exponential sum approximating 1/s (a low Kronecker
 * rank approximation of A_2^-1, Sec. 1).
 *
 * method TP_SYM_SINC (c0 = 0, beta = alpha only): g by the sinc rule u_k = k*h,
 *   k = -sinc_kl..sinc_kr, t = log(1+e^u), weights h phi'(u) [c_neg t^alpha/Gamma(1+alpha)
 *   rho0^-(1+alpha) + c_pos t^-alpha/Gamma(1-alpha) rho0^-(1-alpha)], rho0 = d*lambda_1
 *   (Sec. 2 eqn:sinc_Laplace_tr, Sec. 4.2 with the substitution t = log(1+e^u)).  The paper's
 *   symmetric rule with M is sinc_kl = sinc_kr = M (2M+1 nodes).  sinc_h = 0: the step is
 *   h = c pi / sqrt(M'), M' = (sinc_kl + sinc_kr)/2, with the c of 24 geometric values in
 *   [0.4, 4] whose rule has the smallest measured error (the paper leaves c open).
 * method TP_SYM_FIT: g by relative-error least squares on op_terms geometric
 *   exponents (fewer terms for the same accuracy).
 * The preconditioner always uses the least-squares fit with pre_terms exponents. */
typedef struct {
  int32_t d;
  int32_t n[3];
  double alpha;        /* 0 < alpha <= 1 */
  double c_neg;        /* >= 0 */
  double c_pos;        /* >= 0, c_neg + c_pos > 0 */
  int32_t method;      /* tp_symbol_method */
  int32_t op_terms;    /* TP_SYM_FIT: K (0 = 32); ignored when nothing is left to fit */
  int32_t pre_terms;   /* K' in [1, 64] (0 = 12) */
  int32_t sinc_kl;     /* TP_SYM_SINC: nodes left of u = 0 (0 = 60) */
  int32_t sinc_kr;     /* nodes right of u = 0 (0 = 20) */
  double sinc_h;       /* step (0 = chosen by the library, see above) */
  int32_t prec;        /* precision of the factor matrices (tp_precision) */
  double c0;           /* >= 0: constant term of the symbol (identity part of the operator) */
  double beta;         /* exponent of the c_pos term, in (0, 1]; 0 = alpha */
  int32_t pre_rank;    /* 0: the preconditioner is the pre_terms-term exponential sum (rank K');
                        * r in [1,16]: that sum recompressed by its truncated HOSVD to mode ranks
                        * <= r (in 2D the rank-r SVD of the matrix 1/s(lambda_i + lambda_j)), the
                        * Tucker core spread back to canonical rank r (2D) or r^2 (3D): the rank-r
                        * preconditioner of the Sec. 6 iteration counts.  Its err is then the max of
                        * |p s - 1| over a geometric lattice of grid points. */
  int32_t directional; /* 1: the directionally fractional operator A_(alpha) = sum_l (-Delta_l)^alpha
                        * (Sec. 4.1 Remark rem:direct_fract_Lap, eq:Laplace_1Dfract) takes the
                        * place of A^alpha: the 1D spectra are lambda^alpha, rho' = sum_l
                        * lambda_{i_l}^alpha, and s = c0 + c_neg / rho' + c_pos rho' (beta must be
                        * 0 or 1); the cores eq:3a1d-3c1d are 1/rho', 1/rho' + rho' and its inverse */
} tp_symbol_desc;

/* Build the operator symbol and the preconditioner symbol on the GPU.  Both are
 * owned by the library (free with tp_symbol_free).  err (host, 2 doubles, may be
 * NULL) receives the measured max relative errors of the two exponential sums
 * on 4096 log-spaced points of [rho_min, rho_max] (for pre_rank > 0 the second is
 * max |p s - 1| over the lattice of grid points).  Returns TP_EINDEF, with both symbols
 * built and returned, when the preconditioner p is not positive on those points: for the
 * fitted sum when its relative error reaches 1, for a rank-r preconditioner when
 * min p s <= 0 on the lattice (Algorithm alg:pcg needs a positive definite preconditioner). */
tp_status tp_symbol_build(tp_ctx* ctx, const tp_symbol_desc* desc, tp_symbol** op,
                          tp_symbol** pre, double* err);
/* Release a symbol (NULL is accepted).  Waits for the device, then returns the symbol's device
 * blocks to the context that built it: that context's later builds reuse them (no allocation call
 * once the blocks exist, at most 1 GiB of idle blocks kept), and they are freed with the last of the
 * context and its symbols.  The symbol may outlive its context. */
tp_status tp_symbol_free(tp_symbol* sym);

/* State operator of eqn:State / eqn:L_alp_state, y = beta A^-alpha u: the exponential sum
 * beta rho^-alpha ~ sum_k w_k exp(-tau_k rho) (canonical rank op_terms, least-squares fit; beta is
 * desc->c_neg, desc->c_pos is ignored), for use with tp_apply (with desc->directional:
 * beta / rho', the state of the directionally fractional operator).  err (host, may be NULL)
 * receives its measured max relative error. */
tp_status tp_state_symbol_build(tp_ctx* ctx, const tp_symbol_desc* desc, tp_symbol** state,
                                double* err);
/* rank (host): canonical rank of the symbol; err (host): its measured error. */
tp_status tp_symbol_info(const tp_symbol* sym, int32_t* rank, double* err);
/* Values of the symbol at `count` multi-indices idx (device, count x d int32,
 * 0-based, row i = point i) into out (device, count doubles).  A point outside the
 * grid gives NaN. */
tp_status tp_symbol_eval(tp_ctx* ctx, const tp_symbol* sym, int32_t count,
                         const int32_t* idx, double* out);

/* ---------------------------------------------------------------------------
 * Tensor arithmetic
 * ------------------------------------------------------------------------- */

/* Exact Tucker form of a canonical tensor: orthonormal bases of the factor
 * column spans, core = sum_k w_k (x)_l (Q_l^T f_k^(l)).  If tol > 0 the result
 * is then HOSVD-truncated at tol (relative).  out->cap bounds the ranks. */
tp_status tp_from_cp(tp_ctx* ctx, const tp_cp* b, tp_tensor* out, double tol);

/* y = trunc(F (s (.) F x)): the low-rank matrix-vector product of
 * eqn:Lap3DtimesX with the canonical symbol s, truncated to relative accuracy
 * tol and mode ranks <= cap.  The truncation works in spectral coordinates
 * (F is orthogonal per mode, so it commutes with the truncation) by a sketched
 * HOSVD: Khatri-Rao products of the test matrices span each mode, their
 * orthonormal bases compress the product, and an exact HOSVD of the compressed
 * core selects the ranks.  sketch->q must exceed the output rank.  y may alias x. */
tp_status tp_apply(tp_ctx* ctx, const tp_symbol* sym, const tp_tensor* x, tp_tensor* y,
                   double tol, int32_t cap, const tp_sketch* sketch);

/* y = trunc(sum_i coef[i] F(s_i (.) F xs[i])) for count <= 8 terms; syms[i] == NULL stands
 * for the identity.  The whole sum is truncated at once by the sketched HOSVD of tp_apply,
 * so the truncation error is relative to the norm of the sum (the PCG residual update
 * R - alpha fun(P) uses it).  syms, xs, coef: host arrays of count entries.  y may alias
 * any xs[i]. */
tp_status tp_apply_sum(tp_ctx* ctx, int32_t count, const tp_symbol* const* syms,
                       const tp_tensor* const* xs, const double* coef, tp_tensor* y, double tol,
                       int32_t cap, const tp_sketch* sketch);

/* <x, F(s (.) F y)> without truncation, from the Gram matrices G_k = (F X)^T diag(s_k) (F Y)
 * of every symbol term and the cores (out is host). */
tp_status tp_inner_sym(tp_ctx* ctx, const tp_tensor* x, const tp_symbol* sym, const tp_tensor* y,
                       double* out);

/* y = trunc(sum_i coef[i] * xs[i]) by the exact HOSVD of the sum (Sec. 5, RHOSVD
 * step of Algorithm alg:pcg's trunc): factors are concatenated, orthonormalised,
 * the block core is projected and its mode Gram matrices are diagonalised in FP64.
 * coef: host, count doubles; xs: host array of count tensor pointers.  y may
 * alias any xs[i]. */
tp_status tp_truncate(tp_ctx* ctx, int32_t count, const double* coef,
                      const tp_tensor* const* xs, tp_tensor* y, double tol, int32_t cap);

/* <x, y> (Euclidean, Sec. 3.1 with M = I) from factor Gram matrices and the
 * cores; out is host. */
tp_status tp_inner(tp_ctx* ctx, const tp_tensor* x, const tp_tensor* y, double* out);

/* For callers that cannot allocate device memory or wait on the host (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): <x, y> as tp_inner computes it
 * (same kernels, same arguments), with every temporary (factor Gram matrices, FP64 cores,
 * contraction intermediates, partial sums) in a fixed device array of TP_NOALLOC_SCRATCH_BYTES per
 * GPU, allocated when the library is loaded and held until the process ends, and the result
 * written to out_dev (device, one double) without synchronising the stream.  The call allocates
 * nothing, waits for nothing and records no event.
 * Limit: the temporaries of x and y must fit the array: 8 bytes times (sum_l rank_x[l] rank_y[l] +
 * prod rank_y + 2 prod rank_x + rank_x[0] rank_y[1] rank_y[2] + rank_x[0] rank_x[1] rank_y[2] + 257),
 * each term rounded up to 256 bytes (every 3D pair with ranks <= 64 fits); beyond it the call returns
 * TP_EINVAL before enqueuing anything.  Every call on one GPU shares that GPU's array and it keeps
 * the last call's contents (every temporary is written before it is read): calls that overlap on one
 * GPU (several streams or threads, or contexts on the same device) race and must be serialised by
 * the caller. */
#define TP_NOALLOC_SCRATCH_BYTES (16u << 20)
tp_status tp_inner_noalloc(tp_ctx* ctx, const tp_tensor* x, const tp_tensor* y, double* out_dev);

/* Values of x on the sub-grid rows[0] x rows[1] (x rows[2]) (device int32 arrays
 * of m[l] 0-based indices) into out (device, m[0]*m[1]*m[2] doubles, column-major).
 * An index outside [0, n[l]) gives NaN in the points it enters. */
tp_status tp_eval_grid(tp_ctx* ctx, const tp_tensor* x, const int32_t* const* rows,
                       const int32_t* m, double* out);

/* ---------------------------------------------------------------------------
 * PCG  (Algorithm alg:pcg)
 * ------------------------------------------------------------------------- */
typedef enum {
  TP_STOP_ERROR = 0,     /* ||Z|| <= tau ||X||, Z = trunc(pre(R)) the preconditioned residual */
  TP_STOP_RESIDUAL = 1   /* ||R|| <= tau ||B||, the relative residual of the Sec. 6 iteration counts */
} tp_stop_rule;

typedef struct {
  double tau;        /* stopping tolerance of stop_rule */
  int32_t kmax;      /* iteration limit (paper: 100) */
  double trunc_tol;  /* relative truncation tolerance epsilon of trunc */
  int32_t cap;       /* mode-rank cap of every iterate (<= x->cap) */
  int32_t true_residual; /* nonzero: also compute ||B - A_2 X||/||B|| */
  int32_t stop_rule; /* tp_stop_rule */
  int32_t recursive_residual; /* 0: R = trunc(B - fun(X)) recomputed each step (default);
                               * 1: R = trunc(R - alpha trunc(fun(P))) as printed in Algorithm
                               * alg:pcg (it does not see the truncation error of X, so with
                               * TP_STOP_RESIDUAL it reaches tau below the floor set by it) */
  int32_t spectral_domain;    /* 1: run the iteration in sine coordinates: the right-hand side's
                               * factors are transformed once, every iterate keeps F V as its
                               * factors (F orthogonal: inner products and truncations unchanged),
                               * and only X is transformed back at the end; the products skip
                               * their two transforms.  Same result up to rounding. */
  int32_t warm_start;         /* 1: x holds the initial guess X^(0) of Algorithm alg:pcg on entry
                               * (mode ranks <= cap; ranks 0 = zero), R^(0) = trunc(B - fun(X^(0)));
                               * 0: X^(0) = 0 and x is output only */
} tp_pcg_opts;

typedef struct {
  int32_t iters;
  int32_t status;    /* tp_status of the solve */
  int32_t rank[3];   /* ranks of the returned X */
  double rel_res;    /* ||R||/||B|| of the recursive residual */
  double true_rel_res;  /* only if requested, else -1 */
  double op_applies; /* number of operator/preconditioner products */
  double err_est;    /* the stopping quantity of the returned X: ||Z||/||X|| or ||R||/||B|| */
} tp_pcg_info;

/* Solve A_2 x = b with the operator symbol `op`, the preconditioner symbol `pre`
 * and X0 = 0.  Each step: alpha = <R,Z>/<P,fun(P)> with fun(P) kept exact, X = trunc(X + alpha P),
 * R = trunc(B - fun(X)) (recomputed, one sketched sum; or the recursive update of
 * opts->recursive_residual), stop when ||R|| <= tau ||B||
 * (TP_STOP_RESIDUAL), Z = trunc(pre(R)), stop when ||Z|| <= tau ||X|| (TP_STOP_ERROR),
 * P = trunc(Z + beta P).  Iterates are Tucker tensors (the mixed Tucker-canonical route of
 * Sec. 5); every update is truncated as in Algorithm alg:pcg.  x->prec selects
 * the arithmetic; op and pre must have been built with that precision.
 * Without convergence (kmax reached, or the estimate grown 8-fold over its minimum or not
 * improved for 5 steps: the floor set by the working precision or by the rank cap) the call
 * returns TP_ENOCONV and x holds the iterate with the smallest estimate; TP_ERANK: converged
 * but some truncation hit the cap. */
tp_status tp_pcg_solve(tp_ctx* ctx, const tp_symbol* op, const tp_symbol* pre,
                       const tp_cp* b, tp_tensor* x, const tp_pcg_opts* opts,
                       const tp_sketch* sketch, tp_pcg_info* info);

/* Workspace.  tp_workspace_query: a conservative estimate (host out, bytes) of the workspace
 * that tp_symbol_build(desc) followed by tp_pcg_solve with opts, a sketch of width sketch_q and a
 * right-hand side of canonical rank rhs_rank needs (the largest transient arrays of the product,
 * the symbol inner products and the sums, plus the iteration's tensors).  Needs no context.
 * tp_workspace_peak: the high-water mark of ctx's workspace since tp_create or the last reset
 * (reset != 0 restarts it from the current use). */
tp_status tp_workspace_query(const tp_symbol_desc* desc, const tp_pcg_opts* opts, int32_t sketch_q,
                             int32_t rhs_rank, size_t* bytes);
tp_status tp_workspace_peak(tp_ctx* ctx, int32_t reset, size_t* peak);

/* Many independent control problems (arrays of `count` entries, all host arrays of structs
 * whose tensor/sketch pointers are device memory): problem i builds its symbols from descs[i]
 * and solves into xs[i] with opts[i] and sks[i]; infos[i] receives its result.  The problems
 * are spread over `streams` (1..16) concurrent HIP streams at default priority, each with its
 * own workspace of workspace_per_stream bytes (0 = 2 GiB).  The worker streams and workspaces are
 * created on first use and kept in ctx for later calls (more are added when a call asks for more
 * streams; all are replaced when the workspace size changes; tp_destroy releases them).  A
 * worker's symbols are built in its workspace, so a call allocates no device memory per problem.
 * Problems whose descriptors are equal field by field (several right-hand sides of one operator)
 * share one build of the symbols, made on ctx before the workers start.  Returns the first hard
 * error (TP_ERANK / TP_ENOCONV of a problem are reported only in its info). */
tp_status tp_pcg_solve_batched(tp_ctx* ctx, int32_t count, const tp_symbol_desc* descs,
                               const tp_cp* bs, tp_tensor* xs, const tp_pcg_opts* opts,
                               const tp_sketch* sks, tp_pcg_info* infos, int32_t streams,
                               size_t workspace_per_stream);

/* ---------------------------------------------------------------------------
 * Kernel-level entry points (for parity tests of single steps)
 * ------------------------------------------------------------------------- */

/* Orthonormal DST-I (F_jk = sqrt(2/(n+1)) sin(pi j k/(n+1))) of `cols` columns
 * of length n: in/out device, column-major with ld n, FP64 (prec 0) or FP32
 * (prec 1).  in may equal out. */
tp_status tp_dst(tp_ctx* ctx, int32_t n, int32_t cols, int32_t prec, const void* in, void* out);

/* Symmetric eigendecomposition (cyclic Jacobi, FP64) of `count` K x K matrices
 * a (device, count*K*K, column-major): eigenvalues descending into w (device,
 * count*K), eigenvectors into v (device, count*K*K).  K <= 256. */
tp_status tp_syev(tp_ctx* ctx, int32_t K, int32_t count, const double* a, double* w, double* v);

/* Eigenpairs of `count` (<= 24) positive semidefinite K x K matrices g (device, count*K*K,
 * column-major, FP64) by the solvers of the truncations (Sec. 5, the HOSVD's side-matrix
 * decompositions): eigenvalues descending into w (device, count*K, zero past the rank),
 * eigenvectors into v (device, count*K*K, zero columns past the rank), ranks into rank (host,
 * count) and the eigenvalue mass not represented into rest (host, count, may be NULL).
 * cut = 0: pivoted Cholesky, then one-sided Jacobi (rank = the Cholesky's numerical rank, rest =
 * the trace it left).  cut >= 1e-13 with K <= 64: reduction to tridiagonal form, eigenvalues by
 * multisection, eigenvectors by twisted factorisations; eigenpairs with eigenvalue <= cut * trace
 * are dropped (rank = the number kept, rest = their sum); a matrix whose kept eigenvectors are not
 * orthogonal to 1e-10 (clustered eigenvalues) is solved by the Jacobi path instead.  K <= 256. */
tp_status tp_gram_eig(tp_ctx* ctx, int32_t K, int32_t count, const double* g, double* w, double* v,
                      double cut, int32_t* rank, double* rest);

/* 1D eigenvalues lambda_k = (4/h^2) sin^2(pi k h/2), h = 1/(n+1), into out
 * (device, n doubles). */
tp_status tp_lambda(tp_ctx* ctx, int32_t n, double* out);

/* ---------------------------------------------------------------------------
 * Measurement
 * ------------------------------------------------------------------------- */

/* Kernel classes timed when profiling is on: one class per kernel, whoever launches it (the
 * contraction kernel's four type instantiations count apart). */
typedef enum {
  TP_PROF_GEMM_F64 = 0,      /* k_gemm_mfma, FP64: Gram, sketch, projection and core contractions */
  TP_PROF_GEMM_F32 = 1,      /* k_gemm_mfma, FP32 operands and results (mixed path) */
  TP_PROF_GEMM_F32_F64 = 2,  /* k_gemm_mfma, FP32 operands accumulated into FP64 results */
  TP_PROF_GEMM_F64_F32 = 3,  /* k_gemm_mfma, FP64 operands rounded into FP32 results */
  TP_PROF_DST_F64 = 4,       /* k_dst1, FP64 columns */
  TP_PROF_DST_F32 = 5,       /* k_dst1, FP32 columns */
  TP_PROF_SYEV = 6,          /* k_syev / k_syev_small: two-sided Jacobi of tp_syev */
  TP_PROF_CHOL = 7,          /* k_pchol: pivoted Cholesky of Gram matrices (orthonormal bases) */
  TP_PROF_PSD_EIG = 8,       /* k_psd_eig: Gram eigensolver (HOSVD ranks and bases, fit normal equations) */
  TP_PROF_NS = 9,            /* k_ns_isqrt: Newton-Schulz inverse square root (second orthonormalisation) */
  TP_PROF_GEMM_REDUCE = 10,  /* k_gemm_reduce: split-K partial sums of the contractions (all types) */
  TP_PROF_PSD_TRI = 11,      /* k_psd_tri: Gram eigensolver by tridiagonal reduction (HOSVD ranks and bases) */
  TP_PROF_GEMM_F32_SPLIT64 = 12  /* k_gemm_mfma, FP32 operands accumulated in FP32 per split of K (at most
                                    512 long), the splits summed into FP64 results (sketches, operator
                                    inner products of the mixed path) */
} tp_prof_class;

/* Contraction kernels, process-wide (set it while no call of the library runs):
 *   mfma = 1 (default): FP32 / FP64 matrix-core tiles;
 *   mfma = 0: FMA tiles (the same results up to rounding order);
 *   mfma = 2: as 1, but the contractions with FP32 operands, FP32 accumulation and FP32 results
 *     (the sketch, projection and core contractions of the mixed path's products and truncations)
 *     take split-BF16 products on the BF16 matrix cores, accumulated in FP32: each operand
 *     x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and a product is hi hi' + hi lo' + lo hi'
 *     (relative error at most about 3 * 2^-16 per product, from the dropped lo lo' and the
 *     remainders |x - hi - lo| <= 2^-16 |x|, instead of the FP32 product's 2^-24).  The FP32
 *     contractions that sum into FP64 (inner products, the sketches' FP64 chunk sums) and all FP64
 *     contractions are unchanged.
 * Returns TP_EINVAL for any other value (the mode is then unchanged). */
tp_status tp_gemm_mode(int32_t mfma);

/* enable != 0: record a HIP event pair around every launch of the classes above on the
 * context stream (and reset the totals); enable == 0: stop recording. */
tp_status tp_profile(tp_ctx* ctx, int32_t enable);
/* Totals since tp_profile(ctx, 1) for class cls (host outputs, any may be NULL):
 * summed event time in ms, launch count, algorithmic flops and algorithmic bytes. */
tp_status tp_profile_read(tp_ctx* ctx, int32_t cls, double* ms, double* launches, double* flops,
                          double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* TP_H */
