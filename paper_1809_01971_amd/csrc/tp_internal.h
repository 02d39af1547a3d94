// Internal declarations shared by the kernel and host translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace tpk {

// Face-split operand: F[row, c] = X1[row + ld1*(c % r1)] * X2[row + ld2*(c / r1)].
// It stands for the Hadamard products u_k (.) x_j of the low-rank matrix-vector
// product without forming them (weights of the terms are folded into X2 beforehand).
template <typename T>
struct FaceSplit {
  const T* x1 = nullptr;
  const T* x2 = nullptr;
  int ld1 = 0, ld2 = 0, r1 = 1;
};

// op(A) is M x K, op(B) is K x N, C is M x N, all column-major.
// Batch b uses A + (b / divA) * sA, B + (b / divB) * sB, C + b * sC.
// The matrix cores accumulate in Tacc.  With FP32 operands, an FP64 result and FP32 accumulation
// (TA = TB = float, TC = double, Tacc = float) every split of K is at most kF32Chunk long and the
// splits' partial sums, the scaling and the beta term are added in FP64.
template <typename TA, typename TB, typename TC, typename Tacc>
struct GemmArgs {
  int M = 0, N = 0, K = 0, batch = 1;
  Tacc alpha = 1, beta = 0;
  const TA* A = nullptr; int lda = 0; long sA = 0; int divA = 1; bool tA = false; bool fsA = false; FaceSplit<TA> FA;
  const TB* B = nullptr; int ldb = 0; long sB = 0; int divB = 1; bool tB = false; bool fsB = false; FaceSplit<TB> FB;
  TC* C = nullptr; int ldc = 0; long sC = 0;
  // split-K: `splits` workgroups share each output tile over K; partial sums go to `part`
  // (batch * splits * M * N elements) and a second kernel reduces them.
  int splits = 1; int kchunk = 0; Tacc* part = nullptr;
};

// mid (optional): an event recorded between the contraction and its split-K reduction, so that
// the two kernels can be timed apart.
template <typename TA, typename TB, typename TC, typename Tacc>
hipError_t gemm(const GemmArgs<TA, TB, TC, Tacc>& g, hipStream_t s, hipEvent_t mid = nullptr);

// Up to kGemmGroup independent products with the same operand kinds (plain, transposed or
// face-split A and B) in one launch, and their split-K reductions in a second one.  The group
// travels in the kernel arguments; z0 / r0 (prefix sums of batch x splits and of the split
// products' batches) are set by the launch.
constexpr int kGemmGroup = 3;
constexpr int kF32Chunk = 512;
template <typename TA, typename TB, typename TC, typename Tacc>
struct GemmGroup {
  GemmArgs<TA, TB, TC, Tacc> g[kGemmGroup];
  int z0[kGemmGroup + 1];
  int r0[kGemmGroup + 1];
  int count;
};
template <typename TA, typename TB, typename TC, typename Tacc>
hipError_t gemm_group(const GemmArgs<TA, TB, TC, Tacc>* g, int count, hipStream_t s, hipEvent_t mid = nullptr);
// Matrix-core (MFMA) tiles on (default) or the FMA tiles.
bool gemm_use_mfma();
void gemm_set_mfma(int mode);  // 0 FMA tiles, 1 matrix cores, 2 with split-BF16 FP32 products

// Orthonormal DST-I on `cols` columns of length n = N-1 (N a power of two).
// tab holds cos(pi m/N), sin(pi m/N), m = 0..N-1, interleaved (tab64 the same in double; FP32
// columns are transformed in FP64 arithmetic with it).  N > 16384 needs `work`: cols * N/2
// complex values of the arithmetic type (16 bytes each for FP32 columns) in global memory.
template <typename T>
hipError_t dst1(int N, int cols, const T* in, int ldin, T* out, int ldout, const T* tab, const double* tab64,
                void* work, hipStream_t s);
// The same transform of up to kDstJobs column blocks of one length in one launch (N <= 16384):
// block i maps cols columns of in (ld ldin) to out (ld ldout); in == out is allowed.  The jobs
// travel in the kernel arguments; blk0 is set by the launch.
constexpr int kDstJobs = 6;
template <typename T>
struct DstJob { const T* in; T* out; int cols; int ldin; int ldout; int blk0; };
template <typename T>
hipError_t dst1_batched(int N, const DstJob<T>* jobs, int count, const T* tab, const double* tab64, hipStream_t s);

template <typename T>
hipError_t dst_table(int N, T* tab, hipStream_t s);

// Gram and eigen problems up to this size are kept in LDS; larger ones (up to 256) use global scratch.
constexpr int kGramLds = 128;

// Job descriptors of the batched one-workgroup-per-matrix kernels travel by value in the kernel
// arguments (no staging copy): at most kBatchJobs per launch (24 descriptors of at most 72 bytes).
constexpr int kBatchJobs = 24;
template <typename J>
struct JobBatch { J j[kBatchJobs]; };

// Batched symmetric Jacobi eigensolver, FP64.  Matrix b: K[b] x K[b] at a[b] (ld K[b]);
// eigenvalues (descending) to w[b], eigenvectors to v[b] (ld K[b]).
// Matrices larger than 128 need `work` (Kp x Kp doubles, Kp = K rounded up to even) in global memory.
// tol: the sweeps stop once the off-diagonal Frobenius norm is <= tol * ||A||_F (0 = 1e-14).
struct EigJob { int K; const double* a; double* w; double* v; double* work; double tol; };
hipError_t syev_batched(const JobBatch<EigJob>& jobs, int count, int Kmax, hipStream_t s);

// Batched rank-revealing pivoted Cholesky of Gram matrices: W = P R^-1 (K x q, ld K), q to *q.
// Matrices larger than 64 need `work` (2 K^2 doubles) in global memory.
struct CholJob { int K; double tol; const double* g; double* w; int* q; double* work; };
hipError_t pchol_batched(const JobBatch<CholJob>& jobs, int count, int Kmax, hipStream_t s);

// Batched inverse square root W = G^(-1/2) (K x K, ld K) of Gram matrices near the identity by
// the coupled Newton-Schulz iteration, K <= kNsMax; *ok = 0 (W untouched) when ||G - I||_F > 1/2
// or it has not converged.
constexpr int kNsMax = 64;
struct NsJob { int K; const double* g; double* w; int* ok; };
hipError_t ns_isqrt_batched(const JobBatch<NsJob>& jobs, int count, int Kmax, hipStream_t s);

// Batched eigendecomposition of positive semidefinite Gram matrices (pivoted Cholesky, then
// one-sided Jacobi on R^T).  Per job: eigenvalues descending to w (K entries, zero past the
// numerical rank q), eigenvectors to v (K x K, ld K, zero columns past q), q to *q and the
// trace left in the Schur complement when the Cholesky stopped to *rest.  Cholesky stops at
// pivots <= ctol * max diag(G); a column pair is rotated while |x_p.x_r| > jtol |x_p||x_r|.
// Matrices larger than 64 need `work` (2 K^2 doubles) in global memory.
struct PsdJob { int K; const double* g; double* w; double* v; int* q; double* rest; double* work; double ctol; double jtol; };
hipError_t psd_eig_batched(const JobBatch<PsdJob>& jobs, int count, int Kmax, hipStream_t s);

// The same eigenpairs by reduction to tridiagonal form (K <= kTriMax, one workgroup per matrix,
// everything in LDS): Householder reduction, multisection on qd Sturm counts of a positive
// definite L D L^T, twisted-factorisation eigenvectors.  The job's fields mean: ctol = cut,
// eigenpairs with eigenvalue <= cut * trace(G) are dropped (q counts the others, rest = the
// dropped eigenvalues' sum); jtol = the largest tolerated |Z^T Z - I| over the kept eigenvectors.
// When the check fails the kernel writes q = -1 and nothing else for that job (the caller then
// runs psd_eig_batched on it).
constexpr int kTriMax = 64;
hipError_t psd_tri_batched(const JobBatch<PsdJob>& jobs, int count, int Kmax, hipStream_t s);

// Elementwise helpers.
template <typename TI, typename TO>
hipError_t convert(const TI* in, TO* out, long count, hipStream_t s);
// Up to kConvJobs conversions out[j][i] = (TO) in[j][i], i < count[j], in one launch; jobs with
// count <= 0 are skipped.
constexpr int kConvJobs = 4;
template <typename TI, typename TO>
struct ConvBatch {
  const TI* in[kConvJobs];
  TO* out[kConvJobs];
  long count[kConvJobs];
  int n = 0;
  // the call sites add at most kConvJobs (a core and three factors, or three modes); one more
  // marks the batch invalid, and convert_batch then fails instead of writing past the table
  void add(const TI* i, TO* o, long c) {
    if (n >= kConvJobs) { n = kConvJobs + 1; return; }
    in[n] = i; out[n] = o; count[n] = c; ++n;
  }
};
template <typename TI, typename TO>
hipError_t convert_batch(const ConvBatch<TI, TO>& b, hipStream_t s);
// Copy a rows x cols column-major block (lds in/out) with scale.
template <typename TI, typename TO>
hipError_t copy2d(int rows, int cols, const TI* in, int ldin, TO* out, int ldout, double scale, hipStream_t s);
// out[i,j,l] (dims d0,d1,d2 packed) -> permuted: perm gives which input axis becomes output axis 0,1,2.
template <typename T>
hipError_t permute3(const T* in, int d0, int d1, int d2, T* out, int p0, int p1, int p2, hipStream_t s);
// Columns scaled: out[:,j] = in[:,j] * scale[j] (rows x cols, ld), in place allowed.
hipError_t scale_cols_d(double* a, int rows, int cols, int ld, const double* scale, hipStream_t s);
// out[:, j] = in[:, j] * w[j] (rows x cols, both with leading dimension rows), the product in FP64
template <typename T>
hipError_t scale_cols_copy(const T* in, int rows, int cols, const double* w, T* out, hipStream_t s);
// scale_cols_copy of up to 3 matrices (the modes of a symbol) in one launch.
template <typename T>
struct ScaleBatch {
  const T* in[3];
  T* out[3];
  int rows[3], cols[3];
  const double* w[3];
  int count = 0;
};
template <typename T>
hipError_t scale_cols_copy_batch(const ScaleBatch<T>& b, hipStream_t s);
// W = E[:, 0:q] * diag(1/sqrt(w)) for the leading q eigenpairs; K rows, ld K.
hipError_t eig_inv_sqrt(const double* E, const double* w, int K, int q, double* W, hipStream_t s);
// out[0] = sum(a[i]*b[i]) in FP64; part: device scratch of 256 doubles for per-workgroup sums.
template <typename T>
hipError_t dot(const T* a, const T* b, long count, double* out, double* part, hipStream_t s);
// Face-split dense materialisation: out[(b,c), k] = X2[b,k] * X3[c,k] (q2*q3 x R), used for CP cores.
hipError_t khatri_rao_d(const double* X2, int q2, const double* X3, int q3, int R, double* out, hipStream_t s);
// t[i, col] = sum_j T1[i + rm*(j + ro*col)] * A[j + ro*col]
template <typename T>
hipError_t contract_mid(const T* T1, const T* A, int rm, int ro, int ncol, T* t, hipStream_t s);
// Gather rows: out[p, c] = in[rows[p] + ld*c] for rows[p] in [0, ld) (the factor's n rows), NaN otherwise
template <typename T>
hipError_t gather_rows(const T* in, int ld, const int* rows, int m, int cols, double* out, hipStream_t s);

// Symbol construction.
// lambda_k^power, lambda_k = (4/h^2) sin^2(pi k h/2), k = 1..n (power != 1: the spectra of the
// directionally fractional operator)
hipError_t lambda_1d(int n, double* out, hipStream_t s, double power = 1.0);
// exponential-sum factor columns for a mode with eigenvalues lam (n) and exponents tau (K):
// E[:,k] = exp(-tau_k lam), times lam when withLam (the Lemma 4.1 factor).
template <typename T>
hipError_t expfactors(const double* lam, int n, const double* tau, int K, T* E, int ldE, int withLam, hipStream_t s);
// Several of the above in one launch (the factors of a symbol's modes and blocks).
constexpr int kExpJobs = 12;
template <typename T>
struct ExpJob { const double* lam; const double* tau; T* E; int n, K, ldE, withLam; };
template <typename T>
struct ExpBatch {
  ExpJob<T> j[kExpJobs];
  int count = 0;
  bool add(const double* lam, int n, const double* tau, int K, T* E, int ldE, int withLam) {
    if (count >= kExpJobs) return false;
    j[count++] = ExpJob<T>{lam, tau, E, n, K, ldE, withLam};
    return true;
  }
};
template <typename T>
hipError_t expfactors_batch(const ExpBatch<T>& b, hipStream_t s);
// 1D spectra of several grids (lambda_1d each) in one launch.
constexpr int kLamJobs = 6;
struct LamBatch {
  double* out[kLamJobs];
  int n[kLamJobs];
  double power[kLamJobs];
  int count = 0;
  bool add(int nn, double* o, double p) {
    if (count >= kLamJobs) return false;
    out[count] = o; n[count] = nn; power[count] = p; ++count;
    return true;
  }
};
hipError_t lambda_batch(const LamBatch& b, hipStream_t s);
// The function a least-squares exponential sum approximates, in rho = rho0 y:
//   kind 0 (operator, Lemma 4.1): g = (cn rho^-alpha + [fitpos] cp rho^beta) / rho, the part of
//          s = c0 + cn rho^-alpha + cp rho^beta that is fitted (c0 and a beta = 1 term are exact);
//   kind 1 (preconditioner): 1 / s;   kind 2 (state): cn rho^-alpha.
struct SymFn { double c0, cn, cp, alpha, beta; int fitpos; };
// least-squares design matrix for candidate c: rows y_j (m), columns t_k (K):
// A[j,k] = exp(-t_k y_j) / f(y_j).  Candidates stacked.
struct FitCand { double a, b; };
hipError_t fit_design(int kind, const SymFn& f, double rho0, double B, int K, int m, const FitCand* cands_dev,
                      int ncand, double* A, double* tvec, hipStream_t s);
// max relative error of the fitted sums over m log-spaced points, per candidate; part: device
// scratch of 16 ncand doubles (partial maxima)
hipError_t fit_error(int kind, const SymFn& f, double rho0, double B, int K, const double* t, const double* w,
                     int ncand, int m, double* err, double* part, hipStream_t s);
hipError_t sinc_g_nodes(double alpha, double cneg, double cpos, double rho0, int kl, int kr, double hh,
                        double* tau, double* w, hipStream_t s);
// out = c0 + rho sum_k w_k exp(-tau_k rho) (opkind 0) or sum_k w_k exp(-tau_k rho) at multi-indices
// (count x d, 0-based; n: host, grid sizes; points outside the grid give NaN)
hipError_t symbol_eval(int d, const int* idx, int count, const int* n, const double* lam0, const double* lam1,
                       const double* lam2, int opkind, int K, const double* tau, const double* w, double c0,
                       double* out, hipStream_t s);
// out = sum_k w_k prod_m F_m[i_m, k] for a canonical symbol with factors F_m (n_m x R, ld n_m)
template <typename T>
hipError_t cp_eval(int d, const int* idx, int count, const int* n, const T* const* F, int R, const double* w,
                   double* out, hipStream_t s);

hipError_t fit_scale(int K, int nc, double* G, double* b, double* D, hipStream_t s);
hipError_t fit_solve(int K, int nc, const double* ev, const double* E, const double* b, const double* D, double cut,
                     double* w, hipStream_t s);
hipError_t scale(double* a, long n, double sc, hipStream_t s);

}  // namespace tpk
