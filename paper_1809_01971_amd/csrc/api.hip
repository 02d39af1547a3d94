// Host side of the C ABI declared in include/tp.h.
//
// Orchestrates the kernels of kernels.hip on the context's stream.  Device memory
// for intermediate results comes from one workspace allocated at tp_create and
// handed out by a stack allocator; mode ranks are read back to the host after
// each rank-revealing step (ranks decide the shapes of the following launches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "../../include/tp.h"
#include "tp_internal.h"

using namespace tpk;

namespace {

thread_local std::string g_err;

tp_status fail(tp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(...)                                                                         \
  do {                                                                                      \
    hipError_t e_ = (__VA_ARGS__);                                                          \
    if (e_ != hipSuccess) return fail(TP_EHIP, "%s failed: %s (%s:%d)", #__VA_ARGS__,     \
                                      hipGetErrorString(e_), __FILE__, __LINE__);         \
  } while (0)

#define TPCHK(...)                         \
  do {                                     \
    tp_status s_ = (__VA_ARGS__);          \
    if (s_ != TP_OK) return s_;            \
  } while (0)

constexpr int kMaxRank = 256;   // eigensolver limit: every Gram is at most 256 x 256
constexpr int kMaxCap = 128;    // sums of two iterates stay within kMaxRank
constexpr int kMaxSketch = 192; // sketch width

}  // namespace

// ------------------------------------------------------------------------------ no-allocation scratch
// Temporaries of tp_inner_noalloc live in this fixed array: one copy per GPU the library runs on,
// held until the process ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in symbol); it uses the device address that hipGetSymbolAddress returned for the
// current device, recorded once per device by tp_create.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

// Device blocks of freed symbols, kept for the next builds of the same context: a loop that builds
// and frees its symbols for every solve makes no allocation call and no device-wide wait once the
// blocks exist.  Shared by the context and every symbol built in it, so a symbol freed after its
// context still returns its blocks; the last owner frees them.  A block is handed out again only to
// a later build of the same context, on its stream; tp_symbol_free waits for the device first, so
// no queued work still reads a block that goes back to the pool.
struct SymPool {
  std::mutex mu;
  std::multimap<size_t, void*> idle;  // size in bytes -> block
  size_t idle_bytes = 0;
  static constexpr size_t kMaxIdle = size_t(1) << 30;  // beyond this, freed blocks are released
  ~SymPool() {
    if (!idle.empty()) (void)hipDeviceSynchronize();
    for (auto& kv : idle) (void)hipFree(kv.second);
  }
};

struct tp_ctx {
  int device = 0;
  std::shared_ptr<SymPool> sympool = std::make_shared<SymPool>();
  char* scratch = nullptr;       // device address of `scratch` on this context's device
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_size = 0, ws_top = 0;
  size_t ws_peak = 0;            // high-water mark of ws_top (tp_workspace_peak)
  // batched solves: symbols of a worker live in its workspace (no allocation call, no device-wide
  // synchronisation when they are freed); the workers are kept for later calls
  bool sym_arena = false;
  std::vector<tp_ctx*> workers;
  std::vector<hipStream_t> worker_streams;
  size_t worker_ws = 0;
  double* host = nullptr;        // pinned host scratch (kHost doubles)
  double* hmap = nullptr;        // mapped, coherent pinned host memory (kMap doubles) that small
  double* dmap = nullptr;        //   kernel results (ranks, eigenvalues, inner products) go to; its device address
  std::map<int, double*> tab64;
  std::map<int, float*> tab32;
  std::map<int, double*> ones64;  // all-ones columns (identity symbol), per grid size
  std::map<int, float*> ones32;
  double* unit_w = nullptr;
  // set inside a spectral-domain PCG solve: tensor factors are already in sine coordinates, so
  // products and symbol inner products skip the forward and inverse transforms
  bool spectral = false;
  // optional per-kernel-class timing with HIP events on the context stream
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  struct Rec { int cls; size_t e0, e1; double flops, bytes; };
  std::vector<Rec> recs;
  double prof_ms[16] = {0}, prof_n[16] = {0}, prof_flops[16] = {0}, prof_bytes[16] = {0};  // by PC_* class
  static constexpr size_t kHost = 1 << 16;
  static constexpr size_t kMap = 4096;
  static constexpr int kJobs = 64;
};

struct tp_symbol {
  int d = 0, n[3] = {0, 0, 0}, prec = 0;
  int kind = 0;          // 0: operator rho*g, 1: preconditioner
  int K = 0;             // exponentials
  int R = 0;             // canonical rank (d*K for the operator, +1 with a constant term)
  double err = 0;
  double pmin = 1.0;     // preconditioner: smallest p s on the checked points (rank-r lattice)
  double c0 = 0;         // constant term of the operator symbol (factors all ones)
  double wexact = 0;     // weight of the exact tau = 0 exponential (c_pos rho for beta = 1)
  int tucker = 0;        // > 0: rank-r recompressed preconditioner (general canonical factors)
  double sinc_h = 0;     // step of the sinc rule (TP_SYM_SINC)
  bool arena = false;    // memory in a batched worker's workspace (nothing to free)
  std::shared_ptr<SymPool> pool;  // where the blocks in `owned` go back to
  double* weights = nullptr;   // R (device)
  void* factors[3] = {nullptr, nullptr, nullptr};  // n x R (device, T)
  void* factors_w[3] = {nullptr, nullptr, nullptr};  // the same with column k scaled by weights[k]
  double* tau = nullptr;       // K
  double* w = nullptr;         // K
  double* lam[3] = {nullptr, nullptr, nullptr};
  std::vector<std::pair<void*, size_t>> owned;  // blocks of `pool` (address, bytes)
};

namespace {

// ------------------------------------------------------------------------------ workspace
struct Mark { size_t top; };

template <typename T>
tp_status wsalloc(tp_ctx* c, size_t count, T** out) {
  size_t bytes = ((count * sizeof(T)) + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  if (c->ws_top + bytes > c->ws_size)
    return fail(TP_ENOMEM, "workspace exhausted: need %zu more bytes (top %zu of %zu)", bytes, c->ws_top, c->ws_size);
  *out = reinterpret_cast<T*>(c->ws + c->ws_top);
  c->ws_top += bytes;
  if (c->ws_top > c->ws_peak) c->ws_peak = c->ws_top;
  return TP_OK;
}
struct WsScope {
  tp_ctx* c;
  size_t top;
  explicit WsScope(tp_ctx* cc) : c(cc), top(cc->ws_top) {}
  ~WsScope() { c->ws_top = top; }
};

// ------------------------------------------------------------------------------ profiling
// Kernel classes reported by tp_profile_read.
// One class per kernel (template instantiations of the contraction count apart), whoever calls it.
enum { PC_GEMM_F64 = 0, PC_GEMM_F32 = 1, PC_GEMM_F32_F64 = 2, PC_GEMM_F64_F32 = 3, PC_DST_F64 = 4, PC_DST_F32 = 5,
       PC_SYEV = 6, PC_CHOL = 7, PC_PSD_EIG = 8, PC_NS = 9, PC_GEMM_REDUCE = 10, PC_PSD_TRI = 11,
       PC_GEMM_F32_SPLIT64 = 12, PC_COUNT = 13 };

tp_status prof_begin(tp_ctx* c, size_t* e0) {
  if (!c->prof) return TP_OK;
  if (c->ev_next + 3 > c->ev_pool.size()) {
    size_t old = c->ev_pool.size();
    c->ev_pool.resize(old + 1024);
    for (size_t i = old; i < c->ev_pool.size(); ++i) HIPCHK(hipEventCreate(&c->ev_pool[i]));
  }
  *e0 = c->ev_next++;
  HIPCHK(hipEventRecord(c->ev_pool[*e0], c->stream));
  return TP_OK;
}
tp_status prof_end(tp_ctx* c, int cls, size_t e0, double flops, double bytes) {
  if (!c->prof) return TP_OK;
  size_t e1 = c->ev_next++;
  HIPCHK(hipEventRecord(c->ev_pool[e1], c->stream));
  c->recs.push_back({cls, e0, e1, flops, bytes});
  return TP_OK;
}
// Fold recorded events into the per-class totals (synchronises the stream).
tp_status prof_flush(tp_ctx* c) {
  if (c->recs.empty()) return TP_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (auto& r : c->recs) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[r.e0], c->ev_pool[r.e1]));
    c->prof_ms[r.cls] += ms;
    c->prof_n[r.cls] += 1;
    c->prof_flops[r.cls] += r.flops;
    c->prof_bytes[r.cls] += r.bytes;
  }
  c->recs.clear();
  c->ev_next = 0;
  return TP_OK;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

tp_status check_grid(int n, int prec) {
  if (n < 1) return fail(TP_EINVAL, "grid size n=%d must be >= 1", n);
  if (!pow2(n + 1)) return fail(TP_EINVAL, "grid size n=%d: n+1 must be a power of two", n);
  (void)prec;
  // up to n+1 = 16384 the transform's work array sits in LDS, beyond it in the workspace
  if (n + 1 > 32768) return fail(TP_EINVAL, "grid size n=%d exceeds the sine-transform limit n+1<=32768", n);
  return TP_OK;
}

template <typename T>
tp_status get_table(tp_ctx* c, int N, const T** out);
template <>
tp_status get_table<double>(tp_ctx* c, int N, const double** out) {
  auto it = c->tab64.find(N);
  if (it == c->tab64.end()) {
    double* p = nullptr;
    HIPCHK(hipMalloc(&p, sizeof(double) * 2 * N));
    HIPCHK(dst_table<double>(N, p, c->stream));
    it = c->tab64.emplace(N, p).first;
  }
  *out = it->second;
  return TP_OK;
}
template <>
tp_status get_table<float>(tp_ctx* c, int N, const float** out) {
  auto it = c->tab32.find(N);
  if (it == c->tab32.end()) {
    float* p = nullptr;
    HIPCHK(hipMalloc(&p, sizeof(float) * 2 * N));
    HIPCHK(dst_table<float>(N, p, c->stream));
    it = c->tab32.emplace(N, p).first;
  }
  *out = it->second;
  return TP_OK;
}

template <typename T>
tp_status dst_cols(tp_ctx* c, int n, int cols, const T* in, T* out) {
  if (cols <= 0) return TP_OK;
  const T* tab = nullptr;
  TPCHK(get_table<T>(c, n + 1, &tab));
  const double* tab64 = nullptr;
  TPCHK(get_table<double>(c, n + 1, &tab64));
  WsScope scope(c);
  void* work = nullptr;
  if (n + 1 > 16384) {
    double* w = nullptr;
    TPCHK(wsalloc(c, (size_t)cols * (n + 1), &w));  // cols * (N/2) complex doubles
    work = w;
  }
  size_t e0 = 0;
  TPCHK(prof_begin(c, &e0));
  HIPCHK(dst1<T>(n + 1, cols, in, n, out, n, tab, tab64, work, c->stream));
  // algorithmic work of a real FFT-based DST: ~2.5 N log2(2N) flops per column; bytes: in + out
  double lg = std::log2(2.0 * (n + 1));
  TPCHK(prof_end(c, std::is_same<T, double>::value ? PC_DST_F64 : PC_DST_F32, e0, 2.5 * (n + 1) * lg * cols,
                 2.0 * n * cols * sizeof(T)));
  return TP_OK;
}

// Several transforms at once: jobs of one length share a launch (up to kDstJobs per launch), as
// the modes of the tensors in a product do; mixed lengths and n + 1 > 16384 take one launch each.
template <typename T>
tp_status dst_cols_batch(tp_ctx* c, int cnt, const int* n, const int* cols, const T* const* in, T* const* out) {
  bool same = cnt > 0 && n[0] + 1 <= 16384;
  for (int i = 1; i < cnt; ++i) same = same && n[i] == n[0];
  if (!same) {
    for (int i = 0; i < cnt; ++i) TPCHK(dst_cols<T>(c, n[i], cols[i], in[i], out[i]));
    return TP_OK;
  }
  const T* tab = nullptr;
  TPCHK(get_table<T>(c, n[0] + 1, &tab));
  const double* tab64 = nullptr;
  TPCHK(get_table<double>(c, n[0] + 1, &tab64));
  const double lg = std::log2(2.0 * (n[0] + 1));
  for (int i0 = 0; i0 < cnt; i0 += kDstJobs) {
    const int k = std::min(kDstJobs, cnt - i0);
    DstJob<T> jobs[kDstJobs];
    long tc = 0;
    for (int i = 0; i < k; ++i) {
      jobs[i] = DstJob<T>{in[i0 + i], out[i0 + i], cols[i0 + i], n[0], n[0], 0};
      tc += std::max(0, cols[i0 + i]);
    }
    if (tc == 0) continue;
    size_t e0 = 0;
    TPCHK(prof_begin(c, &e0));
    HIPCHK(dst1_batched<T>(n[0] + 1, jobs, k, tab, tab64, c->stream));
    TPCHK(prof_end(c, std::is_same<T, double>::value ? PC_DST_F64 : PC_DST_F32, e0, 2.5 * (n[0] + 1) * lg * tc,
                   2.0 * n[0] * tc * sizeof(T)));
  }
  return TP_OK;
}

tp_status sync_to_host(tp_ctx* c, const void* dev, size_t bytes, void* host) {
  if (bytes == 0) return TP_OK;
  HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TP_OK;
}

template <typename TA, typename TB, typename TC, typename Tacc>
int gemm_class() {
  if (std::is_same<TA, double>::value && std::is_same<TC, double>::value) return PC_GEMM_F64;
  if (std::is_same<TA, float>::value && std::is_same<TC, float>::value) return PC_GEMM_F32;
  if (std::is_same<TA, float>::value && std::is_same<Tacc, float>::value) return PC_GEMM_F32_SPLIT64;
  if (std::is_same<TA, float>::value) return PC_GEMM_F32_F64;
  return PC_GEMM_F64_F32;
}

// ------------------------------------------------------------------------------ GEMM helpers
// Up to kGemmGroup independent products with the same operand kinds in one launch.  Few output
// tiles and a long contraction: K is split over workgroups (chunks of at least 64) so that about
// kSplitTarget workgroups share the launch; the partial sums are added by a second kernel.
// Workgroups a split-K launch aims at (four per compute unit: with 16-deep stages 1024 measured
// about 1 % faster than 768 on the n = 2047 mixed solve, 512 and 1536 no better)
constexpr long kSplitTarget = 1024;

template <typename TA, typename TB, typename TC, typename Tacc>
tp_status run_group(tp_ctx* c, const GemmArgs<TA, TB, TC, Tacc>* g0, int count) {
  GemmArgs<TA, TB, TC, Tacc> g[kGemmGroup];
  if (count < 1 || count > kGemmGroup) return fail(TP_EINVAL, "GEMM group of %d products", count);
  long tiles = 0;
  for (int i = 0; i < count; ++i) {
    g[i] = g0[i];
    if (g[i].M > 0 && g[i].N > 0) tiles += (long)((g[i].M + 63) / 64) * ((g[i].N + 63) / 64) * g[i].batch;
  }
  size_t mark = c->ws_top;
  bool split = false;
  // FP32 accumulation into an FP64 result: splits of at most kF32Chunk (their sums are FP64)
  constexpr bool chunked = std::is_same<TC, double>::value && std::is_same<Tacc, float>::value;
  for (int i = 0; i < count; ++i) {
    if (g[i].M <= 0 || g[i].N <= 0) continue;
    const int need = chunked ? (g[i].K + kF32Chunk - 1) / kF32Chunk : 1;
    int splits = need;
    if (tiles < kSplitTarget / 2 && g[i].K >= 128)
      splits = std::max(splits, (int)std::min<long>((g[i].K + 63) / 64, std::max<long>(1, kSplitTarget / tiles)));
    if (splits < 2) continue;
    Tacc* part = nullptr;
    if (wsalloc(c, (size_t)g[i].batch * splits * g[i].M * g[i].N, &part) == TP_OK) {
      g[i].splits = splits;
      g[i].part = part;
      split = true;
    } else if (need > 1) {
      c->ws_top = mark;
      return fail(TP_ENOMEM, "workspace exhausted by the split partial sums of a %dx%dx%d product", g[i].M, g[i].N, g[i].K);
    }
  }
  size_t e0 = 0, em = 0;
  TPCHK(prof_begin(c, &e0));
  split = split && c->prof;
  if (split) em = c->ev_next++;  // recorded between the contraction and its reduction
  hipError_t ge = gemm_group<TA, TB, TC, Tacc>(g, count, c->stream, split ? c->ev_pool[em] : nullptr);
  c->ws_top = mark;  // the partial-sum scratch is consumed by the launches just enqueued
  HIPCHK(ge);
  if (c->prof) {
    // algorithmic work: 2 M N K per product; bytes: operands once + result once (face-split
    // operands count their two factor matrices)
    double fl = 0, by = 0, rfl = 0, rby = 0;
    for (int i = 0; i < count; ++i) {
      double M = g[i].M, N = g[i].N, K = g[i].K, b = g[i].batch;
      if (M <= 0 || N <= 0 || b <= 0) continue;
      fl += 2.0 * M * N * K * b;
      double ba = g[i].fsA ? (double)M * (g[i].FA.r1 + K / std::max(1, g[i].FA.r1))
                           : M * K * (g[i].divA > 1 || g[i].sA ? b / g[i].divA : 1);
      double bb = g[i].fsB ? (double)K * (g[i].FB.r1 + N / std::max(1, g[i].FB.r1))
                           : K * N * (g[i].sB ? b / g[i].divB : 1);
      by += ba * sizeof(TA) + bb * sizeof(TB) + M * N * b * sizeof(TC);
      if (g[i].splits > 1) {
        // the reduction adds the partial sums (splits x the output, read once) and writes the output
        rfl += M * N * b * (g[i].splits - 1);
        rby += M * N * b * ((double)g[i].splits * sizeof(Tacc) + sizeof(TC));
      }
    }
    if (split) {
      // the contraction [e0, em] carries the algorithmic work, the reduction is [em, e1]
      c->recs.push_back({gemm_class<TA, TB, TC, Tacc>(), e0, em, fl, by});
      TPCHK(prof_end(c, PC_GEMM_REDUCE, em, rfl, rby));
    } else {
      TPCHK(prof_end(c, gemm_class<TA, TB, TC, Tacc>(), e0, fl, by));
    }
  }
  return TP_OK;
}

template <typename TA, typename TB, typename TC, typename Tacc>
tp_status run(tp_ctx* c, const GemmArgs<TA, TB, TC, Tacc>& g) {
  return run_group(c, &g, 1);
}

// C (M x N) = alpha op(A) op(B) + beta C, plain operands.
template <typename TA, typename TB, typename TC, typename Tacc>
GemmArgs<TA, TB, TC, Tacc> mm_args(bool tA, bool tB, int M, int N, int K, double alpha, const TA* A, int lda,
                                   const TB* B, int ldb, double beta, TC* C, int ldc) {
  GemmArgs<TA, TB, TC, Tacc> g;
  g.M = M; g.N = N; g.K = K;
  g.alpha = (Tacc)alpha; g.beta = (Tacc)beta;
  g.A = A; g.lda = lda; g.tA = tA;
  g.B = B; g.ldb = ldb; g.tB = tB;
  g.C = C; g.ldc = ldc;
  return g;
}

template <typename TA, typename TB, typename TC, typename Tacc>
tp_status mm(tp_ctx* c, bool tA, bool tB, int M, int N, int K, double alpha, const TA* A, int lda, const TB* B,
             int ldb, double beta, TC* C, int ldc) {
  return run(c, mm_args<TA, TB, TC, Tacc>(tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc));
}

// ------------------------------------------------------------------------------ eigen
// Diagonalise `cnt` symmetric matrices (device, double), eigenvalues to W (device) and, when
// host_w is given, also to the host.  Job descriptors travel in the kernel arguments.
tp_status eig(tp_ctx* c, int cnt, const int* K, const double* const* A, double* const* W, double* const* V,
              std::vector<std::vector<double>>* host_w, double tol = 0.0) {
  int Kmax = 0;
  for (int i = 0; i < cnt; ++i) {
    if (K[i] > kMaxRank) return fail(TP_ERANK, "Gram matrix of size %d exceeds the eigensolver limit %d", K[i], kMaxRank);
    Kmax = std::max(Kmax, K[i]);
  }
  if (Kmax == 0) {
    if (host_w) host_w->assign(cnt, {});
    return TP_OK;
  }
  const int Kp = (Kmax + 1) & ~1;
  double* work = nullptr;
  if (Kmax > kGramLds) TPCHK(wsalloc(c, (size_t)Kp * Kp * std::min(cnt, kBatchJobs), &work));
  for (int b0 = 0; b0 < cnt; b0 += kBatchJobs) {
    const int nb = std::min(kBatchJobs, cnt - b0);
    JobBatch<EigJob> jb;
    for (int i = 0; i < nb; ++i)
      jb.j[i] = EigJob{K[b0 + i], A[b0 + i], W[b0 + i], V[b0 + i], work ? work + (size_t)Kp * Kp * i : nullptr, tol};
    size_t e0 = 0;
    TPCHK(prof_begin(c, &e0));
    HIPCHK(syev_batched(jb, nb, Kmax, c->stream));
    // algorithmic work: a symmetric eigendecomposition costs about 9 K^3 flops; bytes: A in, V and w out
    double fl = 0, by = 0;
    for (int i = 0; i < nb; ++i) {
      const double k = K[b0 + i];
      fl += 9.0 * k * k * k;
      by += 8.0 * (2.0 * k * k + k);
    }
    TPCHK(prof_end(c, PC_SYEV, e0, fl, by));
  }
  if (host_w) {
    host_w->assign(cnt, {});
    size_t off = 0;
    for (int i = 0; i < cnt; ++i) {
      if (off + K[i] > tp_ctx::kHost) return fail(TP_EINVAL, "eigenvalue staging too small");
      HIPCHK(hipMemcpyAsync(c->host + off, W[i], sizeof(double) * K[i], hipMemcpyDeviceToHost, c->stream));
      off += K[i];
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    off = 0;
    for (int i = 0; i < cnt; ++i) {
      (*host_w)[i].assign(c->host + off, c->host + off + K[i]);
      off += K[i];
    }
  }
  return TP_OK;
}

// Pivoted Cholesky of cnt Gram matrices G[i] (K[i] x K[i]): W[i] = P R^-1 (K[i] x q[i]) with the
// numerical rank q[i] (pivots above tol * max diagonal) returned on the host.  The kernel writes
// the ranks straight into mapped host memory; only the stream synchronisation remains.
tp_status chol(tp_ctx* c, int cnt, const int* K, const double* const* G, double tol, double* const* W, int* q) {
  if (cnt > kBatchJobs) return fail(TP_EINVAL, "too many Cholesky jobs");
  int Kmax = 0;
  for (int i = 0; i < cnt; ++i) Kmax = std::max(Kmax, K[i]);
  if (Kmax > kMaxRank) return fail(TP_ERANK, "Gram matrix of size %d exceeds %d", Kmax, kMaxRank);
  double* work = nullptr;
  // above 64 the blocked factorisation keeps L (and above 128 the trailing matrix) in global memory
  if (Kmax > 64) TPCHK(wsalloc(c, (size_t)2 * Kmax * Kmax * cnt, &work));
  int* dq = reinterpret_cast<int*>(c->dmap);
  JobBatch<CholJob> jb;
  for (int i = 0; i < cnt; ++i)
    jb.j[i] = CholJob{K[i], tol, G[i], W[i], dq + i, work ? work + (size_t)2 * Kmax * Kmax * i : nullptr};
  size_t e0 = 0;
  TPCHK(prof_begin(c, &e0));
  HIPCHK(pchol_batched(jb, cnt, Kmax, c->stream));
  {
    double fl = 0, by = 0;
    for (int i = 0; i < cnt; ++i) { fl += 2.0 * K[i] * K[i] * K[i] / 3.0; by += 8.0 * 2.0 * K[i] * K[i]; }
    TPCHK(prof_end(c, PC_CHOL, e0, fl, by));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  const int* hq = reinterpret_cast<const int*>(c->hmap);
  for (int i = 0; i < cnt; ++i) q[i] = hq[i];
  return TP_OK;
}

// W[i] = G[i]^(-1/2) (K[i] x K[i]) by Newton-Schulz for Gram matrices near the identity; *all_ok
// tells whether every one converged (otherwise the caller uses the pivoted Cholesky instead).
tp_status ns_isqrt(tp_ctx* c, int cnt, const int* K, const double* const* G, double* const* W, bool* all_ok) {
  if (cnt > kBatchJobs) return fail(TP_EINVAL, "too many Newton-Schulz jobs");
  int Kmax = 0;
  for (int i = 0; i < cnt; ++i) Kmax = std::max(Kmax, K[i]);
  if (Kmax > kNsMax) return fail(TP_EINVAL, "Newton-Schulz limited to %d", kNsMax);
  int* dok = reinterpret_cast<int*>(c->dmap);
  JobBatch<NsJob> jb;
  for (int i = 0; i < cnt; ++i) jb.j[i] = NsJob{K[i], G[i], W[i], dok + i};
  size_t e0 = 0;
  TPCHK(prof_begin(c, &e0));
  HIPCHK(ns_isqrt_batched(jb, cnt, Kmax, c->stream));
  {
    double fl = 0, by = 0;  // about three K^3 products per step, three steps
    for (int i = 0; i < cnt; ++i) { fl += 18.0 * K[i] * K[i] * K[i]; by += 8.0 * 2.0 * K[i] * K[i]; }
    TPCHK(prof_end(c, PC_NS, e0, fl, by));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  const int* hok = reinterpret_cast<const int*>(c->hmap);
  *all_ok = true;
  for (int i = 0; i < cnt; ++i) *all_ok = *all_ok && hok[i] == 1;
  return TP_OK;
}

// Eigenpairs of cnt positive semidefinite Gram matrices (pivoted Cholesky + one-sided Jacobi):
// eigenvectors to V (device), eigenvalues (descending) on the host in host_w, numerical ranks in
// q, and the trace the Cholesky left unresolved in rest (it belongs to the discarded tail).  The
// kernel writes eigenvalues, ranks and traces straight into mapped host memory.
// cut > 0 (relative to the trace, at least kTriCutMin): eigenpairs with eigenvalue <= cut * trace(G)
// are not needed, which lets matrices of order <= kTriMax go to the tridiagonal solver; a matrix
// whose kept eigenvectors it cannot certify orthogonal (clustered eigenvalues) is redone by the
// Jacobi solver.
constexpr double kTriCutMin = 1e-13;
constexpr double kTriOrthTol = 1e-10;
tp_status psd_eig(tp_ctx* c, int cnt, const int* K, const double* const* G, double* const* V, double jtol,
                  std::vector<std::vector<double>>* host_w, int* q, double* rest, double cut = 0.0) {
  if (cnt > kBatchJobs) return fail(TP_EINVAL, "too many eigen jobs");
  int Kmax = 0;
  size_t tot = 0;
  for (int i = 0; i < cnt; ++i) {
    if (K[i] > kMaxRank) return fail(TP_ERANK, "Gram matrix of size %d exceeds the eigensolver limit %d", K[i], kMaxRank);
    Kmax = std::max(Kmax, K[i]);
    tot += K[i];
  }
  if (tot + 2 * cnt > tp_ctx::kMap) return fail(TP_EINVAL, "eigenvalue staging too small");
  host_w->assign(cnt, {});
  if (Kmax == 0) {
    for (int i = 0; i < cnt; ++i) { q[i] = 0; rest[i] = 0.0; }
    return TP_OK;
  }
  double* work = nullptr;
  // above 64 the blocked factorisation keeps L (and above 128 the trailing matrix) in global memory
  if (Kmax > 64) TPCHK(wsalloc(c, (size_t)2 * Kmax * Kmax * cnt, &work));
  // mapped layout: eigenvalues (tot), traces (cnt), ranks (cnt ints)
  double* dres = c->dmap + tot;
  int* dq = reinterpret_cast<int*>(dres + cnt);
  JobBatch<PsdJob> jb;
  size_t off = 0;
  for (int i = 0; i < cnt; ++i) {
    jb.j[i] = PsdJob{K[i], G[i], c->dmap + off, V[i], dq + i, dres + i,
                     work ? work + (size_t)2 * Kmax * Kmax * i : nullptr, 1e-16, jtol};
    off += K[i];
  }
  // algorithmic work: that of a symmetric eigendecomposition with vectors, about 9 K^3 flops
  // (tridiagonal reduction, eigenvalues, back transformation); bytes: G in, V and w out
  auto work_of = [&](const std::vector<int>& idx, double* fl, double* by) {
    *fl = *by = 0;
    for (int i : idx) { *fl += 9.0 * K[i] * K[i] * K[i]; *by += 8.0 * (2.0 * K[i] * K[i] + K[i]); }
  };
  std::vector<int> jacobi;
  const int* hq = reinterpret_cast<const int*>(c->hmap + tot + cnt);
  if (cut >= kTriCutMin && Kmax <= kTriMax) {
    JobBatch<PsdJob> jt = jb;
    for (int i = 0; i < cnt; ++i) { jt.j[i].ctol = cut; jt.j[i].jtol = kTriOrthTol; jt.j[i].work = nullptr; }
    size_t e0 = 0;
    TPCHK(prof_begin(c, &e0));
    HIPCHK(psd_tri_batched(jt, cnt, Kmax, c->stream));
    std::vector<int> all(cnt);
    for (int i = 0; i < cnt; ++i) all[i] = i;
    double fl, by;
    work_of(all, &fl, &by);
    TPCHK(prof_end(c, PC_PSD_TRI, e0, fl, by));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < cnt; ++i)
      if (hq[i] < 0) jacobi.push_back(i);
  } else {
    for (int i = 0; i < cnt; ++i) jacobi.push_back(i);
  }
  if (!jacobi.empty()) {
    JobBatch<PsdJob> jj;
    int kmj = 0;
    for (size_t t = 0; t < jacobi.size(); ++t) {
      jj.j[t] = jb.j[jacobi[t]];
      if (work) jj.j[t].work = work + (size_t)2 * Kmax * Kmax * t;
      kmj = std::max(kmj, K[jacobi[t]]);
    }
    size_t e0 = 0;
    TPCHK(prof_begin(c, &e0));
    HIPCHK(psd_eig_batched(jj, (int)jacobi.size(), kmj, c->stream));
    double fl, by;
    work_of(jacobi, &fl, &by);
    TPCHK(prof_end(c, PC_PSD_EIG, e0, fl, by));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  const double* hres = c->hmap + tot;
  off = 0;
  for (int i = 0; i < cnt; ++i) {
    rest[i] = hres[i];
    q[i] = hq[i];
    (*host_w)[i].assign(c->hmap + off, c->hmap + off + K[i]);
    off += K[i];
  }
  return TP_OK;
}

// The same eigendecomposition with eigenvalues left on the device (W[i], K[i] doubles, zero past
// the numerical rank) and no synchronisation; ranks and traces go to the mapped scratch.
tp_status psd_eig_dev(tp_ctx* c, int cnt, const int* K, const double* const* G, double* const* W, double* const* V,
                      double jtol) {
  if (cnt > kBatchJobs) return fail(TP_EINVAL, "too many eigen jobs");
  int Kmax = 0;
  for (int i = 0; i < cnt; ++i) {
    if (K[i] > kMaxRank) return fail(TP_ERANK, "Gram matrix of size %d exceeds the eigensolver limit %d", K[i], kMaxRank);
    Kmax = std::max(Kmax, K[i]);
  }
  if (Kmax == 0) return TP_OK;
  double* work = nullptr;
  // above 64 the blocked factorisation keeps L (and above 128 the trailing matrix) in global memory
  if (Kmax > 64) TPCHK(wsalloc(c, (size_t)2 * Kmax * Kmax * cnt, &work));
  double* dres = c->dmap + tp_ctx::kMap / 2;
  int* dq = reinterpret_cast<int*>(dres + cnt);
  JobBatch<PsdJob> jb;
  for (int i = 0; i < cnt; ++i)
    jb.j[i] = PsdJob{K[i], G[i], W[i], V[i], dq + i, dres + i, work ? work + (size_t)2 * Kmax * Kmax * i : nullptr,
                     1e-16, jtol};
  size_t e0 = 0;
  TPCHK(prof_begin(c, &e0));
  HIPCHK(psd_eig_batched(jb, cnt, Kmax, c->stream));
  double fl = 0, by = 0;
  for (int i = 0; i < cnt; ++i) { fl += 9.0 * K[i] * K[i] * K[i]; by += 8.0 * (2.0 * K[i] * K[i] + K[i]); }
  TPCHK(prof_end(c, PC_PSD_EIG, e0, fl, by));
  return TP_OK;
}

// Orthonormal bases of the column spans of cnt matrices V[i] (n[i] x K[i], double, ld n[i]) by
// two passes of Cholesky QR: the first pass pivots and drops columns whose residual norm falls
// below sqrt(reltol) of the largest (rank revealing), the second restores orthogonality.  All
// matrices share one launch per pass.  Q[i] is n[i] x q[i] in the workspace; q[i] = 0 for a zero
// matrix.
tp_status ortho_batch(tp_ctx* c, int cnt, const int* n, const int* K, const double* const* V, double reltol,
                      double** Qout, int* qout) {
  typedef GemmArgs<double, double, double, double> GA;
  double *G[3], *W[3], *Q1[3];
  int q1[3];
  GA gs[3];
  int ng = 0;
  for (int i = 0; i < cnt; ++i) {
    qout[i] = 0;
    Qout[i] = nullptr;
    TPCHK(wsalloc(c, (size_t)K[i] * K[i], &G[i]));
    TPCHK(wsalloc(c, (size_t)K[i] * K[i], &W[i]));
    if (K[i] > 0)
      gs[ng++] = mm_args<double, double, double, double>(true, false, K[i], K[i], n[i], 1.0, V[i], n[i], V[i], n[i], 0.0, G[i], K[i]);
  }
  if (ng) TPCHK(run_group(c, gs, ng));
  const double* Gc[3] = {G[0], G[1], G[2]};
  TPCHK(chol(c, cnt, K, Gc, reltol, W, q1));
  int q1c[3];
  ng = 0;
  GA gg[3];
  for (int i = 0; i < cnt; ++i) {
    q1c[i] = q1[i];
    Q1[i] = nullptr;
    if (q1[i] == 0) continue;
    TPCHK(wsalloc(c, (size_t)n[i] * q1[i], &Q1[i]));
    gs[ng] = mm_args<double, double, double, double>(false, false, n[i], q1[i], K[i], 1.0, V[i], n[i], W[i], K[i], 0.0, Q1[i], n[i]);
    gg[ng++] = mm_args<double, double, double, double>(true, false, q1[i], q1[i], n[i], 1.0, Q1[i], n[i], Q1[i], n[i], 0.0, G[i], q1[i]);
  }
  if (ng) {
    TPCHK(run_group(c, gs, ng));
    TPCHK(run_group(c, gg, ng));
  }
  int q2[3];
  // second pass: Q1^T Q1 = I + E with E of the first pass's loss of orthogonality.  Its inverse
  // square root by Newton-Schulz (products of small matrices, no sequential pivot steps) gives an
  // orthonormal basis of the same span; the pivoted Cholesky is the fallback when E is not small.
  bool ns = true;
  for (int i = 0; i < cnt; ++i) ns = ns && q1c[i] <= kNsMax;
  if (ns) TPCHK(ns_isqrt(c, cnt, q1c, Gc, W, &ns));
  if (ns) {
    for (int i = 0; i < cnt; ++i) q2[i] = q1c[i];
  } else {
    TPCHK(chol(c, cnt, q1c, Gc, 1e-14, W, q2));
  }
  ng = 0;
  for (int i = 0; i < cnt; ++i) {
    if (q1[i] == 0 || q2[i] == 0) continue;
    TPCHK(wsalloc(c, (size_t)n[i] * q2[i], &Qout[i]));
    gs[ng++] = mm_args<double, double, double, double>(false, false, n[i], q2[i], q1[i], 1.0, Q1[i], n[i], W[i], q1[i], 0.0, Qout[i], n[i]);
    qout[i] = q2[i];
  }
  if (ng) TPCHK(run_group(c, gs, ng));
  return TP_OK;
}

tp_status ortho(tp_ctx* c, int n, int K, const double* V, double reltol, double** Qout, int* qout) {
  const double* Vp[1] = {V};
  return ortho_batch(c, 1, &n, &K, Vp, reltol, Qout, qout);
}

// out = alpha * C x_1 op(A1) x_2 op(A2) [x_3 op(A3)] + beta*out, all double.
// C is r1 x r2 (x r3) packed; op(A_m) is p_m x r_m.
tp_status tucker_contract(tp_ctx* c, int d, const int* r, const double* C, const double* const* A, const int* lda,
                          const bool* tA, const int* p, double alpha, double beta, double* out) {
  WsScope scope(c);
  if (d == 2) {
    double* Y1;
    TPCHK(wsalloc(c, (size_t)p[0] * r[1], &Y1));
    TPCHK(mm<double, double, double, double>(c, tA[0], false, p[0], r[1], r[0], 1.0, A[0], lda[0], C, r[0], 0.0, Y1, p[0]));
    // out (p0 x p1) = alpha Y1 op(A1)^T
    TPCHK(mm<double, double, double, double>(c, false, !tA[1], p[0], p[1], r[1], alpha, Y1, p[0], A[1], lda[1], beta, out, p[0]));
    return TP_OK;
  }
  double *Y1, *Y2;
  TPCHK(wsalloc(c, (size_t)p[0] * r[1] * r[2], &Y1));
  TPCHK(wsalloc(c, (size_t)p[0] * p[1] * r[2], &Y2));
  TPCHK(mm<double, double, double, double>(c, tA[0], false, p[0], r[1] * r[2], r[0], 1.0, A[0], lda[0], C, r[0], 0.0, Y1, p[0]));
  {
    GemmArgs<double, double, double, double> g;
    g.M = p[0]; g.N = p[1]; g.K = r[1]; g.batch = r[2];
    g.A = Y1; g.lda = p[0]; g.sA = (long)p[0] * r[1];
    g.B = A[1]; g.ldb = lda[1]; g.tB = !tA[1]; g.sB = 0;
    g.C = Y2; g.ldc = p[0]; g.sC = (long)p[0] * p[1];
    TPCHK(run(c, g));
  }
  TPCHK(mm<double, double, double, double>(c, false, !tA[2], p[0] * p[1], p[2], r[2], alpha, Y2, p[0] * p[1], A[2], lda[2], beta, out, p[0] * p[1]));
  return TP_OK;
}

// HOSVD of a dense core M (q1 x q2 x q3, type T): per-mode Gram eigendecompositions,
// ranks by sum_{i>r} s_i^2 <= tol^2 ||M||^2 / d (capped), bases U_m (double, q_m x r_m, ld q_m)
// and the new core M x_m U_m^T written to core_out (type TO).
template <typename T, typename TO>
tp_status hosvd(tp_ctx* c, int d, const int* q, const T* M, double tol, int cap, int* rout, double** U,
                TO* core_out, bool* capped) {
  using Tacc = double;
  double* G[3];
  double* E[3];
  for (int m = 0; m < d; ++m) {
    TPCHK(wsalloc(c, (size_t)q[m] * q[m], &G[m]));
    TPCHK(wsalloc(c, (size_t)q[m] * q[m], &E[m]));
  }
  {
    WsScope scope(c);
    if (d == 2) {
      TPCHK((mm<T, T, double, Tacc>(c, false, true, q[0], q[0], q[1], 1.0, M, q[0], M, q[0], 0.0, G[0], q[0])));
      TPCHK((mm<T, T, double, Tacc>(c, true, false, q[1], q[1], q[0], 1.0, M, q[0], M, q[0], 0.0, G[1], q[1])));
    } else {
      int q23 = q[1] * q[2], q12 = q[0] * q[1];
      T* Mp;
      TPCHK(wsalloc(c, (size_t)q[0] * q[1] * q[2], &Mp));
      HIPCHK(permute3<T>(M, q[0], q[1], q[2], Mp, 1, 0, 2, c->stream));
      // the mode-1 and mode-2 Grams (same operand kinds) share a launch
      GemmArgs<T, T, double, Tacc> g01[2] = {
          mm_args<T, T, double, Tacc>(false, true, q[0], q[0], q23, 1.0, M, q[0], M, q[0], 0.0, G[0], q[0]),
          mm_args<T, T, double, Tacc>(false, true, q[1], q[1], q[0] * q[2], 1.0, Mp, q[1], Mp, q[1], 0.0, G[1], q[1])};
      TPCHK(run_group(c, g01, 2));
      TPCHK((mm<T, T, double, Tacc>(c, true, false, q[2], q[2], q12, 1.0, M, q12, M, q12, 0.0, G[2], q[2])));
    }
  }
  std::vector<std::vector<double>> hw;
  const double* Ap[3] = {G[0], G[1], d == 3 ? G[2] : nullptr};
  int qr[3] = {0, 0, 0};
  double rest[3] = {0, 0, 0};
  // Jacobi rotations stop once every column pair is orthogonal to 1e-2 tol relative: that
  // resolves every eigenvalue to 1e-2 tol of itself (the rank rule needs far less) and moves the
  // kept subspace, hence the truncation error, by about 1e-2 tol ||M||.
  // eigenvalues below tol^2 trace / (2 d K) may be dropped: together they stay under half of the
  // rank rule's threshold tol^2 ||M||^2 / d
  int qmax = 1;
  for (int m = 0; m < d; ++m) qmax = std::max(qmax, q[m]);
  TPCHK(psd_eig(c, d, q, Ap, E, std::max(1e-14, 1e-2 * tol), &hw, qr, rest, tol * tol / (2.0 * d * qmax)));
  *capped = false;
  for (int m = 0; m < d; ++m) {
    double tot = rest[m];
    for (double v : hw[m]) tot += std::max(v, 0.0);
    double thr = tol * tol * tot / d;
    // smallest r <= numerical rank with rest + sum_{i >= r} w_i <= thr
    int r = std::max(qr[m], 1);
    double tail = rest[m];
    for (int i = qr[m] - 1; i >= 1; --i) {
      double v = std::max(hw[m][i], 0.0);
      if (tail + v > thr) break;
      tail += v;
      r = i;
    }
    if (r > cap) { r = cap; *capped = true; }
    if (r < 1) r = 1;
    rout[m] = r;
    U[m] = E[m];
  }
  // core = M x_m U_m^T
  WsScope scope(c);
  if (d == 2) {
    if (std::is_same<T, double>::value) {
      double* X1;
      TPCHK(wsalloc(c, (size_t)rout[0] * q[1], &X1));
      TPCHK((mm<double, double, double, double>(c, true, false, rout[0], q[1], q[0], 1.0, U[0], q[0], (const double*)M, q[0], 0.0, X1, rout[0])));
      TPCHK((mm<double, double, TO, double>(c, false, false, rout[0], rout[1], q[1], 1.0, X1, rout[0], U[1], q[1], 0.0, core_out, rout[0])));
    } else {
      float *Uf0, *Uf1, *X1;
      TPCHK(wsalloc(c, (size_t)q[0] * q[0], &Uf0));
      TPCHK(wsalloc(c, (size_t)q[1] * q[1], &Uf1));
      ConvBatch<double, float> cb;
      cb.add(U[0], Uf0, (long)q[0] * rout[0]);
      cb.add(U[1], Uf1, (long)q[1] * rout[1]);
      HIPCHK(convert_batch(cb, c->stream));
      TPCHK(wsalloc(c, (size_t)rout[0] * q[1], &X1));
      TPCHK((mm<float, float, float, float>(c, true, false, rout[0], q[1], q[0], 1.0, Uf0, q[0], (const float*)M, q[0], 0.0, X1, rout[0])));
      TPCHK((mm<float, float, TO, typename std::conditional<std::is_same<TO, double>::value, double, float>::type>(
          c, false, false, rout[0], rout[1], q[1], 1.0, X1, rout[0], Uf1, q[1], 0.0, core_out, rout[0])));
    }
    return TP_OK;
  }
  // d == 3
  if (std::is_same<T, double>::value) {
    const double* Md = (const double*)M;
    double *X1, *X2;
    TPCHK(wsalloc(c, (size_t)rout[0] * q[1] * q[2], &X1));
    TPCHK(wsalloc(c, (size_t)rout[0] * rout[1] * q[2], &X2));
    TPCHK((mm<double, double, double, double>(c, true, false, rout[0], q[1] * q[2], q[0], 1.0, U[0], q[0], Md, q[0], 0.0, X1, rout[0])));
    GemmArgs<double, double, double, double> g;
    g.M = rout[0]; g.N = rout[1]; g.K = q[1]; g.batch = q[2];
    g.A = X1; g.lda = rout[0]; g.sA = (long)rout[0] * q[1];
    g.B = U[1]; g.ldb = q[1];
    g.C = X2; g.ldc = rout[0]; g.sC = (long)rout[0] * rout[1];
    TPCHK(run(c, g));
    TPCHK((mm<double, double, TO, double>(c, false, false, rout[0] * rout[1], rout[2], q[2], 1.0, X2, rout[0] * rout[1], U[2], q[2], 0.0, core_out, rout[0] * rout[1])));
  } else {
    const float* Mf = (const float*)M;
    float *Uf[3], *X1, *X2;
    ConvBatch<double, float> cb;
    for (int m = 0; m < 3; ++m) {
      TPCHK(wsalloc(c, (size_t)q[m] * rout[m], &Uf[m]));
      cb.add(U[m], Uf[m], (long)q[m] * rout[m]);
    }
    HIPCHK(convert_batch(cb, c->stream));
    TPCHK(wsalloc(c, (size_t)rout[0] * q[1] * q[2], &X1));
    TPCHK(wsalloc(c, (size_t)rout[0] * rout[1] * q[2], &X2));
    TPCHK((mm<float, float, float, float>(c, true, false, rout[0], q[1] * q[2], q[0], 1.0, Uf[0], q[0], Mf, q[0], 0.0, X1, rout[0])));
    GemmArgs<float, float, float, float> g;
    g.M = rout[0]; g.N = rout[1]; g.K = q[1]; g.batch = q[2];
    g.A = X1; g.lda = rout[0]; g.sA = (long)rout[0] * q[1];
    g.B = Uf[1]; g.ldb = q[1];
    g.C = X2; g.ldc = rout[0]; g.sC = (long)rout[0] * rout[1];
    TPCHK(run(c, g));
    TPCHK((mm<float, float, TO, typename std::conditional<std::is_same<TO, double>::value, double, float>::type>(
        c, false, false, rout[0] * rout[1], rout[2], q[2], 1.0, X2, rout[0] * rout[1], Uf[2], q[2], 0.0, core_out, rout[0] * rout[1])));
  }
  return TP_OK;
}

// ------------------------------------------------------------------------------ tensor checks
tp_status check_tensor(const tp_tensor* t, const char* name, bool need_rank) {
  if (!t) return fail(TP_EINVAL, "%s is NULL", name);
  if (t->d != 2 && t->d != 3) return fail(TP_EINVAL, "%s: d=%d must be 2 or 3", name, t->d);
  if (t->prec != TP_FP64 && t->prec != TP_MIXED) return fail(TP_EINVAL, "%s: unknown precision %d", name, t->prec);
  if (t->cap < 1 || t->cap > kMaxCap) return fail(TP_EINVAL, "%s: cap=%d must be in [1,%d]", name, t->cap, kMaxCap);
  for (int m = 0; m < t->d; ++m) {
    TPCHK(check_grid(t->n[m], t->prec));
    if (!t->factor[m]) return fail(TP_EINVAL, "%s: factor[%d] is NULL", name, m);
    if (need_rank && (t->rank[m] < 0 || t->rank[m] > t->cap))
      return fail(TP_EINVAL, "%s: rank[%d]=%d outside [0,cap=%d]", name, m, t->rank[m], t->cap);
  }
  if (!t->core) return fail(TP_EINVAL, "%s: core is NULL", name);
  return TP_OK;
}

bool same_shape(const tp_tensor* a, const tp_tensor* b) {
  if (a->d != b->d || a->prec != b->prec) return false;
  for (int m = 0; m < a->d; ++m)
    if (a->n[m] != b->n[m]) return false;
  return true;
}

bool is_zero(const tp_tensor* t) {
  for (int m = 0; m < t->d; ++m)
    if (t->rank[m] == 0) return true;
  return false;
}

template <typename T>
tp_status set_zero(tp_ctx* c, tp_tensor* y) {
  for (int m = 0; m < y->d; ++m) y->rank[m] = 0;
  (void)c;
  return TP_OK;
}

// ------------------------------------------------------------------------------ truncation of sums
template <typename T>
tp_status truncate_impl(tp_ctx* c, int count, const double* coef, const tp_tensor* const* xs, tp_tensor* y,
                        double tol, int cap, bool* capped) {
  WsScope scope(c);
  const int d = y->d;
  std::vector<int> idx;
  for (int i = 0; i < count; ++i)
    if (!is_zero(xs[i]) && coef[i] != 0.0) idx.push_back(i);
  if (idx.empty()) return set_zero<T>(c, y);
  int K[3] = {0, 0, 0};
  for (int i : idx)
    for (int m = 0; m < d; ++m) K[m] += xs[i]->rank[m];
  double* V[3];
  double* Q[3];
  int q[3];
  double* R[3];
  for (int m = 0; m < d; ++m) {
    int n = y->n[m];
    TPCHK(wsalloc(c, (size_t)n * K[m], &V[m]));
    int off = 0;
    for (int i : idx) {
      HIPCHK((copy2d<T, double>(n, xs[i]->rank[m], (const T*)xs[i]->factor[m], n, V[m] + (size_t)n * off, n, 1.0, c->stream)));
      off += xs[i]->rank[m];
    }
  }
  {
    const double* Vc[3] = {V[0], V[1], V[2]};
    TPCHK(ortho_batch(c, d, y->n, K, Vc, 1e-15, Q, q));
  }
  {
    GemmArgs<double, double, double, double> gs[3];
    for (int m = 0; m < d; ++m) {
      int n = y->n[m];
      if (q[m] == 0) return set_zero<T>(c, y);
      TPCHK(wsalloc(c, (size_t)q[m] * K[m], &R[m]));
      gs[m] = mm_args<double, double, double, double>(true, false, q[m], K[m], n, 1.0, Q[m], n, V[m], n, 0.0, R[m], q[m]);
    }
    TPCHK(run_group(c, gs, d));
  }
  size_t msz = (size_t)q[0] * q[1] * (d == 3 ? q[2] : 1);
  double* M;
  TPCHK(wsalloc(c, msz, &M));
  int off[3] = {0, 0, 0};
  bool first = true;
  for (int i : idx) {
    const tp_tensor* x = xs[i];
    size_t csz = (size_t)x->rank[0] * x->rank[1] * (d == 3 ? x->rank[2] : 1);
    WsScope inner(c);
    double* Cd;
    TPCHK(wsalloc(c, csz, &Cd));
    HIPCHK((convert<T, double>((const T*)x->core, Cd, (long)csz, c->stream)));
    const double* A[3];
    int lda[3];
    bool tA[3] = {false, false, false};
    for (int m = 0; m < d; ++m) {
      A[m] = R[m] + (size_t)q[m] * off[m];
      lda[m] = q[m];
    }
    TPCHK(tucker_contract(c, d, x->rank, Cd, A, lda, tA, q, coef[i], first ? 0.0 : 1.0, M));
    first = false;
    for (int m = 0; m < d; ++m) off[m] += x->rank[m];
  }
  int rn[3] = {1, 1, 1};
  double* U[3];
  TPCHK((hosvd<double, T>(c, d, q, M, tol, cap, rn, U, (T*)y->core, capped)));
  GemmArgs<double, double, T, double> gf[3];
  for (int m = 0; m < d; ++m) {
    int n = y->n[m];
    gf[m] = mm_args<double, double, T, double>(false, false, n, rn[m], q[m], 1.0, Q[m], n, U[m], q[m], 0.0, (T*)y->factor[m], n);
    y->rank[m] = rn[m];
  }
  TPCHK(run_group(c, gf, d));
  return TP_OK;
}

// ------------------------------------------------------------------------------ apply (sketched)
// One term of a combination sum_t coef_t * F(s_t (.) F x_t); sym == nullptr stands for the
// identity symbol (s = 1, one term with unit factors).
struct Term {
  const tp_symbol* sym;
  const tp_tensor* x;
  double coef;
};

// Unit symbol (rank 1, all-ones factors, weight 1) for grid size n, created on first use.
template <typename T>
tp_status unit_symbol(tp_ctx* c, int n, const T** f, const double** w);

// y = trunc(sum_t coef_t F(s_t (.) F x_t)) by a sketched HOSVD in spectral coordinates:
//  1. spectral factors Vh = F V of every term,
//  2. per mode m the Khatri-Rao sketch Y_m = sum_t coef_t [F(s_t (.) x_t)]_(m) (Omega_o2 (.) Omega_o1):
//     A_o[i,(k,q)] = sum_x Vh_o(x,i) s_o(x,k) Omega_o(x,q), contracted with the core, then
//     Y_m = FS(Vh_m, s_m, sigma) t,  FS the face-split (Hadamard) operand,
//  3. orthonormal bases Q_m of the sketches (FP64),
//  4. projected core M = sum_t coef_t sum_k sigma_k C x_1 P1_k x_2 P2_k x_3 P3_k with
//     P_m[a,(i,k)] = sum_x Q_m(x,a) Vh_m(x,i) s_m(x,k),
//  5. HOSVD of M (ranks by tolerance and cap), factors F(Q_m U_m).
// stop_early (optional) is called with ||M||^2 between steps 4 and 5 (||M|| is the norm of the sum up
// to the range finder's error); when it returns true the call ends there and y is left unchanged.
using EarlyStop = std::function<bool(double)>;
template <typename T>
tp_status combo_impl(tp_ctx* c, const Term* terms, int nt, tp_tensor* y, double tol, int cap, const tp_sketch* sk,
                     bool* capped, const EarlyStop* stop_early = nullptr) {
  using Tacc = T;
  WsScope scope(c);
  *capped = false;
  const int d = y->d;
  const int Qs = sk->q;
  std::vector<Term> tv;
  for (int i = 0; i < nt; ++i)
    if (!is_zero(terms[i].x) && terms[i].coef != 0.0) tv.push_back(terms[i]);
  if (tv.empty()) return set_zero<T>(c, y);
  const int nterm = (int)tv.size();
  struct Prep {
    int r[3];
    int R;
    T* Vh[3];
    T* C;
    const T* S[3];
    const T* Sw[3];  // the factors with the weights folded in
    T* A[3];
  };
  std::vector<Prep> pr(nterm);
  // sketch matrices in T
  const T* Om[3];
  {
    ConvBatch<double, T> cb;
    for (int m = 0; m < d; ++m) {
      if (std::is_same<T, double>::value) {
        Om[m] = (const T*)sk->omega[m];
      } else {
        T* o;
        TPCHK(wsalloc(c, (size_t)y->n[m] * Qs, &o));
        cb.add(sk->omega[m], o, (long)y->n[m] * Qs);
        Om[m] = o;
      }
    }
    HIPCHK(convert_batch(cb, c->stream));
  }
  // the factors of every term in sine coordinates (one launch for all of them)
  {
    std::vector<int> jn, jc;
    std::vector<const T*> ji;
    std::vector<T*> jo;
    for (int t = 0; t < nterm; ++t) {
      Prep& P = pr[t];
      const tp_tensor* x = tv[t].x;
      for (int m = 0; m < 3; ++m) P.r[m] = m < d ? x->rank[m] : 1;
      for (int m = 0; m < d; ++m) {
        if (c->spectral) {
          P.Vh[m] = (T*)x->factor[m];  // read only; a y aliasing x is written after the last read
          continue;
        }
        TPCHK(wsalloc(c, (size_t)x->n[m] * P.r[m], &P.Vh[m]));
        jn.push_back(x->n[m]); jc.push_back(P.r[m]);
        ji.push_back((const T*)x->factor[m]); jo.push_back(P.Vh[m]);
      }
    }
    TPCHK(dst_cols_batch<T>(c, (int)jn.size(), jn.data(), jc.data(), ji.data(), jo.data()));
  }
  for (int t = 0; t < nterm; ++t) {
    Prep& P = pr[t];
    const tp_tensor* x = tv[t].x;
    // the core is only read here (a y aliasing x receives its core from the HOSVD after the last read)
    P.C = (T*)x->core;
    if (tv[t].sym) {
      P.R = tv[t].sym->R;
      for (int m = 0; m < d; ++m) {
        P.S[m] = (const T*)tv[t].sym->factors[m];
        P.Sw[m] = (const T*)tv[t].sym->factors_w[m];
      }
    } else {
      P.R = 1;
      for (int m = 0; m < d; ++m) {
        const double* w1 = nullptr;
        TPCHK(unit_symbol<T>(c, x->n[m], &P.S[m], &w1));
        P.Sw[m] = P.S[m];
      }
    }
    // A_m[i + r_m (k + R q)] = sum_x Vh_m(x,i) S_m(x,k) Om_m(x,q), the modes in one launch
    GemmArgs<T, T, T, Tacc> ga[3];
    for (int m = 0; m < d; ++m) {
      TPCHK(wsalloc(c, (size_t)P.r[m] * P.R * Qs, &P.A[m]));
      GemmArgs<T, T, T, Tacc>& g = ga[m];
      g.M = P.r[m]; g.N = P.R * Qs; g.K = x->n[m];
      g.A = P.Vh[m]; g.lda = x->n[m]; g.tA = true;
      g.fsB = true; g.FB.x1 = P.S[m]; g.FB.ld1 = x->n[m]; g.FB.r1 = P.R;
      g.FB.x2 = Om[m]; g.FB.ld2 = x->n[m];
      g.C = P.A[m]; g.ldc = P.r[m];
    }
    TPCHK(run_group(c, ga, d));
  }
  // sketches Y_m (double); per term the d contractions with the face-split operands share a launch
  double* Y[3];
  for (int m = 0; m < d; ++m) TPCHK(wsalloc(c, (size_t)y->n[m] * Qs, &Y[m]));
  for (int t = 0; t < nterm; ++t) {
    Prep& P = pr[t];
    const int* r = P.r;
    const int R = P.R;
    WsScope s2(c);
    // FP32 operands: the matrix cores accumulate in FP32 over chunks of K, summed in FP64
    typedef typename std::conditional<std::is_same<T, float>::value, float, double>::type TaccS;
    GemmArgs<T, T, double, TaccS> gy[3];
    for (int m = 0; m < d; ++m) {
      const int n = y->n[m];
      T* tt;
      TPCHK(wsalloc(c, (size_t)r[m] * R * Qs, &tt));
      WsScope s2m(c);
      size_t csz = (size_t)r[0] * r[1] * r[2];
      if (d == 3) {
        int o1 = m == 0 ? 1 : 0, o2 = m == 2 ? 1 : 2;
        T* Cm = P.C;
        if (m != 0) {
          TPCHK(wsalloc(c, csz, &Cm));
          HIPCHK(permute3<T>(P.C, r[0], r[1], r[2], Cm, m, o1, o2, c->stream));
        }
        T* T1;
        TPCHK(wsalloc(c, (size_t)r[m] * r[o1] * R * Qs, &T1));
        TPCHK((mm<T, T, T, Tacc>(c, false, false, r[m] * r[o1], R * Qs, r[o2], 1.0, Cm, r[m] * r[o1], P.A[o2], r[o2], 0.0, T1, r[m] * r[o1])));
        HIPCHK(contract_mid<T>(T1, P.A[o1], r[m], r[o1], R * Qs, tt, c->stream));
      } else {
        int o = 1 - m;
        T* Cm = P.C;
        if (m == 1) {
          TPCHK(wsalloc(c, csz, &Cm));
          HIPCHK(permute3<T>(P.C, r[0], r[1], 1, Cm, 1, 0, 2, c->stream));
        }
        TPCHK((mm<T, T, T, Tacc>(c, false, false, r[m], R * Qs, r[o], 1.0, Cm, r[m], P.A[o], r[o], 0.0, tt, r[m])));
      }
      GemmArgs<T, T, double, TaccS>& g = gy[m];
      g.M = n; g.N = Qs; g.K = r[m] * R;
      g.alpha = tv[t].coef; g.beta = t == 0 ? 0.0 : 1.0;
      g.fsA = true; g.FA.x1 = P.Vh[m]; g.FA.ld1 = n; g.FA.r1 = r[m];
      g.FA.x2 = P.Sw[m]; g.FA.ld2 = n;
      g.B = tt; g.ldb = r[m] * R;
      g.C = Y[m]; g.ldc = n;
    }
    TPCHK(run_group(c, gy, d));
  }
  // orthonormal bases of the sketches
  double* Qb[3];
  int q[3] = {1, 1, 1};
  {
    int Ks[3] = {Qs, Qs, Qs};
    const double* Yc[3] = {Y[0], Y[1], Y[2]};
    TPCHK(ortho_batch(c, d, y->n, Ks, Yc, 1e-14, Qb, q));
  }
  for (int m = 0; m < d; ++m)
    if (q[m] == 0) return set_zero<T>(c, y);
  T* Qt[3];
  {
    ConvBatch<double, T> cb;
    for (int m = 0; m < d; ++m) {
      if (std::is_same<T, double>::value) {
        Qt[m] = (T*)Qb[m];
      } else {
        TPCHK(wsalloc(c, (size_t)y->n[m] * q[m], &Qt[m]));
        cb.add(Qb[m], Qt[m], (long)y->n[m] * q[m]);
      }
    }
    HIPCHK(convert_batch(cb, c->stream));
  }
  // projected core
  size_t msz = (size_t)q[0] * q[1] * (d == 3 ? q[2] : 1);
  T* M;
  TPCHK(wsalloc(c, msz, &M));
  for (int t = 0; t < nterm; ++t) {
    Prep& P = pr[t];
    const int* r = P.r;
    const int R = P.R;
    WsScope s3(c);
    T* Pm[3];
    GemmArgs<T, T, T, Tacc> gps[3];
    for (int m = 0; m < d; ++m) {
      const int n = y->n[m];
      TPCHK(wsalloc(c, (size_t)q[m] * r[m] * R, &Pm[m]));
      GemmArgs<T, T, T, Tacc>& gp = gps[m];
      gp.M = q[m]; gp.N = r[m] * R; gp.K = n;
      gp.A = Qt[m]; gp.lda = n; gp.tA = true;
      gp.fsB = true; gp.FB.x1 = P.Vh[m]; gp.FB.ld1 = n; gp.FB.r1 = r[m];
      gp.FB.x2 = (m == d - 1) ? P.Sw[m] : P.S[m]; gp.FB.ld2 = n;
      gp.C = Pm[m]; gp.ldc = q[m];
    }
    TPCHK(run_group(c, gps, d));
    const double beta = t == 0 ? 0.0 : 1.0;
    if (d == 3) {
      T *D, *E;
      TPCHK(wsalloc(c, (size_t)R * q[0] * r[1] * r[2], &D));
      TPCHK(wsalloc(c, (size_t)R * r[2] * q[0] * q[1], &E));
      GemmArgs<T, T, T, Tacc> g1;
      g1.M = q[0]; g1.N = r[1] * r[2]; g1.K = r[0]; g1.batch = R;
      g1.A = Pm[0]; g1.lda = q[0]; g1.sA = (long)q[0] * r[0];
      g1.B = P.C; g1.ldb = r[0]; g1.sB = 0;
      g1.C = D; g1.ldc = q[0]; g1.sC = (long)q[0] * r[1] * r[2];
      TPCHK(run(c, g1));
      GemmArgs<T, T, T, Tacc> g2;
      g2.M = q[0]; g2.N = q[1]; g2.K = r[1]; g2.batch = R * r[2];
      g2.A = D; g2.lda = q[0]; g2.sA = (long)q[0] * r[1];
      g2.B = Pm[1]; g2.ldb = q[1]; g2.tB = true; g2.sB = (long)q[1] * r[1]; g2.divB = r[2];
      g2.C = E; g2.ldc = q[0]; g2.sC = (long)q[0] * q[1];
      TPCHK(run(c, g2));
      TPCHK((mm<T, T, T, Tacc>(c, false, true, q[0] * q[1], q[2], r[2] * R, tv[t].coef, E, q[0] * q[1], Pm[2], q[2], beta, M, q[0] * q[1])));
    } else {
      T* D;
      TPCHK(wsalloc(c, (size_t)R * q[0] * r[1], &D));
      GemmArgs<T, T, T, Tacc> g1;
      g1.M = q[0]; g1.N = r[1]; g1.K = r[0]; g1.batch = R;
      g1.A = Pm[0]; g1.lda = q[0]; g1.sA = (long)q[0] * r[0];
      g1.B = P.C; g1.ldb = r[0]; g1.sB = 0;
      g1.C = D; g1.ldc = q[0]; g1.sC = (long)q[0] * r[1];
      TPCHK(run(c, g1));
      TPCHK((mm<T, T, T, Tacc>(c, false, true, q[0], q[1], r[1] * R, tv[t].coef, D, q[0], Pm[1], q[1], beta, M, q[0])));
    }
  }
  if (stop_early) {
    double* part;
    TPCHK(wsalloc(c, 256, &part));
    HIPCHK(dot<T>(M, M, (long)msz, c->dmap, part, c->stream));  // into mapped host memory
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((*stop_early)(c->hmap[0])) return TP_OK;
  }
  // HOSVD of the projected core
  int rn[3] = {1, 1, 1};
  double* U[3];
  TPCHK((hosvd<T, T>(c, d, q, M, tol, cap, rn, U, (T*)y->core, capped)));
  WsScope s4(c);
  T* W[3] = {nullptr, nullptr, nullptr};
  int yn[3];
  T* yf[3];
  GemmArgs<double, double, T, double> gw[3];
  for (int m = 0; m < d; ++m) {
    int n = y->n[m];
    yn[m] = n;
    yf[m] = (T*)y->factor[m];
    if (c->spectral) {
      gw[m] = mm_args<double, double, T, double>(false, false, n, rn[m], q[m], 1.0, Qb[m], n, U[m], q[m], 0.0,
                                                 (T*)y->factor[m], n);
      continue;
    }
    TPCHK(wsalloc(c, (size_t)n * rn[m], &W[m]));
    gw[m] = mm_args<double, double, T, double>(false, false, n, rn[m], q[m], 1.0, Qb[m], n, U[m], q[m], 0.0, W[m], n);
  }
  TPCHK(run_group(c, gw, d));
  if (!c->spectral) {
    const T* Wc[3] = {W[0], W[1], W[2]};
    TPCHK(dst_cols_batch<T>(c, d, yn, rn, Wc, yf));
  }
  for (int m = 0; m < d; ++m) y->rank[m] = rn[m];
  return TP_OK;
}

template <typename T>
tp_status apply_impl(tp_ctx* c, const tp_symbol* S, const tp_tensor* x, tp_tensor* y, double tol, int cap,
                     const tp_sketch* sk, bool* capped, const EarlyStop* stop_early = nullptr) {
  Term t{S, x, 1.0};
  return combo_impl<T>(c, &t, 1, y, tol, cap, sk, capped, stop_early);
}

// <x, F(s (.) F y)> exactly, from the spectral factors: sum_k sigma_k <Cx, Cy x_m G_m,k> with
// G_m,k[i,j] = sum_x Vh_x(x,i) s_m(x,k) Vh_y(x,j).
template <typename T>
tp_status inner_sym_impl(tp_ctx* c, const tp_tensor* x, const tp_symbol* S, const tp_tensor* y, double* out) {
  WsScope scope(c);
  if (is_zero(x) || is_zero(y)) { *out = 0.0; return TP_OK; }
  const int d = x->d, R = S->R;
  int rx[3] = {1, 1, 1}, ry[3] = {1, 1, 1};
  T *Vx[3], *Vy[3];
  double* G[3];
  {
    int jn[6], jc[6];
    const T* ji[6];
    T* jo[6];
    int nj = 0;
    for (int m = 0; m < d; ++m) {
      int n = x->n[m];
      rx[m] = x->rank[m];
      ry[m] = y->rank[m];
      if (c->spectral) {
        Vx[m] = (T*)x->factor[m];
        Vy[m] = (T*)y->factor[m];
        continue;
      }
      TPCHK(wsalloc(c, (size_t)n * rx[m], &Vx[m]));
      TPCHK(wsalloc(c, (size_t)n * ry[m], &Vy[m]));
      jn[nj] = n; jc[nj] = rx[m]; ji[nj] = (const T*)x->factor[m]; jo[nj++] = Vx[m];
      jn[nj] = n; jc[nj] = ry[m]; ji[nj] = (const T*)y->factor[m]; jo[nj++] = Vy[m];
    }
    TPCHK(dst_cols_batch<T>(c, nj, jn, jc, ji, jo));
  }
  // FP32 operands: the matrix cores accumulate in FP32 over chunks of n, summed in FP64
  typedef typename std::conditional<std::is_same<T, float>::value, float, double>::type TaccS;
  GemmArgs<T, T, double, TaccS> gs[3];
  for (int m = 0; m < d; ++m) {
    int n = x->n[m];
    // G[i + rx (j + ry k)] (sigma folded into the last mode)
    TPCHK(wsalloc(c, (size_t)rx[m] * ry[m] * R, &G[m]));
    GemmArgs<T, T, double, TaccS>& g = gs[m];
    g.M = rx[m]; g.N = ry[m] * R; g.K = n;
    g.A = Vx[m]; g.lda = n; g.tA = true;
    g.fsB = true; g.FB.x1 = Vy[m]; g.FB.ld1 = n; g.FB.r1 = ry[m];
    g.FB.x2 = (const T*)(m == d - 1 ? S->factors_w[m] : S->factors[m]); g.FB.ld2 = n;
    g.C = G[m]; g.ldc = rx[m];
  }
  TPCHK(run_group(c, gs, d));
  size_t cx = (size_t)rx[0] * rx[1] * rx[2], cy = (size_t)ry[0] * ry[1] * ry[2];
  double *Cx, *Z, *res;
  TPCHK(wsalloc(c, cx, &Cx));
  TPCHK(wsalloc(c, cx, &Z));
  TPCHK(wsalloc(c, 257, &res));  // result + per-workgroup partial sums
  // the core contractions in the tensors' precision T (FP32: the matrix cores, the last one with its
  // long contraction over ry2 R summed in FP64 chunks); the G's are rounded to T for them
  const T* Cy = (const T*)y->core;
  T* Gt[3];
  {
    ConvBatch<T, double> cb;
    cb.add((const T*)x->core, Cx, (long)cx);
    HIPCHK(convert_batch(cb, c->stream));
    if (std::is_same<T, double>::value) {
      for (int m = 0; m < d; ++m) Gt[m] = (T*)G[m];
    } else {
      ConvBatch<double, T> cg;
      for (int m = 0; m < d; ++m) {
        TPCHK(wsalloc(c, (size_t)rx[m] * ry[m] * R, &Gt[m]));
        cg.add(G[m], Gt[m], (long)rx[m] * ry[m] * R);
      }
      HIPCHK(convert_batch(cg, c->stream));
    }
  }
  // Z = sum_k Cy x_1 G1_k x_2 G2_k x_3 G3_k  (rx1 x rx2 x rx3)
  if (d == 3) {
    T *D, *E;
    TPCHK(wsalloc(c, (size_t)R * rx[0] * ry[1] * ry[2], &D));
    TPCHK(wsalloc(c, (size_t)R * ry[2] * rx[0] * rx[1], &E));
    GemmArgs<T, T, T, T> g1;
    g1.M = rx[0]; g1.N = ry[1] * ry[2]; g1.K = ry[0]; g1.batch = R;
    g1.A = Gt[0]; g1.lda = rx[0]; g1.sA = (long)rx[0] * ry[0];
    g1.B = Cy; g1.ldb = ry[0]; g1.sB = 0;
    g1.C = D; g1.ldc = rx[0]; g1.sC = (long)rx[0] * ry[1] * ry[2];
    TPCHK(run(c, g1));
    GemmArgs<T, T, T, T> g2;
    g2.M = rx[0]; g2.N = rx[1]; g2.K = ry[1]; g2.batch = R * ry[2];
    g2.A = D; g2.lda = rx[0]; g2.sA = (long)rx[0] * ry[1];
    g2.B = Gt[1]; g2.ldb = rx[1]; g2.tB = true; g2.sB = (long)rx[1] * ry[1]; g2.divB = ry[2];
    g2.C = E; g2.ldc = rx[0]; g2.sC = (long)rx[0] * rx[1];
    TPCHK(run(c, g2));
    TPCHK((mm<T, T, double, T>(c, false, true, rx[0] * rx[1], rx[2], ry[2] * R, 1.0, E, rx[0] * rx[1], Gt[2], rx[2], 0.0, Z, rx[0] * rx[1])));
  } else {
    T* D;
    TPCHK(wsalloc(c, (size_t)R * rx[0] * ry[1], &D));
    GemmArgs<T, T, T, T> g1;
    g1.M = rx[0]; g1.N = ry[1]; g1.K = ry[0]; g1.batch = R;
    g1.A = Gt[0]; g1.lda = rx[0]; g1.sA = (long)rx[0] * ry[0];
    g1.B = Cy; g1.ldb = ry[0]; g1.sB = 0;
    g1.C = D; g1.ldc = rx[0]; g1.sC = (long)rx[0] * ry[1];
    TPCHK(run(c, g1));
    TPCHK((mm<T, T, double, T>(c, false, true, rx[0], rx[1], ry[1] * R, 1.0, D, rx[0], Gt[1], rx[1], 0.0, Z, rx[0])));
  }
  // the sum lands in mapped host memory: no copy command, only the synchronisation
  HIPCHK(dot<double>(Cx, Z, (long)cx, c->dmap, res + 1, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *out = c->hmap[0];
  return TP_OK;
}

template <typename T>
tp_status unit_symbol(tp_ctx* c, int n, const T** f, const double** w) {
  auto& mp = *reinterpret_cast<std::map<int, T*>*>(std::is_same<T, double>::value ? (void*)&c->ones64 : (void*)&c->ones32);
  auto it = mp.find(n);
  if (it == mp.end()) {
    T* p = nullptr;
    HIPCHK(hipMalloc(&p, sizeof(T) * n));
    std::vector<T> h(n, (T)1);
    HIPCHK(hipMemcpy(p, h.data(), sizeof(T) * n, hipMemcpyHostToDevice));
    it = mp.emplace(n, p).first;
  }
  if (!c->unit_w) {
    HIPCHK(hipMalloc(&c->unit_w, sizeof(double)));
    double one = 1.0;
    HIPCHK(hipMemcpy(c->unit_w, &one, sizeof(double), hipMemcpyHostToDevice));
  }
  *f = it->second;
  *w = c->unit_w;
  return TP_OK;
}

// ------------------------------------------------------------------------------ inner product
// out is host memory (the stream is synchronised), or device memory when dev_out is set (nothing
// waits: the result is ready when the stream reaches it).
template <typename T>
tp_status inner_impl(tp_ctx* c, const tp_tensor* x, const tp_tensor* y, double* out, bool dev_out = false) {
  WsScope scope(c);
  if (is_zero(x) || is_zero(y)) {
    if (!dev_out) { *out = 0.0; return TP_OK; }
    // an empty dot product writes 0 with one kernel (no memset node for graph capture)
    HIPCHK(dot<double>(nullptr, nullptr, 0, out, nullptr, c->stream));
    return TP_OK;
  }
  const int d = x->d;
  double* G[3];
  int px[3] = {1, 1, 1}, ry[3] = {1, 1, 1};
  GemmArgs<T, T, double, double> gs[3];
  for (int m = 0; m < d; ++m) {
    px[m] = x->rank[m];
    ry[m] = y->rank[m];
    TPCHK(wsalloc(c, (size_t)px[m] * ry[m], &G[m]));
    gs[m] = mm_args<T, T, double, double>(true, false, px[m], ry[m], x->n[m], 1.0, (const T*)x->factor[m], x->n[m],
                                          (const T*)y->factor[m], y->n[m], 0.0, G[m], px[m]);
  }
  TPCHK(run_group(c, gs, d));
  size_t cy = (size_t)ry[0] * ry[1] * ry[2], cx = (size_t)px[0] * px[1] * px[2];
  double *Cy, *Cx, *Z, *res;
  TPCHK(wsalloc(c, cy, &Cy));
  TPCHK(wsalloc(c, cx, &Cx));
  TPCHK(wsalloc(c, cx, &Z));
  TPCHK(wsalloc(c, 257, &res));  // result + per-workgroup partial sums
  {
    ConvBatch<T, double> cb;
    cb.add((const T*)y->core, Cy, (long)cy);
    cb.add((const T*)x->core, Cx, (long)cx);
    HIPCHK(convert_batch(cb, c->stream));
  }
  const double* A[3] = {G[0], G[1], G[2]};
  int lda[3] = {px[0], px[1], px[2]};
  bool tA[3] = {false, false, false};
  TPCHK(tucker_contract(c, d, ry, Cy, A, lda, tA, px, 1.0, 0.0, Z));
  if (dev_out) {
    HIPCHK(dot<double>(Cx, Z, (long)cx, out, res + 1, c->stream));
    return TP_OK;
  }
  // the sum lands in mapped host memory: no copy command, only the synchronisation
  HIPCHK(dot<double>(Cx, Z, (long)cx, c->dmap, res + 1, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *out = c->hmap[0];
  return TP_OK;
}

// Bytes of workspace that inner_impl takes for x and y (3D or 2D), apart from the split-K partial
// sums of its contractions, which are only used when they fit.
size_t ws_bytes(size_t count, size_t elem) {
  size_t b = ((count * elem) + 255) & ~size_t(255);
  return b ? b : 256;
}
size_t inner_ws_bytes(const tp_tensor* x, const tp_tensor* y) {
  if (is_zero(x) || is_zero(y)) return 0;
  const int d = x->d;
  size_t px[3] = {1, 1, 1}, ry[3] = {1, 1, 1};
  size_t b = 0;
  for (int m = 0; m < d; ++m) {
    px[m] = (size_t)x->rank[m];
    ry[m] = (size_t)y->rank[m];
    b += ws_bytes(px[m] * ry[m], 8);
  }
  const size_t cy = ry[0] * ry[1] * ry[2], cx = px[0] * px[1] * px[2];
  b += ws_bytes(cy, 8) + 2 * ws_bytes(cx, 8) + ws_bytes(257, 8);
  if (d == 3) b += ws_bytes(px[0] * ry[1] * ry[2], 8) + ws_bytes(px[0] * px[1] * ry[2], 8);
  else b += ws_bytes(px[0] * ry[1], 8);
  return b;
}

// ------------------------------------------------------------------------------ CP -> Tucker
template <typename T>
tp_status from_cp_impl(tp_ctx* c, const tp_cp* b, tp_tensor* out, double tol, bool* capped) {
  WsScope scope(c);
  const int d = b->d, R = b->rank;
  *capped = false;
  if (R == 0) return set_zero<T>(c, out);
  double* Q[3];
  double* Rm[3];
  int q[3] = {1, 1, 1};
  {
    int Ks[3] = {R, R, R};
    const double* F[3] = {b->factor[0], b->factor[1], d == 3 ? b->factor[2] : nullptr};
    TPCHK(ortho_batch(c, d, b->n, Ks, F, 1e-15, Q, q));
  }
  GemmArgs<double, double, double, double> gs[3];
  for (int m = 0; m < d; ++m) {
    int n = b->n[m];
    if (q[m] == 0) return set_zero<T>(c, out);
    TPCHK(wsalloc(c, (size_t)q[m] * R, &Rm[m]));
    gs[m] = mm_args<double, double, double, double>(true, false, q[m], R, n, 1.0, Q[m], n, b->factor[m], n, 0.0, Rm[m], q[m]);
  }
  TPCHK(run_group(c, gs, d));
  // R1 diag(w)
  HIPCHK(scale_cols_d(Rm[0], q[0], R, q[0], b->weight, c->stream));
  size_t msz = (size_t)q[0] * q[1] * (d == 3 ? q[2] : 1);
  double* M;
  TPCHK(wsalloc(c, msz, &M));
  if (d == 3) {
    double* KR;
    TPCHK(wsalloc(c, (size_t)q[1] * q[2] * R, &KR));
    HIPCHK(khatri_rao_d(Rm[1], q[1], Rm[2], q[2], R, KR, c->stream));
    TPCHK((mm<double, double, double, double>(c, false, true, q[0], q[1] * q[2], R, 1.0, Rm[0], q[0], KR, q[1] * q[2], 0.0, M, q[0])));
  } else {
    TPCHK((mm<double, double, double, double>(c, false, true, q[0], q[1], R, 1.0, Rm[0], q[0], Rm[1], q[1], 0.0, M, q[0])));
  }
  if (tol > 0) {
    int rn[3] = {1, 1, 1};
    double* U[3];
    TPCHK((hosvd<double, T>(c, d, q, M, tol, out->cap, rn, U, (T*)out->core, capped)));
    GemmArgs<double, double, T, double> gf[3];
    for (int m = 0; m < d; ++m) {
      int n = b->n[m];
      gf[m] = mm_args<double, double, T, double>(false, false, n, rn[m], q[m], 1.0, Q[m], n, U[m], q[m], 0.0, (T*)out->factor[m], n);
      out->rank[m] = rn[m];
    }
    TPCHK(run_group(c, gf, d));
    return TP_OK;
  }
  for (int m = 0; m < d; ++m)
    if (q[m] > out->cap) return fail(TP_ERANK, "from_cp: mode %d rank %d exceeds cap %d", m, q[m], out->cap);
  ConvBatch<double, T> cb;
  cb.add(M, (T*)out->core, (long)msz);
  for (int m = 0; m < d; ++m) {
    cb.add(Q[m], (T*)out->factor[m], (long)b->n[m] * q[m]);
    out->rank[m] = q[m];
  }
  HIPCHK(convert_batch(cb, c->stream));
  return TP_OK;
}

// ------------------------------------------------------------------------------ symbol build
// Device memory of a symbol: a block of the context's symbol pool (an idle block of at least the
// size and at most twice it, else a new allocation), returned to the pool by tp_symbol_free; or in
// a batched worker a block of the worker's workspace below every scope (released after each
// problem).
template <typename T>
tp_status sym_alloc(tp_ctx* c, tp_symbol* s, size_t count, T** p) {
  if (c->sym_arena) {
    s->arena = true;
    return wsalloc(c, count, p);
  }
  const size_t bytes = (sizeof(T) * std::max<size_t>(count, 1) + 255) & ~size_t(255);
  SymPool& pool = *c->sympool;
  void* blk = nullptr;
  size_t have = bytes;
  {
    std::lock_guard<std::mutex> g(pool.mu);
    auto it = pool.idle.lower_bound(bytes);
    if (it != pool.idle.end() && it->first <= 2 * bytes) {
      blk = it->second;
      have = it->first;
      pool.idle_bytes -= have;
      pool.idle.erase(it);
    }
  }
  if (!blk && hipMalloc(&blk, bytes) != hipSuccess)
    return fail(TP_ENOMEM, "symbol allocation of %zu bytes failed", bytes);
  if (!s->pool) s->pool = c->sympool;
  s->owned.push_back({blk, have});
  *p = reinterpret_cast<T*>(blk);
  return TP_OK;
}

// A symbol's blocks back to its pool (those beyond the pool's idle limit are freed).
void sym_release(tp_symbol* s) {
  if (s->owned.empty()) return;
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> g(s->pool->mu);
    for (const auto& b : s->owned) {
      if (s->pool->idle_bytes + b.second <= SymPool::kMaxIdle) {
        s->pool->idle.emplace(b.second, b.first);
        s->pool->idle_bytes += b.second;
      } else {
        drop.push_back(b.first);
      }
    }
  }
  s->owned.clear();
  if (!drop.empty()) {
    (void)hipDeviceSynchronize();
    for (void* p : drop) (void)hipFree(p);
  }
}

// factors_w[m] = factors[m] diag(weights): the face-split operands that carry the weights read
// them from there (one product per element instead of a third load and an FP64 multiply)
template <typename T>
tp_status build_weighted(tp_ctx* c, tp_symbol* s) {
  ScaleBatch<T> b;
  for (int m = 0; m < s->d; ++m) {
    T* F = nullptr;
    TPCHK(sym_alloc(c, s, (size_t)s->n[m] * s->R, &F));
    b.in[m] = (const T*)s->factors[m];
    b.out[m] = F;
    b.rows[m] = s->n[m];
    b.cols[m] = s->R;
    b.w[m] = s->weights;
    s->factors_w[m] = F;
  }
  b.count = s->d;
  HIPCHK(scale_cols_copy_batch<T>(b, c->stream));
  return TP_OK;
}

template <typename T>
tp_status build_factors(tp_ctx* c, tp_symbol* s) {
  // every mode and block of the factors in one launch (at most d (d + 1) = 12 jobs)
  ExpBatch<T> eb;
  for (int m = 0; m < s->d; ++m) {
    T* F = nullptr;
    TPCHK(sym_alloc(c, s, (size_t)s->n[m] * s->R, &F));
    s->factors[m] = F;
    if (s->kind == 0) {
      for (int blk = 0; blk < s->d; ++blk)
        if (!eb.add(s->lam[m], s->n[m], s->tau, s->K, F + (size_t)s->n[m] * s->K * blk, s->n[m], blk == m ? 1 : 0))
          return fail(TP_EINVAL, "too many factor blocks");
      // constant term: exp(-0 * lambda) = 1 in every mode (tau holds a trailing zero)
      if (s->R > s->d * s->K)
        if (!eb.add(s->lam[m], s->n[m], s->tau + s->K, 1, F + (size_t)s->n[m] * s->K * s->d, s->n[m], 0))
          return fail(TP_EINVAL, "too many factor blocks");
    } else {
      if (!eb.add(s->lam[m], s->n[m], s->tau, s->K, F, s->n[m], 0)) return fail(TP_EINVAL, "too many factor blocks");
    }
  }
  HIPCHK(expfactors_batch<T>(eb, c->stream));
  TPCHK(sym_alloc(c, s, (size_t)s->R, &s->weights));
  for (int blk = 0; blk < (s->kind == 0 ? s->d : 1); ++blk)
    HIPCHK(hipMemcpyAsync(s->weights + (size_t)blk * s->K, s->w, sizeof(double) * s->K, hipMemcpyDeviceToDevice, c->stream));
  if (s->kind == 0 && s->R > s->d * s->K)
    HIPCHK(hipMemcpyAsync(s->weights + (size_t)s->d * s->K, &s->c0, sizeof(double), hipMemcpyHostToDevice, c->stream));
  return build_weighted<T>(c, s);
}

// Rank-r preconditioner of the Sec. 6 tests: the truncated HOSVD of the exponential sum (a
// canonical tensor of rank K') at mode ranks <= r, which in 2D is the rank-r SVD of the matrix
// 1/s(lambda_i + lambda_j), then the Tucker core spread back into canonical form: rank r0 in 2D
// (factors U0 and U1 G^T), r0*r1 in 3D (column (a,b): U0[:,a], U1[:,b], sum_c G[a,b,c] U2[:,c]).
// Factors are formed in FP64 and stored in the symbol's precision.
template <typename T>
tp_status recompress_pre(tp_ctx* c, tp_symbol* s, int r) {
  // the symbol's factors and weights first (at most r^(d-1) columns), then the scoped temporaries
  const int Rmax = s->d == 2 ? r : r * r;
  T* Fout[3] = {nullptr, nullptr, nullptr};
  for (int m = 0; m < s->d; ++m) TPCHK(sym_alloc(c, s, (size_t)s->n[m] * Rmax, &Fout[m]));
  TPCHK(sym_alloc(c, s, (size_t)Rmax, &s->weights));
  WsScope scope(c);
  const int d = s->d, K = s->K;
  tp_cp cp{};
  cp.d = d;
  cp.rank = K;
  cp.weight = s->w;
  for (int m = 0; m < d; ++m) {
    cp.n[m] = s->n[m];
    double* E;
    TPCHK(wsalloc(c, (size_t)s->n[m] * K, &E));
    HIPCHK(expfactors<double>(s->lam[m], s->n[m], s->tau, K, E, s->n[m], 0, c->stream));
    cp.factor[m] = E;
  }
  tp_tensor t{};
  t.d = d;
  t.cap = r;
  t.prec = TP_FP64;
  double* core;
  TPCHK(wsalloc(c, (size_t)r * r * (d == 3 ? r : 1), &core));
  t.core = core;
  for (int m = 0; m < d; ++m) {
    t.n[m] = s->n[m];
    double* U;
    TPCHK(wsalloc(c, (size_t)s->n[m] * r, &U));
    t.factor[m] = U;
  }
  bool capped = false;
  TPCHK(from_cp_impl<double>(c, &cp, &t, 1e-15, &capped));
  const int r0 = t.rank[0], r1 = t.rank[1], r2 = d == 3 ? t.rank[2] : 1;
  const int R = d == 2 ? r0 : r0 * r1;
  if (R < 1) return fail(TP_EINVAL, "preconditioner recompression produced rank 0");
  const double* U[3] = {(const double*)t.factor[0], (const double*)t.factor[1],
                        d == 3 ? (const double*)t.factor[2] : nullptr};
  double* last;  // FP64 factor of the last mode: U_last times the core unfolding
  const int nl = s->n[d - 1];
  TPCHK(wsalloc(c, (size_t)nl * R, &last));
  // core column-major: 2D G[a + r0 b]; 3D G[(a + r0 b) + r0 r1 c], i.e. an (R x r_last) matrix
  TPCHK((mm<double, double, double, double>(c, false, true, nl, R, d == 2 ? r1 : r2, 1.0, U[d - 1], nl, core, R, 0.0,
                                            last, nl)));
  for (int m = 0; m < d; ++m) {
    T* F = Fout[m];
    s->factors[m] = F;
    const int n = s->n[m];
    if (m == d - 1) {
      HIPCHK((convert<double, T>(last, F, (long)n * R, c->stream)));
    } else if (m == 0) {
      // U0 once (2D) or repeated for every b (3D)
      for (int b = 0; b < (d == 3 ? r1 : 1); ++b)
        HIPCHK((copy2d<double, T>(n, r0, U[0], n, F + (size_t)n * r0 * b, n, 1.0, c->stream)));
    } else {
      // 3D mode 1: column b of U1 repeated r0 times (input leading dimension 0)
      for (int b = 0; b < r1; ++b)
        HIPCHK((copy2d<double, T>(n, r0, U[1] + (size_t)n * b, 0, F + (size_t)n * r0 * b, n, 1.0, c->stream)));
    }
  }
  std::vector<double> ones(R, 1.0);
  HIPCHK(hipMemcpyAsync(s->weights, ones.data(), sizeof(double) * R, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));  // the host vector and the workspace are released here
  s->R = R;
  s->tucker = r;
  // unit weights: the weighted factors are the factors
  for (int m = 0; m < d; ++m) s->factors_w[m] = s->factors[m];
  return TP_OK;
}

// max |p s - 1| and min p s of a recompressed preconditioner p over a lattice of grid points whose
// indices are geometric in every mode (64 per mode in 2D, 16 in 3D), s the exact symbol of fn in
// rho = sum_l lambda_{i_l}^power.
tp_status pre_lattice_error(tp_ctx* c, const tp_symbol* s, const SymFn& fn, double power, double* err,
                            double* pmin) {
  WsScope scope(c);
  const int d = s->d, L = d == 2 ? 64 : 16;
  std::vector<int> ax[3];
  std::vector<double> lam[3];
  for (int m = 0; m < d; ++m) {
    const int n = s->n[m];
    const double h = 1.0 / (n + 1.0);
    for (int k = 0; k < L; ++k) {
      int i = (int)std::floor(std::pow((double)n, (double)k / (L - 1))) - 1;
      i = std::min(std::max(i, 0), n - 1);
      ax[m].push_back(i);
      lam[m].push_back(std::pow(4.0 / (h * h) * std::pow(std::sin(M_PI * (i + 1) * h / 2), 2), power));
    }
  }
  const int cnt = d == 2 ? L * L : L * L * L;
  std::vector<int> idx((size_t)cnt * d);
  std::vector<double> sv(cnt), pv(cnt);
  for (int p = 0; p < cnt; ++p) {
    int q = p;
    double rho = 0;
    for (int m = 0; m < d; ++m) {
      idx[(size_t)p * d + m] = ax[m][q % L];
      rho += lam[m][q % L];
      q /= L;
    }
    sv[p] = fn.c0 + (fn.cn > 0 ? fn.cn * std::pow(rho, -fn.alpha) : 0.0) + (fn.cp > 0 ? fn.cp * std::pow(rho, fn.beta) : 0.0);
  }
  int* di;
  double* dout;
  TPCHK(wsalloc(c, idx.size(), &di));
  TPCHK(wsalloc(c, (size_t)cnt, &dout));
  HIPCHK(hipMemcpyAsync(di, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, c->stream));
  if (s->prec == TP_FP64) {
    const double* F[3] = {(const double*)s->factors[0], (const double*)s->factors[1], (const double*)s->factors[2]};
    HIPCHK(cp_eval<double>(d, di, cnt, s->n, F, s->R, s->weights, dout, c->stream));
  } else {
    const float* F[3] = {(const float*)s->factors[0], (const float*)s->factors[1], (const float*)s->factors[2]};
    HIPCHK(cp_eval<float>(d, di, cnt, s->n, F, s->R, s->weights, dout, c->stream));
  }
  TPCHK(sync_to_host(c, dout, sizeof(double) * cnt, pv.data()));
  double mx = 0, mn = HUGE_VAL;
  for (int p = 0; p < cnt; ++p) {
    const double ps = pv[p] * sv[p];
    const double e = std::fabs(ps - 1.0);
    if (!(e <= mx)) mx = e;
    if (!(ps >= mn)) mn = ps;
  }
  *err = mx;
  *pmin = mn;
  return TP_OK;
}

// Least-squares exponential sums for several functions f (kind 0: g, 1: 1/s, 2: the state
// symbol), each over its candidate exponent grids; keeps each fit's best candidate.  The design
// matrices, scalings, solves and error evaluations run per fit; the eigensolves of all candidates
// go to one launch of the Gram eigensolver when they fit in one batch, and one synchronisation
// reads every fit error.
struct FitSpec {
  int kind;
  SymFn f;
  double rho0, B;
  int K;
  std::vector<FitCand> cands;
  double* tau_out;
  double* w_out;
  double err;
};

tp_status fit_expsum_multi(tp_ctx* c, std::vector<FitSpec>& fits) {
  WsScope scope(c);
  const int m = 1000, nf = (int)fits.size();
  struct Buf { double *A, *t, *G, *bvec, *ew, *E, *cn, *wsol; int nc, off; };
  std::vector<Buf> bf(nf);
  int tot = 0;
  for (int i = 0; i < nf; ++i) {
    const int K = fits[i].K, nc = (int)fits[i].cands.size();
    Buf& b = bf[i];
    b.nc = nc;
    b.off = tot;
    tot += nc;
    TPCHK(wsalloc(c, (size_t)nc * m * K, &b.A));
    TPCHK(wsalloc(c, (size_t)nc * K, &b.t));
    TPCHK(wsalloc(c, (size_t)nc * K * K, &b.G));
    TPCHK(wsalloc(c, (size_t)nc * K, &b.bvec));
    TPCHK(wsalloc(c, (size_t)nc * K, &b.ew));
    TPCHK(wsalloc(c, (size_t)nc * K * K, &b.E));
    TPCHK(wsalloc(c, (size_t)nc * K, &b.cn));
    TPCHK(wsalloc(c, (size_t)nc * K, &b.wsol));
  }
  // the candidates travel through the mapped host scratch (read once by the design kernels;
  // every user of the mapped scratch synchronises the stream before returning, so it is free)
  if (tot * sizeof(FitCand) > tp_ctx::kMap / 4 * sizeof(double)) return fail(TP_EINVAL, "too many fit candidates");
  FitCand* hc = reinterpret_cast<FitCand*>(c->hmap + tp_ctx::kMap / 4);
  FitCand* dc = reinterpret_cast<FitCand*>(c->dmap + tp_ctx::kMap / 4);
  const double* ones = nullptr;
  {
    const double* w1 = nullptr;
    TPCHK(unit_symbol<double>(c, m, &ones, &w1));
  }
  std::vector<int> Ks;
  std::vector<const double*> Ap;
  std::vector<double*> Wp, Vp;
  for (int i = 0; i < nf; ++i) {
    const FitSpec& F = fits[i];
    const Buf& b = bf[i];
    const int K = F.K, nc = b.nc;
    for (int ci = 0; ci < nc; ++ci) hc[b.off + ci] = F.cands[ci];
    HIPCHK(fit_design(F.kind, F.f, F.rho0, F.B, K, m, dc + b.off, nc, b.A, b.t, c->stream));
    // column scaling: cn = 1/||A_k|| from the Gram diagonal; scaled Gram = D G D
    GemmArgs<double, double, double, double> g;
    g.M = K; g.N = K; g.K = m; g.batch = nc;
    g.A = b.A; g.lda = m; g.tA = true; g.sA = (long)m * K;
    g.B = b.A; g.ldb = m; g.sB = (long)m * K;
    g.C = b.G; g.ldc = K; g.sC = (long)K * K;
    TPCHK(run(c, g));
    GemmArgs<double, double, double, double> gb;
    gb.M = K; gb.N = 1; gb.K = m; gb.batch = nc;
    gb.A = b.A; gb.lda = m; gb.tA = true; gb.sA = (long)m * K;
    gb.B = ones; gb.ldb = m; gb.sB = 0;
    gb.C = b.bvec; gb.ldc = K; gb.sC = K;
    TPCHK(run(c, gb));
    HIPCHK(fit_scale(K, nc, b.G, b.bvec, b.cn, c->stream));
    for (int ci = 0; ci < nc; ++ci) {
      Ks.push_back(K);
      Ap.push_back(b.G + (size_t)ci * K * K);
      Wp.push_back(b.ew + (size_t)ci * K);
      Vp.push_back(b.E + (size_t)ci * K * K);
    }
  }
  // the scaled normal matrices are positive semidefinite Gram matrices: the Gram eigensolver
  // (eigenvalues to 1e-14 of themselves, ranks below 1e-16 of the largest pivot dropped)
  if (tot <= kBatchJobs) {
    TPCHK(psd_eig_dev(c, tot, Ks.data(), Ap.data(), Wp.data(), Vp.data(), 1e-14));
  } else {
    for (int i = 0; i < nf; ++i)
      TPCHK(psd_eig_dev(c, bf[i].nc, Ks.data() + bf[i].off, Ap.data() + bf[i].off, Wp.data() + bf[i].off,
                        Vp.data() + bf[i].off, 1e-14));
  }
  for (int i = 0; i < nf; ++i) {
    const FitSpec& F = fits[i];
    const Buf& b = bf[i];
    HIPCHK(fit_solve(F.K, b.nc, b.ew, b.E, b.bvec, b.cn, 1e-15, b.wsol, c->stream));
    // errors straight to the mapped host scratch
    double* part;
    TPCHK(wsalloc(c, (size_t)16 * b.nc, &part));
    HIPCHK(fit_error(F.kind, F.f, F.rho0, F.B, F.K, b.t, b.wsol, b.nc, 4096, c->dmap + b.off, part, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  const double* herr = c->hmap;
  // copies on the compute stream (the workspace they read is released in stream order), two fits
  // per launch
  ConvBatch<double, double> cb;
  for (int i = 0; i < nf; ++i) {
    FitSpec& F = fits[i];
    const Buf& b = bf[i];
    int best = 0;
    for (int ci = 1; ci < b.nc; ++ci)
      if (herr[b.off + ci] < herr[b.off + best] || std::isnan(herr[b.off + best])) best = ci;
    F.err = herr[b.off + best];
    cb.add(b.t + (size_t)best * F.K, F.tau_out, F.K);
    cb.add(b.wsol + (size_t)best * F.K, F.w_out, F.K);
    if (cb.n + 2 > kConvJobs || i + 1 == nf) {
      HIPCHK(convert_batch(cb, c->stream));
      cb.n = 0;
    }
  }
  return TP_OK;
}

// Step hh of the sinc rule u_k = k hh, k = -kl..kr, for g (kind 0 of fit_error): the candidates
// hh = c pi / sqrt(M), M = (kl + kr) / 2, c geometric in [0.4, 4], are all evaluated on 4096
// log-spaced points of [rho_min, rho_max] in one launch; the smallest measured error wins.
tp_status sinc_step_scan(tp_ctx* c, double alpha, double cn, double cp, const SymFn& fn, double rho0, double B,
                         int kl, int kr, double* hh) {
  WsScope scope(c);
  constexpr int nc = 24;
  const int K = kl + kr + 1 + (std::fabs(1.0 - alpha) < 1e-15 ? 1 : 0);
  const double M = std::max(1.0, 0.5 * (kl + kr));
  double *t, *w, *part;
  TPCHK(wsalloc(c, (size_t)nc * K, &t));
  TPCHK(wsalloc(c, (size_t)nc * K, &w));
  TPCHK(wsalloc(c, (size_t)16 * nc, &part));
  double cand[nc];
  for (int j = 0; j < nc; ++j) {
    cand[j] = 0.4 * std::pow(10.0, (double)j / (nc - 1)) * M_PI / std::sqrt(M);
    HIPCHK(sinc_g_nodes(alpha, cn, cp, rho0, kl, kr, cand[j], t + (size_t)j * K, w + (size_t)j * K, c->stream));
  }
  // the nodes come out as tau = t / rho0; the error kernel works in y = rho / rho0
  HIPCHK(scale(t, (long)nc * K, rho0, c->stream));
  HIPCHK(fit_error(0, fn, rho0, B, K, t, w, nc, 4096, c->dmap, part, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  int best = 0;
  for (int j = 1; j < nc; ++j)
    if (c->hmap[j] < c->hmap[best] || std::isnan(c->hmap[best])) best = j;
  *hh = cand[best];
  return TP_OK;
}

tp_status fit_expsum(tp_ctx* c, int kind, const SymFn& f, double rho0, double B, int K,
                     const std::vector<FitCand>& cands, double* tau_out, double* w_out, double* err_out) {
  std::vector<FitSpec> fits(1, FitSpec{kind, f, rho0, B, K, cands, tau_out, w_out, 0.0});
  TPCHK(fit_expsum_multi(c, fits));
  *err_out = fits[0].err;
  return TP_OK;
}

}  // namespace

// Worker contexts of batched solves kept in a context (destroyed with it or when the workspace
// size of a call changes).
void release_workers(tp_ctx* c) {
  for (size_t w = 0; w < c->workers.size(); ++w) {
    tp_destroy(c->workers[w]);
    (void)hipStreamDestroy(c->worker_streams[w]);
  }
  c->workers.clear();
  c->worker_streams.clear();
}

// ==================================================================================== C ABI
extern "C" {

int tp_version(void) { return 100; }

const char* tp_last_error(void) { return g_err.c_str(); }

tp_status tp_create(int device, void* stream, size_t workspace_bytes, tp_ctx** out) {
  if (!out) return fail(TP_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(TP_EINVAL, "device %d not in [0,%d)", device, ndev);
  HIPCHK(hipSetDevice(device));
  tp_ctx* c = new tp_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->ws_size = workspace_bytes ? workspace_bytes : (size_t(2) << 30);
  hipError_t e = hipMalloc(&c->ws, c->ws_size);
  if (e != hipSuccess) {
    delete c;
    return fail(TP_ENOMEM, "workspace allocation of %zu bytes failed: %s", workspace_bytes, hipGetErrorString(e));
  }
  HIPCHK(hipHostMalloc(&c->host, sizeof(double) * tp_ctx::kHost, hipHostMallocDefault));
  HIPCHK(hipHostMalloc(&c->hmap, sizeof(double) * tp_ctx::kMap, hipHostMallocMapped | hipHostMallocCoherent));
  HIPCHK(hipHostGetDevicePointer((void**)&c->dmap, c->hmap, 0));
  {
    // address of the no-allocation scratch on this device (the device is current), looked up once
    // per device and shared by every context on it
    static std::mutex mu;
    static std::map<int, char*> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
      void* p = nullptr;
      hipError_t se = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (se != hipSuccess || !p) {
        tp_destroy(c);
        return fail(TP_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(se));
      }
      it = addr.emplace(device, (char*)p).first;
    }
    c->scratch = it->second;
  }
  *out = c;
  return TP_OK;
}

tp_status tp_destroy(tp_ctx* c) {
  if (!c) return TP_OK;
  release_workers(c);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (auto& e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& kv : c->ones64) (void)hipFree(kv.second);
  for (auto& kv : c->ones32) (void)hipFree(kv.second);
  if (c->unit_w) (void)hipFree(c->unit_w);
  for (auto& kv : c->tab64) (void)hipFree(kv.second);
  for (auto& kv : c->tab32) (void)hipFree(kv.second);
  (void)hipFree(c->ws);
  (void)hipHostFree(c->hmap);
  (void)hipHostFree(c->host);
  delete c;
  return TP_OK;
}

tp_status tp_gemm_mode(int32_t mfma) {
  if (mfma < 0 || mfma > 2) return fail(TP_EINVAL, "gemm mode %d must be 0, 1 or 2", mfma);
  gemm_set_mfma(mfma);
  return TP_OK;
}

tp_status tp_profile(tp_ctx* c, int32_t enable) {
  if (!c) return fail(TP_EINVAL, "NULL context");
  TPCHK(prof_flush(c));
  c->prof = enable != 0;
  for (int i = 0; i < 16; ++i) c->prof_ms[i] = c->prof_n[i] = c->prof_flops[i] = c->prof_bytes[i] = 0;
  return TP_OK;
}

tp_status tp_profile_read(tp_ctx* c, int32_t cls, double* ms, double* launches, double* flops, double* bytes) {
  if (!c) return fail(TP_EINVAL, "NULL context");
  if (cls < 0 || cls >= PC_COUNT) return fail(TP_EINVAL, "class %d outside [0,%d)", cls, (int)PC_COUNT);
  TPCHK(prof_flush(c));
  if (ms) *ms = c->prof_ms[cls];
  if (launches) *launches = c->prof_n[cls];
  if (flops) *flops = c->prof_flops[cls];
  if (bytes) *bytes = c->prof_bytes[cls];
  return TP_OK;
}

tp_status tp_gram_eig(tp_ctx* c, int32_t K, int32_t count, const double* g, double* w, double* v, double cut,
                      int32_t* rank, double* rest) {
  if (!c || !g || !w || !v || !rank) return fail(TP_EINVAL, "NULL argument");
  if (K < 1 || K > kMaxRank) return fail(TP_EINVAL, "K=%d outside [1,%d]", K, kMaxRank);
  if (count < 1 || count > kBatchJobs) return fail(TP_EINVAL, "count=%d outside [1,%d]", count, kBatchJobs);
  if (cut != 0.0 && !(cut >= kTriCutMin)) return fail(TP_EINVAL, "cut=%g must be 0 or >= %g", cut, kTriCutMin);
  if (cut != 0.0 && K > kTriMax) return fail(TP_EINVAL, "cut > 0 needs K <= %d", kTriMax);
  WsScope scope(c);
  std::vector<int> Ks(count, K);
  std::vector<const double*> G(count);
  std::vector<double*> V(count);
  for (int i = 0; i < count; ++i) {
    G[i] = g + (size_t)K * K * i;
    V[i] = v + (size_t)K * K * i;
  }
  std::vector<std::vector<double>> hw;
  std::vector<int> q(count);
  std::vector<double> rs(count);
  TPCHK(psd_eig(c, count, Ks.data(), G.data(), V.data(), 1e-14, &hw, q.data(), rs.data(), cut));
  for (int i = 0; i < count; ++i) {
    std::memcpy(c->host + (size_t)K * i, hw[i].data(), sizeof(double) * K);
    rank[i] = q[i];
    if (rest) rest[i] = rs[i];
  }
  HIPCHK(hipMemcpyAsync(w, c->host, sizeof(double) * K * count, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TP_OK;
}

tp_status tp_lambda(tp_ctx* c, int32_t n, double* out) {
  if (!c || !out) return fail(TP_EINVAL, "NULL argument");
  if (n < 1) return fail(TP_EINVAL, "n=%d must be >= 1", n);
  HIPCHK(lambda_1d(n, out, c->stream));
  return TP_OK;
}

tp_status tp_dst(tp_ctx* c, int32_t n, int32_t cols, int32_t prec, const void* in, void* out) {
  if (!c || !in || !out) return fail(TP_EINVAL, "NULL argument");
  if (cols < 0) return fail(TP_EINVAL, "cols=%d < 0", cols);
  TPCHK(check_grid(n, prec));
  if (prec == TP_FP64) return dst_cols<double>(c, n, cols, (const double*)in, (double*)out);
  if (prec == TP_MIXED) return dst_cols<float>(c, n, cols, (const float*)in, (float*)out);
  return fail(TP_EINVAL, "unknown precision %d", prec);
}

tp_status tp_syev(tp_ctx* c, int32_t K, int32_t count, const double* a, double* w, double* v) {
  if (!c || !a || !w || !v) return fail(TP_EINVAL, "NULL argument");
  if (K < 1 || K > kMaxRank) return fail(TP_EINVAL, "K=%d must be in [1,%d]", K, kMaxRank);
  if (count < 0 || count > tp_ctx::kJobs) return fail(TP_EINVAL, "count=%d must be in [0,%d]", count, tp_ctx::kJobs);
  std::vector<int> Ks(count, K);
  std::vector<const double*> Ap(count);
  std::vector<double*> Wp(count), Vp(count);
  for (int i = 0; i < count; ++i) {
    Ap[i] = a + (size_t)i * K * K;
    Wp[i] = w + (size_t)i * K;
    Vp[i] = v + (size_t)i * K * K;
  }
  TPCHK(eig(c, count, Ks.data(), Ap.data(), Wp.data(), Vp.data(), nullptr));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TP_OK;
}

tp_status tp_symbol_build(tp_ctx* c, const tp_symbol_desc* desc, tp_symbol** op, tp_symbol** pre, double* err) {
  if (!c || !desc || !op || !pre) return fail(TP_EINVAL, "NULL argument");
  *op = nullptr;
  *pre = nullptr;
  const tp_symbol_desc& D = *desc;
  if (D.d != 2 && D.d != 3) return fail(TP_EINVAL, "d=%d must be 2 or 3", D.d);
  if (!(D.alpha > 0.0 && D.alpha <= 1.0)) return fail(TP_EINVAL, "alpha=%g must be in (0,1]", D.alpha);
  if (!(D.c_neg >= 0.0) || !(D.c_pos >= 0.0) || !(D.c_neg + D.c_pos > 0.0))
    return fail(TP_EINVAL, "coefficients c_neg=%g c_pos=%g must be >= 0 and not both 0", D.c_neg, D.c_pos);
  if (!(D.c0 >= 0.0)) return fail(TP_EINVAL, "c0=%g must be >= 0", D.c0);
  if (D.directional != 0 && D.directional != 1) return fail(TP_EINVAL, "directional=%d must be 0 or 1", D.directional);
  // directional: the 1D spectra are lambda^alpha and the symbol is a function of rho' = sum lambda^alpha
  // with unit exponents, c0 + c_neg / rho' + c_pos rho'
  const double power = D.directional ? D.alpha : 1.0;
  const double alpha = D.directional ? 1.0 : D.alpha;
  if (D.directional && D.beta != 0.0 && D.beta != 1.0)
    return fail(TP_EINVAL, "directional symbols take beta = 0 or 1 (got %g)", D.beta);
  const double beta = D.directional ? 1.0 : (D.beta == 0.0 ? D.alpha : D.beta);
  if (!(beta > 0.0 && beta <= 1.0)) return fail(TP_EINVAL, "beta=%g must be in (0,1]", D.beta);
  if (D.prec != TP_FP64 && D.prec != TP_MIXED) return fail(TP_EINVAL, "unknown precision %d", D.prec);
  for (int m = 0; m < D.d; ++m) TPCHK(check_grid(D.n[m], D.prec));
  int Kop = D.op_terms > 0 ? D.op_terms : 32;
  int Kpre = D.pre_terms > 0 ? D.pre_terms : 12;
  if (D.method == TP_SYM_FIT && (Kop < 2 || Kop > 64)) return fail(TP_EINVAL, "op_terms=%d must be in [2,64]", Kop);
  if (Kpre < 1 || Kpre > 64) return fail(TP_EINVAL, "pre_terms=%d must be in [1,64]", Kpre);
  if (D.pre_rank < 0 || D.pre_rank > 16) return fail(TP_EINVAL, "pre_rank=%d must be in [0,16]", D.pre_rank);
  if (D.method != TP_SYM_FIT && D.method != TP_SYM_SINC) return fail(TP_EINVAL, "unknown method %d", D.method);
  if (D.method == TP_SYM_SINC && (D.c0 != 0.0 || beta != alpha))
    return fail(TP_EINVAL, "the sinc rule covers c0 = 0 and beta = alpha only");
  // beta = 1: c_pos rho is exact (a tau = 0 exponential); what is left to fit is c_neg rho^-(1+alpha)
  const bool exact_pos = beta == 1.0 && D.c_pos > 0.0;
  const SymFn fn{D.c0, D.c_neg, D.c_pos, alpha, beta, exact_pos ? 0 : 1};
  const bool fit_op = !(exact_pos && D.c_neg == 0.0);
  int kl = D.sinc_kl > 0 ? D.sinc_kl : 60, kr = D.sinc_kr > 0 ? D.sinc_kr : 20;
  double hh = D.sinc_h > 0 ? D.sinc_h : 0.55;
  if (D.method == TP_SYM_SINC && kl + kr + 2 > 2048) return fail(TP_EINVAL, "sinc rule too long");

  tp_symbol* s[2] = {new tp_symbol(), new tp_symbol()};
  auto cleanup = [&](tp_status st) {
    for (int i = 0; i < 2; ++i) {
      if (s[i]) { sym_release(s[i]); delete s[i]; }
    }
    return st;
  };
  double lam1[3], lamn[3];
  LamBatch lb;  // the 1D spectra of both symbols in one launch
  for (int i = 0; i < 2; ++i) {
    s[i]->d = D.d;
    s[i]->prec = D.prec;
    s[i]->kind = i;
    for (int m = 0; m < D.d; ++m) {
      s[i]->n[m] = D.n[m];
      double* l = nullptr;
      if (sym_alloc(c, s[i], (size_t)D.n[m], &l) != TP_OK) return cleanup(TP_ENOMEM);
      s[i]->lam[m] = l;
      if (!lb.add(D.n[m], l, power)) return cleanup(fail(TP_EINVAL, "too many spectra"));
    }
  }
  if (lambda_batch(lb, c->stream) != hipSuccess) return cleanup(fail(TP_EHIP, "lambda kernel failed"));
  for (int m = 0; m < D.d; ++m) {
    double h = 1.0 / (D.n[m] + 1.0);
    lam1[m] = std::pow(4.0 / (h * h) * std::pow(std::sin(M_PI * h / 2), 2), power);
    lamn[m] = std::pow(4.0 / (h * h) * std::pow(std::sin(M_PI * D.n[m] * h / 2), 2), power);
  }
  double rmin = 0, rmax = 0;
  for (int m = 0; m < D.d; ++m) { rmin += lam1[m]; rmax += lamn[m]; }
  const double rho0 = rmin, B = rmax / rmin * 1.0000001;
  std::vector<FitSpec> fits;  // the operator's fit (if any) and the preconditioner's, run together below
  int op_fit = -1;
  // operator
  {
    tp_symbol* so = s[0];
    const int Kfit = D.method == TP_SYM_FIT ? (fit_op ? Kop : 0) : kl + kr + 1 + (std::fabs(1.0 - alpha) < 1e-15 ? 1 : 0);
    const int K = Kfit + (D.method == TP_SYM_FIT && exact_pos ? 1 : 0);
    so->K = K;
    so->c0 = D.c0;
    so->R = D.d * K + (D.c0 > 0.0 ? 1 : 0);
    // tau and w hold the K terms and a trailing zero exponent (the constant term's factors)
    if (sym_alloc(c, so, (size_t)K + 1, &so->tau) != TP_OK || sym_alloc(c, so, (size_t)K + 1, &so->w) != TP_OK)
      return cleanup(TP_ENOMEM);
    if (hipMemsetAsync(so->tau, 0, sizeof(double) * (K + 1), c->stream) != hipSuccess)
      return cleanup(fail(TP_EHIP, "memset failed"));
    if (D.method == TP_SYM_FIT) {
      if (Kfit > 0) {
        std::vector<FitCand> cands;
        for (double a : {-1.5, -1.0, -0.5})
          for (double b : {1.75, 2.25, 2.75}) cands.push_back({a, b});
        fits.push_back(FitSpec{0, fn, rho0, B, Kfit, cands, so->tau, so->w, 0.0});
        op_fit = 0;
      }
      if (exact_pos) {
        so->wexact = D.c_pos;
        if (hipMemcpyAsync(so->w + Kfit, &so->wexact, sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
          return cleanup(fail(TP_EHIP, "copy failed"));
      }
      so->err = 0.0;
    } else {
      if (D.sinc_h <= 0) {
        // the paper leaves the step constant of hh = c pi / sqrt(M) open: the library takes the c of
        // a geometric scan over [0.4, 4] whose rule has the smallest measured error on [rho_min, rho_max]
        tp_status st = sinc_step_scan(c, alpha, D.c_neg, D.c_pos, fn, rho0, B, kl, kr, &hh);
        if (st != TP_OK) return cleanup(st);
      }
      if (sinc_g_nodes(alpha, D.c_neg, D.c_pos, rho0, kl, kr, hh, so->tau, so->w, c->stream) != hipSuccess)
        return cleanup(fail(TP_EHIP, "sinc kernel failed"));
      so->err = -1;
      so->sinc_h = hh;
    }
  }
  // preconditioner
  {
    tp_symbol* sp = s[1];
    int K = Kpre;
    sp->K = K;
    sp->R = K;
    if (sym_alloc(c, sp, (size_t)K, &sp->tau) != TP_OK || sym_alloc(c, sp, (size_t)K, &sp->w) != TP_OK)
      return cleanup(TP_ENOMEM);
    std::vector<FitCand> cands;
    for (double a : {-2.5, -2.0, -1.5})
      for (double b : {0.5, 1.0, 1.5, 2.0, 2.5}) cands.push_back({a, b});
    fits.push_back(FitSpec{1, fn, rho0, B, K, cands, sp->tau, sp->w, 0.0});
  }
  // both least-squares fits at once (one launch of the eigensolver for all their candidates); the
  // fits are in the scaled variable y = rho/rho0: tau = t/rho0
  {
    tp_status st = fit_expsum_multi(c, fits);
    if (st != TP_OK) return cleanup(st);
    if (op_fit >= 0) {
      if (scale(s[0]->tau, fits[op_fit].K, 1.0 / rho0, c->stream) != hipSuccess) return cleanup(fail(TP_EHIP, "scale failed"));
      s[0]->err = fits[op_fit].err;
    }
    FitSpec& fp = fits.back();
    if (scale(s[1]->tau, fp.K, 1.0 / rho0, c->stream) != hipSuccess) return cleanup(fail(TP_EHIP, "scale failed"));
    s[1]->err = fp.err;
  }
  // measured error of the operator sum (also for the sinc rule): rho*g vs s on log samples
  for (int i = 0; i < 2; ++i) {
    tp_status st;
    if (i == 1 && D.pre_rank > 0)
      st = D.prec == TP_FP64 ? recompress_pre<double>(c, s[1], D.pre_rank) : recompress_pre<float>(c, s[1], D.pre_rank);
    else
      st = D.prec == TP_FP64 ? build_factors<double>(c, s[i]) : build_factors<float>(c, s[i]);
    if (st != TP_OK) return cleanup(st);
  }
  if (D.pre_rank > 0) {
    // measured error of the recompressed preconditioner: max |p s - 1| over a lattice of grid points
    tp_status st = pre_lattice_error(c, s[1], fn, power, &s[1]->err, &s[1]->pmin);
    if (st != TP_OK) return cleanup(st);
  }
  if (s[0]->err < 0) {
    // evaluate rho*g(rho)/s(rho)-1 with fit_error in the unscaled variable (rho0 = 1 scaling: y = rho/rho0)
    WsScope scope(c);
    double *ts, *e, *part;
    if (wsalloc(c, (size_t)s[0]->K, &ts) != TP_OK || wsalloc(c, 1, &e) != TP_OK || wsalloc(c, 16, &part) != TP_OK)
      return cleanup(TP_ENOMEM);
    if (hipMemcpyAsync(ts, s[0]->tau, sizeof(double) * s[0]->K, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        scale(ts, s[0]->K, rho0, c->stream) != hipSuccess)
      return cleanup(fail(TP_EHIP, "scale failed"));
    if (fit_error(0, fn, rho0, B, s[0]->K, ts, s[0]->w, 1, 4096, e, part, c->stream) != hipSuccess)
      return cleanup(fail(TP_EHIP, "error kernel failed"));
    double he = 0;
    if (sync_to_host(c, e, sizeof(double), &he) != TP_OK) return cleanup(TP_EHIP);
    s[0]->err = he;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return cleanup(fail(TP_EHIP, "stream sync failed"));
  if (err) { err[0] = s[0]->err; err[1] = s[1]->err; }
  // positivity of the preconditioner on the checked points: a fitted sum with relative error
  // below 1 is positive there; a rank-r recompression is checked on its lattice
  if (D.pre_rank == 0) s[1]->pmin = 1.0 - s[1]->err;
  const bool indefinite = !(s[1]->pmin > 0.0);
  const double pmin = s[1]->pmin;
  *op = s[0];
  *pre = s[1];
  s[0] = s[1] = nullptr;
  if (indefinite)
    return fail(TP_EINDEF, "preconditioner not positive: min p*s = %g on the checked points (max |p*s - 1| = %g)",
                pmin, (*pre)->err);
  return TP_OK;
}

tp_status tp_state_symbol_build(tp_ctx* c, const tp_symbol_desc* desc, tp_symbol** out, double* err) {
  if (!c || !desc || !out) return fail(TP_EINVAL, "NULL argument");
  *out = nullptr;
  const tp_symbol_desc& D = *desc;
  if (D.d != 2 && D.d != 3) return fail(TP_EINVAL, "d=%d must be 2 or 3", D.d);
  if (!(D.alpha > 0.0 && D.alpha <= 1.0)) return fail(TP_EINVAL, "alpha=%g must be in (0,1]", D.alpha);
  if (!(D.c_neg > 0.0)) return fail(TP_EINVAL, "c_neg (beta) must be > 0");
  if (D.prec != TP_FP64 && D.prec != TP_MIXED) return fail(TP_EINVAL, "unknown precision %d", D.prec);
  if (D.directional != 0 && D.directional != 1) return fail(TP_EINVAL, "directional=%d must be 0 or 1", D.directional);
  const double power = D.directional ? D.alpha : 1.0, alpha = D.directional ? 1.0 : D.alpha;
  for (int m = 0; m < D.d; ++m) TPCHK(check_grid(D.n[m], D.prec));
  int K = D.op_terms > 0 ? D.op_terms : 28;
  if (K < 2 || K > 64) return fail(TP_EINVAL, "op_terms=%d must be in [2,64]", K);
  tp_symbol* s = new tp_symbol();
  auto cleanup = [&](tp_status st) {
    sym_release(s);
    delete s;
    return st;
  };
  s->d = D.d;
  s->prec = D.prec;
  s->kind = 2;
  s->K = K;
  s->R = K;
  double rmin = 0, rmax = 0;
  for (int m = 0; m < D.d; ++m) {
    s->n[m] = D.n[m];
    double* l = nullptr;
    if (sym_alloc(c, s, (size_t)D.n[m], &l) != TP_OK) return cleanup(TP_ENOMEM);
    s->lam[m] = l;
    if (lambda_1d(D.n[m], l, c->stream, power) != hipSuccess) return cleanup(fail(TP_EHIP, "lambda kernel failed"));
    double h = 1.0 / (D.n[m] + 1.0);
    rmin += std::pow(4.0 / (h * h) * std::pow(std::sin(M_PI * h / 2), 2), power);
    rmax += std::pow(4.0 / (h * h) * std::pow(std::sin(M_PI * D.n[m] * h / 2), 2), power);
  }
  const double rho0 = rmin, B = rmax / rmin * 1.0000001;
  if (sym_alloc(c, s, (size_t)K, &s->tau) != TP_OK || sym_alloc(c, s, (size_t)K, &s->w) != TP_OK)
    return cleanup(TP_ENOMEM);
  std::vector<FitCand> cands;
  for (double a : {-1.5, -1.0, -0.5})
    for (double b : {1.75, 2.25, 2.75}) cands.push_back({a, b});
  double e = 0;
  const SymFn fn{0.0, D.c_neg, 0.0, alpha, alpha, 0};
  tp_status st = fit_expsum(c, 2, fn, rho0, B, K, cands, s->tau, s->w, &e);
  if (st != TP_OK) return cleanup(st);
  if (scale(s->tau, K, 1.0 / rho0, c->stream) != hipSuccess) return cleanup(fail(TP_EHIP, "scale failed"));
  s->err = e;
  // kind 2 factors: exp(-tau_k lambda) in every mode (one exponential sum, rank K)
  s->kind = 1;
  st = D.prec == TP_FP64 ? build_factors<double>(c, s) : build_factors<float>(c, s);
  s->kind = 2;
  if (st != TP_OK) return cleanup(st);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return cleanup(fail(TP_EHIP, "stream sync failed"));
  if (err) *err = e;
  *out = s;
  return TP_OK;
}

tp_status tp_symbol_free(tp_symbol* s) {
  if (!s) return TP_OK;
  if (s->arena) {  // workspace memory of a batched worker: released with the worker's workspace
    delete s;
    return TP_OK;
  }
  (void)hipDeviceSynchronize();  // work of any stream that still reads the symbol ends first
  sym_release(s);
  delete s;
  return TP_OK;
}

tp_status tp_symbol_info(const tp_symbol* s, int32_t* rank, double* err) {
  if (!s) return fail(TP_EINVAL, "NULL symbol");
  if (rank) *rank = s->R;
  if (err) *err = s->err;
  return TP_OK;
}

tp_status tp_symbol_eval(tp_ctx* c, const tp_symbol* s, int32_t count, const int32_t* idx, double* out) {
  if (!c || !s || (count > 0 && (!idx || !out))) return fail(TP_EINVAL, "NULL argument");
  if (count < 0) return fail(TP_EINVAL, "count < 0");
  if (s->tucker > 0) {
    if (s->prec == TP_FP64) {
      const double* F[3] = {(const double*)s->factors[0], (const double*)s->factors[1], (const double*)s->factors[2]};
      HIPCHK(cp_eval<double>(s->d, idx, count, s->n, F, s->R, s->weights, out, c->stream));
    } else {
      const float* F[3] = {(const float*)s->factors[0], (const float*)s->factors[1], (const float*)s->factors[2]};
      HIPCHK(cp_eval<float>(s->d, idx, count, s->n, F, s->R, s->weights, out, c->stream));
    }
    return TP_OK;
  }
  HIPCHK(symbol_eval(s->d, idx, count, s->n, s->lam[0], s->lam[1], s->d == 3 ? s->lam[2] : s->lam[1], s->kind,
                     s->K, s->tau, s->w, s->kind == 0 ? s->c0 : 0.0, out, c->stream));
  return TP_OK;
}

tp_status tp_from_cp(tp_ctx* c, const tp_cp* b, tp_tensor* out, double tol) {
  if (!c || !b || !out) return fail(TP_EINVAL, "NULL argument");
  TPCHK(check_tensor(out, "out", false));
  if (b->d != out->d) return fail(TP_EINVAL, "dimension mismatch");
  for (int m = 0; m < b->d; ++m) {
    if (b->n[m] != out->n[m]) return fail(TP_EINVAL, "grid mismatch in mode %d", m);
    if (b->rank > 0 && !b->factor[m]) return fail(TP_EINVAL, "b.factor[%d] NULL", m);
  }
  if (b->rank < 0 || b->rank > kMaxRank) return fail(TP_EINVAL, "b.rank=%d must be in [0,%d]", b->rank, kMaxRank);
  if (b->rank > 0 && !b->weight) return fail(TP_EINVAL, "b.weight NULL");
  bool capped = false;
  tp_status st = out->prec == TP_FP64 ? from_cp_impl<double>(c, b, out, tol, &capped)
                                      : from_cp_impl<float>(c, b, out, tol, &capped);
  if (st != TP_OK) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  return capped ? fail(TP_ERANK, "rank cap reached") : TP_OK;
}

tp_status tp_apply(tp_ctx* c, const tp_symbol* s, const tp_tensor* x, tp_tensor* y, double tol, int32_t cap,
                   const tp_sketch* sk) {
  if (!c || !s || !x || !y || !sk) return fail(TP_EINVAL, "NULL argument");
  TPCHK(check_tensor(x, "x", true));
  TPCHK(check_tensor(y, "y", false));
  if (!same_shape(x, y)) return fail(TP_EINVAL, "x and y differ in shape or precision");
  if (s->d != x->d || s->prec != x->prec) return fail(TP_EINVAL, "symbol does not match the tensor (d or precision)");
  for (int m = 0; m < x->d; ++m)
    if (s->n[m] != x->n[m]) return fail(TP_EINVAL, "symbol grid differs in mode %d", m);
  if (cap < 1 || cap > y->cap) return fail(TP_EINVAL, "cap=%d must be in [1, y.cap=%d]", cap, y->cap);
  if (!(tol >= 0.0)) return fail(TP_EINVAL, "tol must be >= 0");
  if (sk->q < 2 || sk->q > kMaxSketch) return fail(TP_EINVAL, "sketch q=%d must be in [2,%d]", sk->q, kMaxSketch);
  for (int m = 0; m < x->d; ++m)
    if (!sk->omega[m]) return fail(TP_EINVAL, "sketch omega[%d] NULL", m);
  bool capped = false;
  tp_status st = x->prec == TP_FP64 ? apply_impl<double>(c, s, x, y, tol, cap, sk, &capped)
                                    : apply_impl<float>(c, s, x, y, tol, cap, sk, &capped);
  if (st != TP_OK) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  return capped ? fail(TP_ERANK, "rank cap reached") : TP_OK;
}

tp_status tp_apply_sum(tp_ctx* c, int32_t count, const tp_symbol* const* syms, const tp_tensor* const* xs,
                       const double* coef, tp_tensor* y, double tol, int32_t cap, const tp_sketch* sk) {
  if (!c || !y || !sk || (count > 0 && (!syms || !xs || !coef))) return fail(TP_EINVAL, "NULL argument");
  if (count < 1 || count > 8) return fail(TP_EINVAL, "count=%d must be in [1,8]", count);
  TPCHK(check_tensor(y, "y", false));
  std::vector<Term> terms(count);
  for (int i = 0; i < count; ++i) {
    TPCHK(check_tensor(xs[i], "xs[i]", true));
    if (!same_shape(xs[i], y)) return fail(TP_EINVAL, "xs[%d] differs from y in shape or precision", i);
    const tp_symbol* s = syms[i];
    if (s) {
      if (s->d != y->d || s->prec != y->prec) return fail(TP_EINVAL, "symbol %d does not match y (d or precision)", i);
      for (int m = 0; m < y->d; ++m)
        if (s->n[m] != y->n[m]) return fail(TP_EINVAL, "symbol %d grid differs in mode %d", i, m);
    }
    terms[i] = Term{s, xs[i], coef[i]};
  }
  if (cap < 1 || cap > y->cap) return fail(TP_EINVAL, "cap=%d must be in [1, y.cap=%d]", cap, y->cap);
  if (!(tol >= 0.0)) return fail(TP_EINVAL, "tol must be >= 0");
  if (sk->q < 2 || sk->q > kMaxSketch) return fail(TP_EINVAL, "sketch q=%d must be in [2,%d]", sk->q, kMaxSketch);
  for (int m = 0; m < y->d; ++m)
    if (!sk->omega[m]) return fail(TP_EINVAL, "sketch omega[%d] NULL", m);
  bool capped = false;
  tp_status st = y->prec == TP_FP64 ? combo_impl<double>(c, terms.data(), count, y, tol, cap, sk, &capped)
                                    : combo_impl<float>(c, terms.data(), count, y, tol, cap, sk, &capped);
  if (st != TP_OK) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  return capped ? fail(TP_ERANK, "rank cap reached") : TP_OK;
}

tp_status tp_inner_sym(tp_ctx* c, const tp_tensor* x, const tp_symbol* s, const tp_tensor* y, double* out) {
  if (!c || !x || !s || !y || !out) return fail(TP_EINVAL, "NULL argument");
  TPCHK(check_tensor(x, "x", true));
  TPCHK(check_tensor(y, "y", true));
  if (!same_shape(x, y)) return fail(TP_EINVAL, "x and y differ in shape or precision");
  if (s->d != x->d || s->prec != x->prec) return fail(TP_EINVAL, "symbol does not match the tensors");
  for (int m = 0; m < x->d; ++m)
    if (s->n[m] != x->n[m]) return fail(TP_EINVAL, "symbol grid differs in mode %d", m);
  return x->prec == TP_FP64 ? inner_sym_impl<double>(c, x, s, y, out) : inner_sym_impl<float>(c, x, s, y, out);
}

tp_status tp_truncate(tp_ctx* c, int32_t count, const double* coef, const tp_tensor* const* xs, tp_tensor* y,
                      double tol, int32_t cap) {
  if (!c || !y || (count > 0 && (!coef || !xs))) return fail(TP_EINVAL, "NULL argument");
  if (count < 1 || count > 8) return fail(TP_EINVAL, "count=%d must be in [1,8]", count);
  TPCHK(check_tensor(y, "y", false));
  int tot[3] = {0, 0, 0};
  for (int i = 0; i < count; ++i) {
    TPCHK(check_tensor(xs[i], "xs[i]", true));
    if (!same_shape(xs[i], y)) return fail(TP_EINVAL, "xs[%d] differs from y in shape or precision", i);
    for (int m = 0; m < y->d; ++m) tot[m] += xs[i]->rank[m];
  }
  for (int m = 0; m < y->d; ++m)
    if (tot[m] > kMaxRank) return fail(TP_ERANK, "sum of ranks %d in mode %d exceeds %d", tot[m], m, kMaxRank);
  if (cap < 1 || cap > y->cap) return fail(TP_EINVAL, "cap=%d must be in [1, y.cap=%d]", cap, y->cap);
  bool capped = false;
  tp_status st = y->prec == TP_FP64 ? truncate_impl<double>(c, count, coef, xs, y, tol, cap, &capped)
                                    : truncate_impl<float>(c, count, coef, xs, y, tol, cap, &capped);
  if (st != TP_OK) return st;
  HIPCHK(hipStreamSynchronize(c->stream));
  return capped ? fail(TP_ERANK, "rank cap reached") : TP_OK;
}

tp_status tp_inner(tp_ctx* c, const tp_tensor* x, const tp_tensor* y, double* out) {
  if (!c || !x || !y || !out) return fail(TP_EINVAL, "NULL argument");
  TPCHK(check_tensor(x, "x", true));
  TPCHK(check_tensor(y, "y", true));
  if (!same_shape(x, y)) return fail(TP_EINVAL, "x and y differ in shape or precision");
  return x->prec == TP_FP64 ? inner_impl<double>(c, x, y, out) : inner_impl<float>(c, x, y, out);
}

tp_status tp_inner_noalloc(tp_ctx* c, const tp_tensor* x, const tp_tensor* y, double* out_dev) {
  if (!c || !x || !y || !out_dev) return fail(TP_EINVAL, "NULL argument");
  TPCHK(check_tensor(x, "x", true));
  TPCHK(check_tensor(y, "y", true));
  if (!same_shape(x, y)) return fail(TP_EINVAL, "x and y differ in shape or precision");
  const size_t need = inner_ws_bytes(x, y);
  if (need > kNoAllocScratchBytes)
    return fail(TP_EINVAL, "tp_inner_noalloc: ranks (%d,%d,%d) x (%d,%d,%d) need %zu bytes of scratch, more than its %zu",
                x->rank[0], x->rank[1], x->d == 3 ? x->rank[2] : 1, y->rank[0], y->rank[1],
                y->d == 3 ? y->rank[2] : 1, need, kNoAllocScratchBytes);
  if (!c->scratch) return fail(TP_EHIP, "no scratch address for device %d", c->device);
  // the same kernels as tp_inner, with the context's workspace replaced by the scratch for the call
  // (profiling events are not recorded: creating them could allocate)
  struct Swap {
    tp_ctx* c;
    char* ws; size_t size, top, peak; bool prof;
    explicit Swap(tp_ctx* cc) : c(cc), ws(cc->ws), size(cc->ws_size), top(cc->ws_top), peak(cc->ws_peak), prof(cc->prof) {
      c->ws = c->scratch; c->ws_size = kNoAllocScratchBytes; c->ws_top = 0; c->prof = false;
    }
    ~Swap() { c->ws = ws; c->ws_size = size; c->ws_top = top; c->ws_peak = peak; c->prof = prof; }
  } swap(c);
  return x->prec == TP_FP64 ? inner_impl<double>(c, x, y, out_dev, true) : inner_impl<float>(c, x, y, out_dev, true);
}

tp_status tp_eval_grid(tp_ctx* c, const tp_tensor* x, const int32_t* const* rows, const int32_t* mm_, double* out) {
  if (!c || !x || !rows || !mm_ || !out) return fail(TP_EINVAL, "NULL argument");
  TPCHK(check_tensor(x, "x", true));
  const int d = x->d;
  for (int m = 0; m < d; ++m)
    if (mm_[m] < 1 || !rows[m]) return fail(TP_EINVAL, "rows[%d] empty", m);
  WsScope scope(c);
  size_t tot = (size_t)mm_[0] * mm_[1] * (d == 3 ? mm_[2] : 1);
  if (is_zero(x)) {
    HIPCHK(hipMemsetAsync(out, 0, sizeof(double) * tot, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TP_OK;
  }
  double* Vr[3];
  int r[3] = {x->rank[0], x->rank[1], d == 3 ? x->rank[2] : 1};
  int p[3] = {mm_[0], mm_[1], d == 3 ? mm_[2] : 1};
  for (int m = 0; m < d; ++m) {
    TPCHK(wsalloc(c, (size_t)mm_[m] * r[m], &Vr[m]));
    if (x->prec == TP_FP64)
      HIPCHK(gather_rows<double>((const double*)x->factor[m], x->n[m], rows[m], mm_[m], r[m], Vr[m], c->stream));
    else
      HIPCHK(gather_rows<float>((const float*)x->factor[m], x->n[m], rows[m], mm_[m], r[m], Vr[m], c->stream));
  }
  size_t csz = (size_t)r[0] * r[1] * r[2];
  double* Cd;
  TPCHK(wsalloc(c, csz, &Cd));
  if (x->prec == TP_FP64) HIPCHK((convert<double, double>((const double*)x->core, Cd, (long)csz, c->stream)));
  else HIPCHK((convert<float, double>((const float*)x->core, Cd, (long)csz, c->stream)));
  const double* A[3] = {Vr[0], Vr[1], d == 3 ? Vr[2] : nullptr};
  int lda[3] = {p[0], p[1], p[2]};
  bool tA[3] = {false, false, false};
  TPCHK(tucker_contract(c, d, r, Cd, A, lda, tA, p, 1.0, 0.0, out));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------ PCG
namespace {

struct Iter {
  tp_tensor t;
};

template <typename T>
tp_status make_tensor(tp_ctx* c, const tp_tensor* like, int cap, tp_tensor* out) {
  *out = *like;
  out->cap = cap;
  for (int m = 0; m < 3; ++m) out->rank[m] = 0;
  T* core;
  size_t csz = (size_t)cap * cap * (like->d == 3 ? cap : 1);
  TPCHK(wsalloc(c, csz, &core));
  out->core = core;
  for (int m = 0; m < like->d; ++m) {
    T* f;
    TPCHK(wsalloc(c, (size_t)like->n[m] * cap, &f));
    out->factor[m] = f;
  }
  return TP_OK;
}

template <typename T>
tp_status copy_tensor(tp_ctx* c, const tp_tensor* src, tp_tensor* dst) {
  const int d = src->d;
  size_t csz = (size_t)src->rank[0] * src->rank[1] * (d == 3 ? src->rank[2] : 1);
  ConvBatch<T, T> cb;
  cb.add((const T*)src->core, (T*)dst->core, (long)csz);
  for (int m = 0; m < d; ++m) {
    cb.add((const T*)src->factor[m], (T*)dst->factor[m], (long)src->n[m] * src->rank[m]);
    dst->rank[m] = src->rank[m];
  }
  HIPCHK(convert_batch(cb, c->stream));
  return TP_OK;
}

// dst = a * src (the core is scaled, factors copied).
template <typename T>
tp_status scaled_copy(tp_ctx* c, double a, const tp_tensor* src, tp_tensor* dst) {
  TPCHK(copy_tensor<T>(c, src, dst));
  const int d = src->d;
  const int csz = src->rank[0] * src->rank[1] * (d == 3 ? src->rank[2] : 1);
  HIPCHK((copy2d<T, T>(csz, 1, (const T*)src->core, csz, (T*)dst->core, csz, a, c->stream)));
  return TP_OK;
}

template <typename T>
tp_status pcg_impl(tp_ctx* c, const tp_symbol* op, const tp_symbol* pre, const tp_cp* b, tp_tensor* x,
                   const tp_pcg_opts* o, const tp_sketch* sk, tp_pcg_info* info) {
  WsScope scope(c);
  const int cap = o->cap;
  const double eps = o->trunc_tol;
  tp_tensor B, X, R, P, Z, Xb, S;
  TPCHK(make_tensor<T>(c, x, cap, &B));
  if (o->recursive_residual) TPCHK(make_tensor<T>(c, x, cap, &S));
  TPCHK(make_tensor<T>(c, x, cap, &X));
  TPCHK(make_tensor<T>(c, x, cap, &Xb));
  TPCHK(make_tensor<T>(c, x, cap, &R));
  TPCHK(make_tensor<T>(c, x, cap, &P));
  TPCHK(make_tensor<T>(c, x, cap, &Z));
  info->iters = 0;
  info->status = TP_OK;
  info->rel_res = 0;
  info->true_rel_res = -1;
  info->err_est = -1;
  info->op_applies = 0;
  bool capped = false, anycap = false;
  // spectral domain: the right-hand side's factors go to sine coordinates once, every iterate
  // stays there (F is orthogonal per mode, so inner products and truncations are unchanged), and
  // X comes back once at the end
  struct SpectralScope {
    tp_ctx* c;
    ~SpectralScope() { c->spectral = false; }
  } spec_scope{c};
  tp_cp bs = *b;
  if (o->spectral_domain && b->rank > 0) {
    for (int m = 0; m < b->d; ++m) {
      double* F;
      TPCHK(wsalloc(c, (size_t)b->n[m] * b->rank, &F));
      TPCHK(dst_cols<double>(c, b->n[m], b->rank, b->factor[m], F));
      bs.factor[m] = F;
    }
  }
  // B: exact Tucker form of the canonical right-hand side, truncated well below eps
  TPCHK(from_cp_impl<T>(c, &bs, &B, eps * 1e-2, &capped));
  c->spectral = o->spectral_domain != 0;
  anycap |= capped;
  double nb2 = 0;
  TPCHK(inner_impl<T>(c, &B, &B, &nb2));
  if (!(nb2 > 0)) {
    for (int m = 0; m < x->d; ++m) x->rank[m] = 0;
    info->rank[0] = info->rank[1] = info->rank[2] = 0;
    return TP_OK;
  }
  const double nb = std::sqrt(nb2);
  const bool warm = o->warm_start && !is_zero(x);
  if (warm) {
    // X0 given: R0 = trunc(B - fun(X0)) (one sketched sum); X0 itself is taken as it is
    TPCHK(copy_tensor<T>(c, x, &X));
    if (c->spectral)  // the iteration runs in sine coordinates: transform X0's factors once
      for (int m = 0; m < x->d; ++m) TPCHK(dst_cols<T>(c, x->n[m], X.rank[m], (const T*)X.factor[m], (T*)X.factor[m]));
    Term t[2] = {{nullptr, &B, 1.0}, {op, &X, -1.0}};
    TPCHK(combo_impl<T>(c, t, 2, &R, eps, cap, sk, &capped));
    anycap |= capped;
    info->op_applies += 1;
  } else {
    TPCHK(copy_tensor<T>(c, &B, &R));  // R0 = B - fun(X0), X0 = 0 (no truncation)
  }
  TPCHK(apply_impl<T>(c, pre, &R, &Z, eps, cap, sk, &capped));
  anycap |= capped;
  info->op_applies += 1;
  TPCHK(copy_tensor<T>(c, &Z, &P));
  double rz = 0;
  TPCHK(inner_impl<T>(c, &R, &Z, &rz));
  bool converged = false, stalled = false;
  // breakdown: <R,Z> <= 0 or <P,fun(P)> <= 0 (a preconditioner or operator that is not
  // positive definite); the loop ends there and the best iterate so far is returned
  double breakdown_val = 0.0;
  const char* breakdown = !(rz > 0) ? "<R,Z>" : nullptr;
  if (breakdown) breakdown_val = rz;
  double best = HUGE_VAL;  // smallest error estimate so far; its iterate is kept in Xb
  int kbest = 0;
  int k = 0;
  for (; k < o->kmax && !breakdown; ++k) {
    // S = fun(P) stays in exact factored form (canonical symbol times P): <P,S> is computed
    // without truncation, and by default the residual is recomputed from X each step,
    // R = trunc(B - fun(X)), so residual components a truncation drops are seen again at the
    // next step
    double ps = 0;
    TPCHK(inner_sym_impl<T>(c, &P, op, &P, &ps));
    if (!(ps > 0)) { breakdown = "<P,fun(P)>"; breakdown_val = ps; break; }
    const double a = rz / ps;
    if (k == 0 && !warm) {
      // X0 = 0: X1 = a P exactly (P is already truncated, a sum with zero adds nothing to cut)
      TPCHK(scaled_copy<T>(c, a, &P, &X));
    } else {
      const tp_tensor* xs[2] = {&X, &P};
      double cf[2] = {1.0, a};
      TPCHK(truncate_impl<T>(c, 2, cf, xs, &X, eps, cap, &capped));
      anycap |= capped;
    }
    if (o->recursive_residual) {
      // the update of Algorithm alg:pcg as printed: S = trunc(fun(P)), R = trunc(R - a S)
      TPCHK(apply_impl<T>(c, op, &P, &S, eps, cap, sk, &capped));
      anycap |= capped;
      info->op_applies += 1;
      const tp_tensor* rs[2] = {&R, &S};
      double cf[2] = {1.0, -a};
      TPCHK(truncate_impl<T>(c, 2, cf, rs, &R, eps, cap, &capped));
      anycap |= capped;
    } else {
      Term t[2] = {{nullptr, &B, 1.0}, {op, &X, -1.0}};
      TPCHK(combo_impl<T>(c, t, 2, &R, eps, cap, sk, &capped));
      anycap |= capped;
      info->op_applies += 1;
    }
    double rr = 0;
    TPCHK(inner_impl<T>(c, &R, &R, &rr));
    info->rel_res = std::sqrt(std::max(rr, 0.0)) / nb;
    if (o->stop_rule == TP_STOP_RESIDUAL) {
      // the relative residual of the Sec. 6 iteration counts
      info->err_est = info->rel_res;
      if (info->err_est <= o->tau) { converged = true; ++k; break; }
    }
    if (o->stop_rule == TP_STOP_ERROR) {
      // "R sufficiently small": the preconditioned residual Z ~ A_2^-1 R estimates the error of X,
      // so the test ||Z|| <= tau ||X|| bounds the relative error instead of the residual (whose
      // norm under-weights the smooth error components by s_min/s_max).  ||Z|| is taken from the
      // projected core of the product (before its HOSVD), and the product is only completed into Z
      // when the iteration goes on.
      double xx = 0, zz = -1.0;
      TPCHK(inner_impl<T>(c, &X, &X, &xx));
      bool stop_now = false;
      const EarlyStop test = [&](double nz2) {
        zz = nz2;
        info->err_est = std::sqrt(std::max(nz2, 0.0) / std::max(xx, 1e-300));
        stop_now = info->err_est <= o->tau;
        return stop_now;
      };
      TPCHK(apply_impl<T>(c, pre, &R, &Z, eps, cap, sk, &capped, &test));
      info->op_applies += 1;
      if (stop_now) { converged = true; ++k; break; }
      anycap |= capped;
      if (zz < 0.0) {  // the product ended before its projection (a zero sum): Z itself
        TPCHK(inner_impl<T>(c, &Z, &Z, &zz));
        info->err_est = std::sqrt(std::max(zz, 0.0) / std::max(xx, 1e-300));
        if (info->err_est <= o->tau) { converged = true; ++k; break; }
      }
    } else {
      TPCHK(apply_impl<T>(c, pre, &R, &Z, eps, cap, sk, &capped));
      anycap |= capped;
      info->op_applies += 1;
    }
    // Safeguard (not part of the method): once the truncated iteration has reached the floor
    // set by the working precision or by the rank cap, further steps only amplify rounding
    // noise or repeat the truncation error.  The iterate with the smallest estimate is kept, and
    // the loop stops when the estimate has grown 8-fold or has not improved for 5 steps.
    if (info->err_est < best) {
      best = info->err_est;
      kbest = k;
      TPCHK(copy_tensor<T>(c, &X, &Xb));
    } else if (info->err_est > 8.0 * best || k - kbest >= 5) {
      stalled = true;
      ++k;
      break;
    }
    double rz_new = 0;
    TPCHK(inner_impl<T>(c, &R, &Z, &rz_new));
    if (!(rz_new > 0)) { breakdown = "<R,Z>"; breakdown_val = rz_new; ++k; break; }
    const double beta = rz_new / rz;
    rz = rz_new;
    {
      const tp_tensor* xs[2] = {&Z, &P};
      double cf[2] = {1.0, beta};
      TPCHK(truncate_impl<T>(c, 2, cf, xs, &P, eps, cap, &capped));
      anycap |= capped;
    }
  }
  info->iters = k;
  if (!converged && best < info->err_est) {
    TPCHK(copy_tensor<T>(c, &Xb, &X));
    info->err_est = best;
  }
  if (c->spectral) {
    c->spectral = false;
    TPCHK(copy_tensor<T>(c, &X, x));
    for (int m = 0; m < x->d; ++m) TPCHK(dst_cols<T>(c, x->n[m], x->rank[m], (const T*)X.factor[m], (T*)x->factor[m]));
    c->spectral = true;
  } else {
    TPCHK(copy_tensor<T>(c, &X, x));
  }
  for (int m = 0; m < 3; ++m) info->rank[m] = m < x->d ? x->rank[m] : 0;
  if (o->true_residual) {
    // ||B - A_2 X|| / ||B||: the sum is formed and truncated tightly relative to its own norm
    Term t[2] = {{nullptr, &B, 1.0}, {op, &X, -1.0}};
    TPCHK(combo_impl<T>(c, t, 2, &Z, 1e-4, cap, sk, &capped));
    double zz = 0;
    TPCHK(inner_impl<T>(c, &Z, &Z, &zz));
    info->true_rel_res = std::sqrt(std::max(zz, 0.0)) / nb;
  }
  if (!converged) {
    info->status = TP_ENOCONV;
    if (breakdown)
      return fail(TP_ENOCONV, "PCG breakdown after %d iterations: %s = %g (operator or preconditioner not "
                  "positive definite); x holds the best iterate", k, breakdown, breakdown_val);
    if (stalled)
      return fail(TP_ENOCONV, "PCG stalled at error estimate %g > tau=%g after %d iterations (precision or rank-cap "
                  "floor); x holds the best iterate", info->err_est, o->tau, k);
    return fail(TP_ENOCONV, "PCG did not reach tau=%g in %d iterations (error estimate %g); x holds the best iterate",
                o->tau, o->kmax, info->err_est);
  }
  info->status = anycap ? TP_ERANK : TP_OK;
  return TP_OK;
}

}  // namespace

extern "C" tp_status tp_pcg_solve(tp_ctx* c, const tp_symbol* op, const tp_symbol* pre, const tp_cp* b, tp_tensor* x,
                                  const tp_pcg_opts* o, const tp_sketch* sk, tp_pcg_info* info) {
  if (!c || !op || !pre || !b || !x || !o || !sk || !info) return fail(TP_EINVAL, "NULL argument");
  TPCHK(check_tensor(x, "x", false));
  if (op->kind != 0 || pre->kind != 1) return fail(TP_EINVAL, "op/pre symbols swapped");
  if (op->prec != x->prec || pre->prec != x->prec) return fail(TP_EINVAL, "symbol precision differs from x");
  if (b->d != x->d || op->d != x->d) return fail(TP_EINVAL, "dimension mismatch");
  for (int m = 0; m < x->d; ++m)
    if (b->n[m] != x->n[m] || op->n[m] != x->n[m] || pre->n[m] != x->n[m])
      return fail(TP_EINVAL, "grid mismatch in mode %d", m);
  if (o->cap < 1 || o->cap > x->cap) return fail(TP_EINVAL, "opts.cap=%d must be in [1, x.cap=%d]", o->cap, x->cap);
  if (!(o->tau > 0) || o->kmax < 1 || !(o->trunc_tol > 0)) return fail(TP_EINVAL, "invalid PCG options");
  if (o->stop_rule != TP_STOP_ERROR && o->stop_rule != TP_STOP_RESIDUAL)
    return fail(TP_EINVAL, "unknown stop rule %d", o->stop_rule);
  if (o->recursive_residual != 0 && o->recursive_residual != 1)
    return fail(TP_EINVAL, "recursive_residual=%d must be 0 or 1", o->recursive_residual);
  if (o->spectral_domain != 0 && o->spectral_domain != 1)
    return fail(TP_EINVAL, "spectral_domain=%d must be 0 or 1", o->spectral_domain);
  if (o->warm_start != 0 && o->warm_start != 1)
    return fail(TP_EINVAL, "warm_start=%d must be 0 or 1", o->warm_start);
  if (o->warm_start)
    for (int m = 0; m < x->d; ++m)
      if (x->rank[m] < 0 || x->rank[m] > o->cap)
        return fail(TP_EINVAL, "warm start: x.rank[%d]=%d outside [0, opts.cap=%d]", m, x->rank[m], o->cap);
  if (sk->q < 2 || sk->q > kMaxSketch) return fail(TP_EINVAL, "sketch q=%d must be in [2,%d]", sk->q, kMaxSketch);
  if (b->rank < 0 || b->rank > kMaxRank) return fail(TP_EINVAL, "b.rank=%d outside [0,%d]", b->rank, kMaxRank);
  tp_status st = x->prec == TP_FP64 ? pcg_impl<double>(c, op, pre, b, x, o, sk, info)
                                    : pcg_impl<float>(c, op, pre, b, x, o, sk, info);
  if (st != TP_OK && st != TP_ENOCONV) info->status = st;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(TP_EHIP, "stream sync: %s", hipGetErrorString(e));
  if (st == TP_OK && info->status == TP_ERANK) return fail(TP_ERANK, "rank cap reached during the solve");
  return st;
}

// ------------------------------------------------------------------------------ workspace size
extern "C" tp_status tp_workspace_peak(tp_ctx* c, int32_t reset, size_t* peak) {
  if (!c || !peak) return fail(TP_EINVAL, "NULL argument");
  *peak = c->ws_peak;
  if (reset) c->ws_peak = c->ws_top;
  return TP_OK;
}

extern "C" tp_status tp_workspace_query(const tp_symbol_desc* D, const tp_pcg_opts* o, int32_t q, int32_t rb,
                                        size_t* bytes) {
  if (!D || !o || !bytes) return fail(TP_EINVAL, "NULL argument");
  if (D->d != 2 && D->d != 3) return fail(TP_EINVAL, "d=%d must be 2 or 3", D->d);
  if (o->cap < 1 || q < 2 || rb < 0) return fail(TP_EINVAL, "cap, sketch width or rhs rank out of range");
  const int d = D->d;
  double nmax = 0, nsum = 0;
  for (int m = 0; m < d; ++m) {
    if (D->n[m] < 1) return fail(TP_EINVAL, "n[%d]=%d", m, D->n[m]);
    nmax = std::max(nmax, (double)D->n[m]);
    nsum += D->n[m];
  }
  const double T = D->prec == TP_FP64 ? 8.0 : 4.0, cap = o->cap, Q = q, B = std::max(rb, 1);
  const int kop = D->method == TP_SYM_SINC ? (D->sinc_kl > 0 ? D->sinc_kl : 60) + (D->sinc_kr > 0 ? D->sinc_kr : 20) + 2
                                           : (D->op_terms > 0 ? D->op_terms : 32) + 1;
  const int kpre = D->pre_terms > 0 ? D->pre_terms : 12;
  const double rop = (double)d * kop + 1, rpre = D->pre_rank > 0 ? std::pow((double)D->pre_rank, d - 1) : kpre;
  const double R = std::max(rop, rpre);
  auto pw = [d](double v) { return d == 3 ? v * v * v : v * v; };
  // the iteration's tensors (B, X, best X, R, P, Z, S and the caller-visible copy)
  const double tens = 8.0 * (pw(cap) * T + nsum * cap * T);
  // right-hand side to Tucker form: bases, projected factors, Khatri-Rao product, core, HOSVD
  const double fromcp = 4.0 * d * nmax * B * 8 + 4.0 * d * B * B * 8 + cap * B * B * 8 + 6.0 * pw(B) * 8;
  // one sketched product of two terms: inputs in sine coordinates, sketch contractions, sketches
  // and their bases, projection (the two batched core contractions dominate), HOSVD of the core
  const double term = d * nmax * cap * T + pw(cap) * T + d * cap * R * Q * T;
  // (3D: the core contracted with two sketches, r^2 R q, and the two projection stages R q r^2 and
  // R r q^2; 2D: one stage each, r R q and R q r)
  const double sk2 = d == 3 ? cap * cap * R * Q * T : 0.0;
  const double proj = d == 3 ? (R * Q * cap * cap + R * cap * Q * Q) * T : R * Q * cap * T;
  // FP32-accumulated sketches: one partial sum per 512 of the cap R contraction length
  const double skparts = D->prec == TP_FP64 ? 0.0 : d * nmax * Q * 4.0 * std::ceil(cap * R / 512.0);
  const double combo = skparts + d * nmax * Q * T + 2.0 * term + sk2 + cap * R * Q * T + pw(cap) * T +
                       d * nmax * Q * 8 * 4 + 4.0 * d * Q * Q * 8 + d * nmax * Q * T + pw(Q) * T +
                       d * Q * cap * R * T + proj + 6.0 * pw(Q) * 8 + 4.0 * d * Q * Q * 8 + d * nmax * cap * T;
  // symbol inner product (Grams per term, two batched core contractions)
  const double isym = 2.0 * d * nmax * cap * T + d * cap * cap * R * 8 + 3.0 * pw(cap) * 8 +
                      (d == 3 ? 2.0 : 1.0) * R * pw(cap) * 8;
  // sum of two iterates: concatenated factors, bases, block core and its HOSVD
  const double c2 = 2 * cap;
  const double sum = d * nmax * c2 * 8 * 4 + 4.0 * d * c2 * c2 * 8 + 6.0 * pw(c2) * 8 + d * nmax * c2 * T;
  // least-squares fits of the symbols (design matrices of the candidates)
  const double fits = 15.0 * 1000 * 64 * 8 * 2 + 15.0 * 64 * 64 * 8 * 4;
  // the operator and preconditioner symbols (factors and weighted factors) in a worker's arena
  const double syms = 4.0 * d * nmax * R * T;
  const double total = tens + fromcp + syms + std::max(std::max(combo, isym), std::max(sum, fits)) + (64 << 20);
  *bytes = (size_t)(1.25 * total);
  return TP_OK;
}

// ------------------------------------------------------------------------------ batched solves
// The symbols are a function of the descriptor alone: descriptors equal field by field build the
// same symbols.
static bool same_desc(const tp_symbol_desc& a, const tp_symbol_desc& b) {
  if (a.d != b.d) return false;
  for (int m = 0; m < a.d && m < 3; ++m)
    if (a.n[m] != b.n[m]) return false;
  return a.alpha == b.alpha && a.c_neg == b.c_neg && a.c_pos == b.c_pos && a.method == b.method &&
         a.op_terms == b.op_terms && a.pre_terms == b.pre_terms && a.sinc_kl == b.sinc_kl &&
         a.sinc_kr == b.sinc_kr && a.sinc_h == b.sinc_h && a.prec == b.prec && a.c0 == b.c0 && a.beta == b.beta &&
         a.pre_rank == b.pre_rank && a.directional == b.directional;
}

// Independent problems run concurrently on `streams` HIP streams (default priority), each
// stream owned by a worker thread with its own context and workspace; workers take the next
// problem from a shared counter, so uneven problems balance themselves.  Problems that share a
// descriptor (several right-hand sides of one operator) share one build of its symbols: it runs on
// the calling context before the workers start, and the workers only read the symbols.
extern "C" tp_status tp_pcg_solve_batched(tp_ctx* c, int32_t count, const tp_symbol_desc* descs, const tp_cp* bs,
                                          tp_tensor* xs, const tp_pcg_opts* opts, const tp_sketch* sks,
                                          tp_pcg_info* infos, int32_t streams, size_t workspace_per_stream) {
  if (!c || (count > 0 && (!descs || !bs || !xs || !opts || !sks || !infos))) return fail(TP_EINVAL, "NULL argument");
  if (count < 0) return fail(TP_EINVAL, "count < 0");
  if (streams < 1 || streams > 16) return fail(TP_EINVAL, "streams=%d must be in [1,16]", streams);
  if (count == 0) return TP_OK;
  HIPCHK(hipStreamSynchronize(c->stream));
  const int nw = std::min<int>(streams, count);
  const size_t wsz = workspace_per_stream ? workspace_per_stream : (size_t(2) << 30);
  // worker contexts (stream, workspace, sine tables) are kept in c for later calls with the same
  // workspace size; more workers are added when a call asks for more streams
  if (c->worker_ws != wsz) {
    release_workers(c);
    c->worker_ws = wsz;
  }
  while ((int)c->workers.size() < nw) {
    hipStream_t sw = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&sw, hipStreamNonBlocking));
    tp_ctx* cw = nullptr;
    tp_status st = tp_create(c->device, sw, wsz, &cw);
    if (st != TP_OK) {
      (void)hipStreamDestroy(sw);
      return st;
    }
    cw->prof = false;
    cw->sym_arena = true;
    c->workers.push_back(cw);
    c->worker_streams.push_back(sw);
  }
  const std::vector<tp_ctx*>& ctxs = c->workers;
  // descriptors of two or more problems: symbols built once here (freed after the workers end)
  struct Shared { tp_symbol* op = nullptr; tp_symbol* pre = nullptr; tp_status st = TP_OK; std::string msg; };
  std::vector<int> group(count, -1);
  std::vector<Shared> shared;
  for (int i = 0; i < count; ++i) {
    if (group[i] >= 0) continue;
    bool more = false;
    for (int j = i + 1; j < count && !more; ++j) more = same_desc(descs[i], descs[j]);
    if (!more) continue;
    const int g = (int)shared.size();
    for (int j = i; j < count; ++j)
      if (group[j] < 0 && same_desc(descs[i], descs[j])) group[j] = g;
    Shared sh;
    double errs[2];
    sh.st = tp_symbol_build(c, &descs[i], &sh.op, &sh.pre, errs);
    if (sh.st != TP_OK) sh.msg = g_err;  // the error text is per thread
    shared.push_back(sh);
  }
  auto free_shared = [&]() {
    for (Shared& sh : shared) {
      if (sh.op) tp_symbol_free(sh.op);
      if (sh.pre) tp_symbol_free(sh.pre);
    }
  };
  std::atomic<int> next(0);
  std::vector<tp_status> wst(nw, TP_OK);
  std::vector<std::string> werr(nw);
  auto worker = [&](int w) {
    (void)hipSetDevice(c->device);
    tp_ctx* cw = ctxs[w];
    for (;;) {
      int i = next.fetch_add(1);
      if (i >= count) break;
      tp_symbol *op = nullptr, *pre = nullptr;
      double errs[2];
      const size_t mark = cw->ws_top;  // the symbols go to the workspace below the solve's scopes
      const bool own = group[i] < 0;
      tp_status st;
      if (own) {
        st = tp_symbol_build(cw, &descs[i], &op, &pre, errs);
      } else {
        op = shared[group[i]].op;
        pre = shared[group[i]].pre;
        st = shared[group[i]].st;
      }
      const bool indefinite = st == TP_EINDEF;  // symbols returned; the solve may break down
      if (st == TP_OK || indefinite) {
        st = tp_pcg_solve(cw, op, pre, &bs[i], &xs[i], &opts[i], &sks[i], &infos[i]);
        if (indefinite && st == TP_OK) infos[i].status = st = TP_EINDEF;
      } else {
        infos[i].status = st;
      }
      if (own && op) tp_symbol_free(op);
      if (own && pre) tp_symbol_free(pre);
      (void)hipStreamSynchronize(cw->stream);  // the next problem reuses the symbols' workspace
      cw->ws_top = mark;
      if (st != TP_OK && st != TP_ERANK && st != TP_ENOCONV && st != TP_EINDEF && wst[w] == TP_OK) {
        wst[w] = st;
        werr[w] = (!own && !op) ? shared[group[i]].msg : g_err;
      }
    }
  };
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w) th.emplace_back(worker, w);
  for (auto& t : th) t.join();
  free_shared();
  tp_status res = TP_OK;
  std::string msg;
  for (int w = 0; w < nw; ++w)
    if (wst[w] != TP_OK && res == TP_OK) { res = wst[w]; msg = werr[w]; }
  if (res != TP_OK) return fail(res, "batched solve: %s", msg.c_str());
  return TP_OK;
}
