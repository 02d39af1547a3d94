// Device kernels of the rank-structured PCG solver (gfx950, wave64).
//
//  * gemm        : LDS-tiled batched GEMM with optional face-split operands (the
//                  Hadamard products of the low-rank product eqn:Lap3DtimesX are
//                  formed while the tile is loaded, never in memory).
//  * dst1        : orthonormal DST-I of many columns, radix-2 FFT of length N/2 in LDS.
//  * syev        : batched cyclic Jacobi eigensolver in FP64, matrix resident in LDS.
//  * symbol      : 1D spectra, exponential-sum factors, sinc nodes, least-squares design.
#include "tp_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

namespace tpk {

// ---------------------------------------------------------------------------------------------
// GEMM
// ---------------------------------------------------------------------------------------------
constexpr int GBM = 64, GBN = 64, GBK = 16, GTHREADS = 256;

template <typename T>
__device__ __forceinline__ T fs_load(const FaceSplit<T>& F, int row, int c) {
  int a = c % F.r1, b = c / F.r1;
  T v = F.x1[row + (long)F.ld1 * a] * F.x2[row + (long)F.ld2 * b];
  if (F.w) v = (T)((double)v * F.w[b]);
  return v;
}

template <typename TA, typename TB, typename TC, typename Tacc>
__global__ __launch_bounds__(GTHREADS) void k_gemm(GemmArgs<TA, TB, TC, Tacc> g) {
  __shared__ Tacc As[GBK][GBM + 1];
  __shared__ Tacc Bs[GBK][GBN + 1];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const int b = blockIdx.z / g.splits;
  const int sp = blockIdx.z - b * g.splits;
  const int kbeg = sp * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const TA* A = g.A ? g.A + (long)(b / g.divA) * g.sA : nullptr;
  const TB* B = g.B ? g.B + (long)(b / g.divB) * g.sB : nullptr;
  FaceSplit<TA> FA = g.FA;
  FaceSplit<TB> FB = g.FB;
  if (g.fsA) { FA.x1 += (long)(b / g.divA) * g.sA; FA.x2 += (long)(b / g.divA) * g.sA; }
  if (g.fsB) { FB.x1 += (long)(b / g.divB) * g.sB; FB.x2 += (long)(b / g.divB) * g.sB; }
  TC* C = g.C + (long)b * g.sC;
  const int tm = tid % 16, tn = tid / 16;
  Tacc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0;

  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
    // A tile: op(A)[m0+m, k0+kk]
    if (!g.tA) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int m = tid % 64, kk = tid / 64 + 4 * i;
        int row = m0 + m, col = k0 + kk;
        Tacc v = 0;
        if (row < g.M && col < kend) v = g.fsA ? (Tacc)fs_load(FA, row, col) : (Tacc)A[row + (long)g.lda * col];
        As[kk][m] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int kk = tid % 16, m = tid / 16 + 16 * i;
        int row = m0 + m, col = k0 + kk;
        Tacc v = 0;
        if (row < g.M && col < kend) v = (Tacc)A[col + (long)g.lda * row];
        As[kk][m] = v;
      }
    }
    // B tile: op(B)[k0+kk, n0+n]
    if (!g.tB) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int kk = tid % 16, n = tid / 16 + 16 * i;
        int row = k0 + kk, col = n0 + n;
        Tacc v = 0;
        if (row < kend && col < g.N) v = g.fsB ? (Tacc)fs_load(FB, row, col) : (Tacc)B[row + (long)g.ldb * col];
        Bs[kk][n] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int n = tid % 64, kk = tid / 64 + 4 * i;
        int row = k0 + kk, col = n0 + n;
        Tacc v = 0;
        if (row < kend && col < g.N) v = (Tacc)B[col + (long)g.ldb * row];
        Bs[kk][n] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; ++kk) {
      Tacc a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tn + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
  if (g.part) {
    // split-K: raw partial sums, reduced by k_gemm_reduce
    Tacc* Pp = g.part + (long)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int row = m0 + tm + 16 * i;
      if (row >= g.M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int col = n0 + tn + 16 * j;
        if (col < g.N) Pp[row + (long)g.M * col] = acc[i][j];
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int row = m0 + tm + 16 * i;
    if (row >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int col = n0 + tn + 16 * j;
      if (col >= g.N) continue;
      long o = row + (long)g.ldc * col;
      Tacc v = g.alpha * acc[i][j];
      if (g.beta != (Tacc)0) v += g.beta * (Tacc)C[o];
      C[o] = (TC)v;
    }
  }
}

// MFMA variant: the same tiling and loaders, and each of the 4 waves owns a 32x32 quarter of
// the 64x64 tile as 2x2 MFMA 16x16x4 blocks (FP32 or FP64 matrix cores).  Operand layout of the
// single-block 16x16x4 instructions: lane l supplies A[l%16][l/16] and B[l/16][l%16]; result
// element v of lane l is D[4*(l/16)+v][l%16] for FP32 and D[l/16+4v][l%16] for FP64 (checked
// on gfx950 with a one-wavefront probe).
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename TA, typename TB, typename TC, typename Tacc>
__global__ __launch_bounds__(GTHREADS) void k_gemm_mfma(GemmArgs<TA, TB, TC, Tacc> g) {
  typedef typename std::conditional<std::is_same<Tacc, double>::value, d4_t, f4_t>::type V4;
  __shared__ Tacc As[GBK][GBM + 4];
  __shared__ Tacc Bs[GBK][GBN + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const int b = blockIdx.z / g.splits;
  const int sp = blockIdx.z - b * g.splits;
  const int kbeg = sp * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const TA* A = g.A ? g.A + (long)(b / g.divA) * g.sA : nullptr;
  const TB* B = g.B ? g.B + (long)(b / g.divB) * g.sB : nullptr;
  FaceSplit<TA> FA = g.FA;
  FaceSplit<TB> FB = g.FB;
  if (g.fsA) { FA.x1 += (long)(b / g.divA) * g.sA; FA.x2 += (long)(b / g.divA) * g.sA; }
  if (g.fsB) { FB.x1 += (long)(b / g.divB) * g.sB; FB.x2 += (long)(b / g.divB) * g.sB; }
  TC* C = g.C + (long)b * g.sC;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
    if (!g.tA) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int m = tid % 64, kk = tid / 64 + 4 * i;
        int row = m0 + m, col = k0 + kk;
        Tacc v = 0;
        if (row < g.M && col < kend) v = g.fsA ? (Tacc)fs_load(FA, row, col) : (Tacc)A[row + (long)g.lda * col];
        As[kk][m] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int kk = tid % 16, m = tid / 16 + 16 * i;
        int row = m0 + m, col = k0 + kk;
        Tacc v = 0;
        if (row < g.M && col < kend) v = (Tacc)A[col + (long)g.lda * row];
        As[kk][m] = v;
      }
    }
    if (!g.tB) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int kk = tid % 16, n = tid / 16 + 16 * i;
        int row = k0 + kk, col = n0 + n;
        Tacc v = 0;
        if (row < kend && col < g.N) v = g.fsB ? (Tacc)fs_load(FB, row, col) : (Tacc)B[row + (long)g.ldb * col];
        Bs[kk][n] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int n = tid % 64, kk = tid / 64 + 4 * i;
        int row = k0 + kk, col = n0 + n;
        Tacc v = 0;
        if (row < kend && col < g.N) v = (Tacc)B[col + (long)g.ldb * row];
        Bs[kk][n] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 4) {
      const int kr = kk + (lane >> 4), c16 = lane & 15;
      Tacc a0 = As[kr][wm + c16], a1 = As[kr][wm + 16 + c16];
      Tacc b0 = Bs[kr][wn + c16], b1 = Bs[kr][wn + 16 + c16];
      acc[0][0] = mfma16(a0, b0, acc[0][0]);
      acc[0][1] = mfma16(a0, b1, acc[0][1]);
      acc[1][0] = mfma16(a1, b0, acc[1][0]);
      acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  const bool f64 = std::is_same<Tacc, double>::value;
  const int rbase = f64 ? (lane >> 4) : 4 * (lane >> 4), rstep = f64 ? 4 : 1, cl = lane & 15;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row = m0 + wm + 16 * i + rbase + rstep * v;
        int col = n0 + wn + 16 * j + cl;
        if (row >= g.M || col >= g.N) continue;
        Tacc x = acc[i][j][v];
        if (g.part) {
          g.part[(long)blockIdx.z * g.M * g.N + row + (long)g.M * col] = x;
        } else {
          long o = row + (long)g.ldc * col;
          Tacc y = g.alpha * x;
          if (g.beta != (Tacc)0) y += g.beta * (Tacc)C[o];
          C[o] = (TC)y;
        }
      }
}

template <typename TC, typename Tacc>
__global__ void k_gemm_reduce(int M, int N, int splits, const Tacc* part, Tacc alpha, Tacc beta, TC* C, int ldc,
                              long sC) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int b = blockIdx.y;
  long mn = (long)M * N;
  if (e >= mn) return;
  int row = (int)(e % M), col = (int)(e / M);
  const Tacc* p = part + (long)b * splits * mn + e;
  Tacc acc = 0;
  for (int s = 0; s < splits; ++s) acc += p[(long)s * mn];
  long o = (long)b * sC + row + (long)ldc * col;
  Tacc v = alpha * acc;
  if (beta != (Tacc)0) v += beta * (Tacc)C[o];
  C[o] = (TC)v;
}

static int g_use_mfma = 1;
bool gemm_use_mfma() { return g_use_mfma != 0; }
void gemm_set_mfma(int on) { g_use_mfma = on; }

template <typename TA, typename TB, typename TC, typename Tacc>
hipError_t gemm(const GemmArgs<TA, TB, TC, Tacc>& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) {
    // C = beta*C: handled by a degenerate launch with K = 0 (the loop body is skipped).
  }
  GemmArgs<TA, TB, TC, Tacc> h = g;
  if (h.splits < 1 || !h.part) { h.splits = 1; h.part = nullptr; }
  h.kchunk = h.splits > 1 ? ((h.K + h.splits - 1) / h.splits + GBK - 1) / GBK * GBK : h.K;
  dim3 grid((h.M + GBM - 1) / GBM, (h.N + GBN - 1) / GBN, h.batch * h.splits);
  if (gemm_use_mfma())
    hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TC, Tacc>), grid, dim3(GTHREADS), 0, s, h);
  else
    hipLaunchKernelGGL((k_gemm<TA, TB, TC, Tacc>), grid, dim3(GTHREADS), 0, s, h);
  if (h.splits > 1) {
    long mn = (long)h.M * h.N;
    dim3 rg((mn + 255) / 256, h.batch);
    hipLaunchKernelGGL((k_gemm_reduce<TC, Tacc>), rg, dim3(256), 0, s, h.M, h.N, h.splits, (const Tacc*)h.part,
                       h.alpha, h.beta, h.C, h.ldc, h.sC);
  }
  return hipGetLastError();
}

template hipError_t gemm<double, double, double, double>(const GemmArgs<double, double, double, double>&, hipStream_t);
template hipError_t gemm<float, float, float, float>(const GemmArgs<float, float, float, float>&, hipStream_t);
template hipError_t gemm<float, float, double, double>(const GemmArgs<float, float, double, double>&, hipStream_t);
template hipError_t gemm<double, double, float, double>(const GemmArgs<double, double, float, double>&, hipStream_t);

// ---------------------------------------------------------------------------------------------
// DST-I via a length-N/2 complex FFT (N = n+1 a power of two).
//
// With x_0 = x_N = 0 and v_j = sin(pi j/N)(x_j + x_{N-j}) + (x_j - x_{N-j})/2, the real DFT
// V_k = sum_j v_j e^{-2 pi i jk/N} gives the unnormalised sine sums y_k = sum_j x_j sin(pi jk/N)
// as y_{2k} = -Im V_k and y_{2k+1} = y_{2k-1} + Re V_k, y_1 = Re V_0 / 2.  The real DFT of
// length N comes from the complex FFT of z_m = v_{2m} + i v_{2m+1} (length L = N/2).
// ---------------------------------------------------------------------------------------------
template <typename T>
struct C2 { T re, im; };

template <typename T>
__global__ void k_dst_table(int N, T* tab) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) {
    double sv, cv;
    sincospi((double)m / (double)N, &sv, &cv);
    tab[2 * m] = (T)cv;
    tab[2 * m + 1] = (T)sv;
  }
}

template <typename T>
hipError_t dst_table(int N, T* tab, hipStream_t s) {
  hipLaunchKernelGGL(k_dst_table<T>, dim3((N + 255) / 256), dim3(256), 0, s, N, tab);
  return hipGetLastError();
}
template hipError_t dst_table<double>(int, double*, hipStream_t);
template hipError_t dst_table<float>(int, float*, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void k_dst1(int N, int logL, int cols, int cpw, const T* in,
                                              int ldin, T* out, int ldout,
                                              const T* __restrict__ tab, T scale) {
  extern __shared__ char smem_raw[];
  C2<T>* X = reinterpret_cast<C2<T>*>(smem_raw);
  const int L = N >> 1;
  const int tot = cpw * L;
  T* partial = reinterpret_cast<T*>(X + tot);  // 256 chunk totals
  const int tid = threadIdx.x;
  const int col0 = blockIdx.x * cpw;

  auto xval = [&](int c, int j) -> T {  // x_j, 1-based, zero outside 1..N-1
    int col = col0 + c;
    if (j <= 0 || j >= N || col >= cols) return (T)0;
    return in[(j - 1) + (long)ldin * col];
  };
  // pre-processing and bit-reversed load
  for (int e = tid; e < tot; e += 256) {
    int c = e / L, m = e - c * L;
    C2<T> z;
    int j0 = 2 * m, j1 = 2 * m + 1;
    T a0 = xval(c, j0), b0 = xval(c, N - j0);
    T a1 = xval(c, j1), b1 = xval(c, N - j1);
    T s0 = tab[2 * j0 + 1], s1 = tab[2 * j1 + 1];
    z.re = s0 * (a0 + b0) + (T)0.5 * (a0 - b0);
    z.im = s1 * (a1 + b1) + (T)0.5 * (a1 - b1);
    int rm = logL ? (int)(__brev((unsigned)m) >> (32 - logL)) : 0;
    X[c * L + rm] = z;
  }
  __syncthreads();
  // radix-2 decimation-in-time butterflies
  for (int st = 1; st <= logL; ++st) {
    int half = 1 << (st - 1);
    int tstep = N / half;  // twiddle e^{-i pi pos/half} = tab[pos*N/half]
    int nb = tot >> 1;
    for (int e = tid; e < nb; e += 256) {
      int c = e / (L >> 1), bidx = e - c * (L >> 1);
      int grp = bidx / half, pos = bidx - grp * half;
      int i0 = c * L + grp * 2 * half + pos, i1 = i0 + half;
      T wr = tab[2 * (pos * tstep)], wi = -tab[2 * (pos * tstep) + 1];
      C2<T> a = X[i0], bq = X[i1];
      C2<T> t;
      t.re = bq.re * wr - bq.im * wi;
      t.im = bq.re * wi + bq.im * wr;
      X[i0].re = a.re + t.re; X[i0].im = a.im + t.im;
      X[i1].re = a.re - t.re; X[i1].im = a.im - t.im;
    }
    __syncthreads();
  }
  // post-processing: V_k for k = 0..L/2 and its partner L-k, then y values in place
  const int hp = (L >> 1) + 1;
  for (int e = tid; e < cpw * hp; e += 256) {
    int c = e / hp, k = e - c * hp;
    int kc = (L - k) % L;
    C2<T> Zk = X[c * L + k], Zc = X[c * L + kc];
    // E = (Zk + conj(Zc))/2, O = (Zk - conj(Zc))/(2i)
    T Er = (T)0.5 * (Zk.re + Zc.re), Ei = (T)0.5 * (Zk.im - Zc.im);
    T Or = (T)0.5 * (Zk.im + Zc.im), Oi = (T)-0.5 * (Zk.re - Zc.re);
    // w = e^{-2 pi i k/N} = tab[2k]
    T cr = tab[2 * (2 * k % N)], ci = -tab[2 * (2 * k % N) + 1];
    if (2 * k >= N) { cr = -1; ci = 0; }  // k = L/2 when L = 1 is impossible; guard only
    T wOr = cr * Or - ci * Oi, wOi = cr * Oi + ci * Or;
    T Vr = Er + wOr, Vi = Ei + wOi;        // V_k
    if (k == 0) {
      X[c * L].re = (T)0.5 * Vr;            // y_1 seed
      X[c * L].im = 0;                      // y_0 unused
    } else {
      X[c * L + k].re = Vr;
      X[c * L + k].im = -Vi;                // y_{2k}
      if (kc != k) {
        // V_{L-k} = conj(E - w O)
        T Ur = Er - wOr, Ui = -(Ei - wOi);
        X[c * L + kc].re = Ur;
        X[c * L + kc].im = -Ui;
      }
    }
  }
  __syncthreads();
  // segmented inclusive scan of X[].re per column (odd outputs)
  const int chunk = tot / 256;  // >= 1, divides L
  {
    int beg = tid * chunk;
    T run = 0;
    for (int i = 0; i < chunk; ++i) { run += X[beg + i].re; X[beg + i].re = run; }
    partial[tid] = run;
  }
  __syncthreads();
  {
    int beg = tid * chunk;
    int cstart = (beg / L) * L;  // first element of this column
    int t0 = cstart / chunk;
    T off = 0;
    for (int t = t0; t < tid; ++t) off += partial[t];
    for (int i = 0; i < chunk; ++i) X[beg + i].re += off;
  }
  __syncthreads();
  for (int e = tid; e < tot; e += 256) {
    int c = e / L, k = e - c * L;
    int col = col0 + c;
    if (col >= cols) continue;
    out[2 * k + (long)ldout * col] = scale * X[e].re;              // y_{2k+1}
    if (k >= 1) out[2 * k - 1 + (long)ldout * col] = scale * X[e].im;  // y_{2k}
  }
}

template <typename T>
hipError_t dst1(int N, int cols, const T* in, int ldin, T* out, int ldout, const T* tab, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  int L = N / 2;
  int logL = 0;
  while ((1 << logL) < L) ++logL;
  int cpw = L >= 256 ? 1 : 256 / L;
  size_t shm = (size_t)cpw * L * sizeof(C2<T>) + 256 * sizeof(T);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dst1<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  T scale = (T)sqrt(2.0 / (double)N);
  int blocks = (cols + cpw - 1) / cpw;
  hipLaunchKernelGGL(k_dst1<T>, dim3(blocks), dim3(256), shm, s, N, logL, cols, cpw, in, ldin, out, ldout, tab, scale);
  return hipGetLastError();
}
template hipError_t dst1<double>(int, int, const double*, int, double*, int, const double*, hipStream_t);
template hipError_t dst1<float>(int, int, const float*, int, float*, int, const float*, hipStream_t);

// ---------------------------------------------------------------------------------------------
// Cyclic Jacobi eigensolver (FP64), round-robin parallel ordering, A in LDS, V in global.
// ---------------------------------------------------------------------------------------------
constexpr int EIG_LDS_MAX = 128;   // matrices up to this size live in LDS
constexpr int EIG_MAX = 256;       // larger ones (up to this) live in global scratch

__device__ __forceinline__ int rr_index(int j, int s, int Kp) {
  // circle method: position 0 fixed, others rotate by s
  return j == 0 ? 0 : ((j - 1 + s) % (Kp - 1)) + 1;
}

// One workgroup per matrix.  A (Kp x Kp) in LDS when SMEM, else in J.work (global, L2 resident).
template <bool SMEM>
__global__ __launch_bounds__(256) void k_syev(const EigJob* jobs) {
  extern __shared__ double sm[];
  const EigJob J = jobs[blockIdx.x];
  const int K = J.K;
  const int tid = threadIdx.x;
  if (K <= 0) return;
  const int Kp = (K + 1) & ~1;  // even
  double* A = SMEM ? sm : J.work;                 // Kp x Kp, ld Kp
  double* cs = SMEM ? sm + Kp * Kp : sm;          // Kp/2 pairs: c, s
  int* pp = reinterpret_cast<int*>(cs + Kp);      // Kp/2 pairs: p, q
  double* red = reinterpret_cast<double*>(pp + Kp);  // 256 reduction slots
  __shared__ int done;
  __shared__ double thr;
  double* V = J.v;
  for (int e = tid; e < Kp * Kp; e += 256) {
    int i = e % Kp, j = e / Kp;
    A[e] = (i < K && j < K) ? J.a[i + (long)K * j] : 0.0;
  }
  for (int e = tid; e < K * K; e += 256) {
    int i = e % K, j = e / K;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int np = Kp / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test: off-diagonal Frobenius norm vs total
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < Kp * Kp; e += 256) {
      int i = e % Kp, j = e / Kp;
      double v = A[e] * A[e];
      tot += v;
      if (i != j) off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) { if (tid < w) red[tid] += red[tid + w]; __syncthreads(); }
    double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) { if (tid < w) red[tid] += red[tid + w]; __syncthreads(); }
    double tots = red[0];
    // stop once the off-diagonal part is below J.tol ||A||_F (default 1e-14; the FP64 rounding
    // floor of the rotations is about K * 1e-16 ||A||_F); rotations below 1e-16 ||A||_F are skipped
    if (tid == 0) {
      const double t2 = J.tol > 0 ? J.tol * J.tol : 1e-28;
      done = (offs <= t2 * tots || tots == 0.0) ? 1 : 0;
      thr = 1e-16 * sqrt(tots);
    }
    __syncthreads();
    if (done) break;
    for (int st = 0; st < Kp - 1; ++st) {
      for (int pr = tid; pr < np; pr += 256) {
        int p = rr_index(pr, st, Kp), q = rr_index(Kp - 1 - pr, st, Kp);
        if (p > q) { int t = p; p = q; q = t; }
        double apq = A[p + Kp * q], app = A[p + Kp * p], aqq = A[q + Kp * q];
        double c = 1.0, s = 0.0;
        if (q < K && fabs(apq) > thr && fabs(apq) > 1e-300) {
          double tau = (aqq - app) / (2.0 * apq);
          double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[2 * pr] = c; cs[2 * pr + 1] = s;
        pp[2 * pr] = p; pp[2 * pr + 1] = q;
      }
      __syncthreads();
      // rows: new row p = c row_p - s row_q ; new row q = s row_p + c row_q
      for (int e = tid; e < np * Kp; e += 256) {
        int pr = e / Kp, j = e - pr * Kp;
        double c = cs[2 * pr], s = cs[2 * pr + 1];
        if (s == 0.0) continue;
        int p = pp[2 * pr], q = pp[2 * pr + 1];
        double ap = A[p + Kp * j], aq = A[q + Kp * j];
        A[p + Kp * j] = c * ap - s * aq;
        A[q + Kp * j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int e = tid; e < np * Kp; e += 256) {
        int pr = e / Kp, i = e - pr * Kp;
        double c = cs[2 * pr], s = cs[2 * pr + 1];
        if (s == 0.0) continue;
        int p = pp[2 * pr], q = pp[2 * pr + 1];
        double ap = A[i + Kp * p], aq = A[i + Kp * q];
        A[i + Kp * p] = c * ap - s * aq;
        A[i + Kp * q] = s * ap + c * aq;
      }
      for (int e = tid; e < np * K; e += 256) {
        int pr = e / K, i = e - pr * K;
        double c = cs[2 * pr], s = cs[2 * pr + 1];
        if (s == 0.0) continue;
        int p = pp[2 * pr], q = pp[2 * pr + 1];
        if (q >= K) continue;
        double vp = V[i + (long)K * p], vq = V[i + (long)K * q];
        V[i + (long)K * p] = c * vp - s * vq;
        V[i + (long)K * q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // sort eigenvalues descending (ties by index): rank of each diagonal entry
  double* diag = cs;  // reuse (Kp entries)
  for (int i = tid; i < K; i += 256) diag[i] = A[i + Kp * i];
  __syncthreads();
  int* rk = pp;
  for (int i = tid; i < K; i += 256) {
    double di = diag[i];
    int r = 0;
    for (int j = 0; j < K; ++j) {
      double dj = diag[j];
      if (dj > di || (dj == di && j < i)) ++r;
    }
    rk[i] = r;
  }
  __syncthreads();
  // copy V into A's storage (A no longer needed) then write permuted
  for (int e = tid; e < K * K; e += 256) A[e] = V[e];
  __syncthreads();
  for (int e = tid; e < K * K; e += 256) {
    int i = e % K, j = e / K;
    V[i + (long)K * rk[j]] = A[e];
  }
  for (int i = tid; i < K; i += 256) J.w[rk[i]] = diag[i];
}

// Small matrices (K <= 96): A and V both resident in LDS (FP64), 512 threads, and every step
// updates 2x2 blocks B_ij <- J_i^T B_ij J_j of the pair partition, so one barrier separates
// the rotation parameters from the update and no element is touched by two threads.
constexpr int EIG_SMALL = 96;
constexpr int EIG_NT = 512;

__global__ __launch_bounds__(EIG_NT) void k_syev_small(const EigJob* jobs) {
  extern __shared__ double sm[];
  const EigJob J = jobs[blockIdx.x];
  const int K = J.K;
  const int tid = threadIdx.x;
  if (K <= 0) return;
  const int Kp = (K + 1) & ~1;
  const int np = Kp / 2;
  double* A = sm;                    // Kp x Kp
  double* V = A + Kp * Kp;           // Kp x Kp (rows = original basis)
  double* cs = V + Kp * Kp;          // np pairs (c, s)
  int* pp = reinterpret_cast<int*>(cs + 2 * np);  // np pairs (p, q)
  double* red = reinterpret_cast<double*>(pp + 2 * np);
  __shared__ int done;
  __shared__ double thr;
  for (int e = tid; e < Kp * Kp; e += EIG_NT) {
    int i = e % Kp, j = e / Kp;
    A[e] = (i < K && j < K) ? J.a[i + (long)K * j] : 0.0;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < Kp * Kp; e += EIG_NT) {
      int i = e % Kp, j = e / Kp;
      double v = A[e] * A[e];
      tot += v;
      if (i != j) off += v;
    }
    red[tid] = off;
    red[tid + EIG_NT] = tot;
    __syncthreads();
    for (int w = EIG_NT / 2; w > 0; w >>= 1) {
      if (tid < w) { red[tid] += red[tid + w]; red[tid + EIG_NT] += red[tid + EIG_NT + w]; }
      __syncthreads();
    }
    if (tid == 0) {
      const double t2 = J.tol > 0 ? J.tol * J.tol : 1e-28;
      done = (red[0] <= t2 * red[EIG_NT] || red[EIG_NT] == 0.0) ? 1 : 0;
      thr = 1e-16 * sqrt(red[EIG_NT]);
    }
    __syncthreads();
    if (done) break;
    for (int st = 0; st < Kp - 1; ++st) {
      for (int pr = tid; pr < np; pr += EIG_NT) {
        int p = rr_index(pr, st, Kp), q = rr_index(Kp - 1 - pr, st, Kp);
        if (p > q) { int t = p; p = q; q = t; }
        double apq = A[p + Kp * q], app = A[p + Kp * p], aqq = A[q + Kp * q];
        double c = 1.0, s = 0.0;
        if (q < K && fabs(apq) > thr && fabs(apq) > 1e-300) {
          double tau = (aqq - app) / (2.0 * apq);
          double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[2 * pr] = c; cs[2 * pr + 1] = s;
        pp[2 * pr] = p; pp[2 * pr + 1] = q;
      }
      __syncthreads();
      // blocks (i, j) of the pair partition: rows {p_i, q_i} x columns {p_j, q_j}
      for (int e = tid; e < np * np; e += EIG_NT) {
        int bi = e % np, bj = e / np;
        double ci = cs[2 * bi], si = cs[2 * bi + 1], cj = cs[2 * bj], sj = cs[2 * bj + 1];
        if (si == 0.0 && sj == 0.0) continue;
        int pi = pp[2 * bi], qi = pp[2 * bi + 1], pj = pp[2 * bj], qj = pp[2 * bj + 1];
        double a11 = A[pi + Kp * pj], a12 = A[pi + Kp * qj], a21 = A[qi + Kp * pj], a22 = A[qi + Kp * qj];
        // left: rows p = c row_p - s row_q, q = s row_p + c row_q
        double b11 = ci * a11 - si * a21, b12 = ci * a12 - si * a22;
        double b21 = si * a11 + ci * a21, b22 = si * a12 + ci * a22;
        // right: cols p = c col_p - s col_q, q = s col_p + c col_q
        A[pi + Kp * pj] = cj * b11 - sj * b12;
        A[pi + Kp * qj] = sj * b11 + cj * b12;
        A[qi + Kp * pj] = cj * b21 - sj * b22;
        A[qi + Kp * qj] = sj * b21 + cj * b22;
      }
      // V <- V G (columns p, q of every row)
      for (int e = tid; e < np * Kp; e += EIG_NT) {
        int pr = e / Kp, i = e - pr * Kp;
        double c = cs[2 * pr], s = cs[2 * pr + 1];
        if (s == 0.0) continue;
        int p = pp[2 * pr], q = pp[2 * pr + 1];
        double vp = V[i + Kp * p], vq = V[i + Kp * q];
        V[i + Kp * p] = c * vp - s * vq;
        V[i + Kp * q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  double* diag = cs;
  for (int i = tid; i < K; i += EIG_NT) diag[i] = A[i + Kp * i];
  __syncthreads();
  int* rk = pp;
  for (int i = tid; i < K; i += EIG_NT) {
    double di = diag[i];
    int r = 0;
    for (int j = 0; j < K; ++j) {
      double dj = diag[j];
      if (dj > di || (dj == di && j < i)) ++r;
    }
    rk[i] = r;
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += EIG_NT) {
    int i = e % K, j = e / K;
    J.v[i + (long)K * rk[j]] = V[i + Kp * j];
  }
  for (int i = tid; i < K; i += EIG_NT) J.w[rk[i]] = diag[i];
}

// Rank-revealing pivoted Cholesky of a Gram matrix G (K x K), one workgroup per job:
// G[p,p] = R^T R with pivots chosen by the largest remaining diagonal; it stops when the largest
// remaining diagonal is <= tol * max diag(G).  Output W (K x q, ld K) = P[:, :q] R^-1, so that
// V W has orthonormal columns spanning V's numerically independent columns; q written to *qout.
// G is copied into S (LDS when K <= 128, else the job's global scratch).
template <bool SMEM>
__global__ __launch_bounds__(EIG_NT) void k_pchol(const CholJob* jobs) {
  extern __shared__ double sm[];
  const CholJob J = jobs[blockIdx.x];
  const int K = J.K;
  const int tid = threadIdx.x;
  if (K <= 0) { if (tid == 0 && J.q) *J.q = 0; return; }
  double* S = SMEM ? sm : J.work;                 // K x K Schur complement / R (row k holds R[k][:])
  double* red = SMEM ? sm + K * K : sm;           // EIG_NT values + EIG_NT indices
  int* redi = reinterpret_cast<int*>(red + EIG_NT);
  int* perm = redi + EIG_NT;                      // K
  __shared__ double dmax0, piv, dk;
  __shared__ int pidx, qfinal;
  for (int e = tid; e < K * K; e += EIG_NT) S[e] = J.g[e];
  for (int i = tid; i < K; i += EIG_NT) perm[i] = i;
  __syncthreads();
  // largest initial diagonal
  {
    double m = 0.0;
    for (int i = tid; i < K; i += EIG_NT) m = fmax(m, S[i + K * i]);
    red[tid] = m;
    __syncthreads();
    for (int w = EIG_NT / 2; w > 0; w >>= 1) { if (tid < w) red[tid] = fmax(red[tid], red[tid + w]); __syncthreads(); }
    if (tid == 0) { dmax0 = red[0]; qfinal = K; }
    __syncthreads();
  }
  for (int k = 0; k < K; ++k) {
    // pivot: largest remaining diagonal (ties: lowest index)
    double m = -1.0;
    int mi = k;
    for (int i = k + tid; i < K; i += EIG_NT) {
      double v = S[i + K * i];
      if (v > m) { m = v; mi = i; }
    }
    red[tid] = m;
    redi[tid] = mi;
    __syncthreads();
    for (int w = EIG_NT / 2; w > 0; w >>= 1) {
      if (tid < w) {
        double a = red[tid], b = red[tid + w];
        int ia = redi[tid], ib = redi[tid + w];
        if (b > a || (b == a && ib < ia)) { red[tid] = b; redi[tid] = ib; }
      }
      __syncthreads();
    }
    if (tid == 0) { piv = red[0]; pidx = redi[0]; }
    __syncthreads();
    if (!(piv > J.tol * dmax0) || dmax0 <= 0.0) {
      if (tid == 0) qfinal = k;
      __syncthreads();
      break;
    }
    const int p = pidx;
    if (p != k) {
      // symmetric swap of rows/columns k and p (full storage)
      for (int i = tid; i < K; i += EIG_NT) {
        double t = S[k + K * i]; S[k + K * i] = S[p + K * i]; S[p + K * i] = t;
      }
      __syncthreads();
      for (int i = tid; i < K; i += EIG_NT) {
        double t = S[i + K * k]; S[i + K * k] = S[i + K * p]; S[i + K * p] = t;
      }
      if (tid == 0) { int t = perm[k]; perm[k] = perm[p]; perm[p] = t; }
      __syncthreads();
    }
    // d is read once and published before row k is overwritten (the thread that handles
    // column k writes d into S[k][k])
    if (tid == 0) dk = sqrt(S[k + K * k]);
    __syncthreads();
    const double d = dk;
    // row k of R: R[k][j] = S[k][j] / d for j >= k (stored in S's row k)
    for (int j = k + tid; j < K; j += EIG_NT) S[k + K * j] = (j == k) ? d : S[k + K * j] / d;
    __syncthreads();
    // trailing update S[i][j] -= R[k][i] R[k][j], i, j > k
    const int rem = K - k - 1;
    for (int e = tid; e < rem * rem; e += EIG_NT) {
      int i = k + 1 + e % rem, j = k + 1 + e / rem;
      S[i + K * j] -= S[k + K * i] * S[k + K * j];
    }
    __syncthreads();
  }
  const int q = qfinal;
  // X = R^-1 (upper triangular), row by row from the bottom:
  // X[i][j] = (delta_ij - sum_{i<l<=j} R[i][l] X[l][j]) / R[i][i].
  // X[i][j], j > i, is kept at S[j][i] (the free lower triangle), its diagonal in xd.
  double* xd = reinterpret_cast<double*>(perm + K + (K & 1));
  for (int i = q - 1; i >= 0; --i) {
    const double rii = S[i + K * i];
    for (int j = i + tid; j < q; j += EIG_NT) {
      double acc = (j == i) ? 1.0 : 0.0;
      for (int l = i + 1; l <= j; ++l) {
        double xlj = (l == j) ? xd[l] : S[j + K * l];
        acc -= S[i + K * l] * xlj;
      }
      if (j == i) xd[i] = acc / rii;
      else S[j + K * i] = acc / rii;
    }
    __syncthreads();
  }
  // W = P[:, :q] X: row perm[i] of W is row i of X
  for (int e = tid; e < K * q; e += EIG_NT) {
    int r = e % K, j = e / K;
    J.w[r + (long)K * j] = 0.0;
  }
  __syncthreads();
  for (int e = tid; e < q * q; e += EIG_NT) {
    int i = e % q, j = e / q;
    if (j >= i) J.w[perm[i] + (long)K * j] = (j == i) ? xd[i] : S[j + K * i];
  }
  if (tid == 0 && J.q) *J.q = q;
}

hipError_t pchol_batched(const CholJob* jobs_dev, int count, int Kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (Kmax > EIG_MAX) return hipErrorInvalidValue;
  if (Kmax <= EIG_LDS_MAX) {
    size_t shm = (size_t)Kmax * Kmax * 8 + EIG_NT * 12 + (size_t)Kmax * 12 + 64;
    hipError_t e = hipFuncSetAttribute((const void*)k_pchol<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pchol<true>, dim3(count), dim3(EIG_NT), shm, s, jobs_dev);
  } else {
    size_t shm = EIG_NT * 12 + (size_t)Kmax * 12 + 64;
    hipLaunchKernelGGL(k_pchol<false>, dim3(count), dim3(EIG_NT), shm, s, jobs_dev);
  }
  return hipGetLastError();
}

hipError_t syev_batched(const EigJob* jobs_dev, int count, int Kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (Kmax > EIG_MAX) return hipErrorInvalidValue;
  int Kp = (Kmax + 1) & ~1;
  if (Kmax <= EIG_SMALL) {
    size_t shm = (size_t)Kp * Kp * 16 + (size_t)Kp * 8 + (size_t)Kp * 4 + 2 * EIG_NT * 8 + 64;
    hipError_t e = hipFuncSetAttribute((const void*)k_syev_small, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_syev_small, dim3(count), dim3(EIG_NT), shm, s, jobs_dev);
  } else if (Kmax <= EIG_LDS_MAX) {
    size_t shm = (size_t)Kp * Kp * 8 + (size_t)Kp * 8 + (size_t)Kp * 4 * 2 + 256 * 8 + 64;
    if (shm > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)k_syev<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_syev<true>, dim3(count), dim3(256), shm, s, jobs_dev);
  } else {
    size_t shm = (size_t)Kp * 8 + (size_t)Kp * 4 * 2 + 256 * 8 + 64;
    hipLaunchKernelGGL(k_syev<false>, dim3(count), dim3(256), shm, s, jobs_dev);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Elementwise helpers
// ---------------------------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void k_convert(const TI* in, TO* out, long count) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (TO)in[i];
}
template <typename TI, typename TO>
hipError_t convert(const TI* in, TO* out, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3((count + 255) / 256), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}
template hipError_t convert<double, float>(const double*, float*, long, hipStream_t);
template hipError_t convert<float, double>(const float*, double*, long, hipStream_t);
template hipError_t convert<double, double>(const double*, double*, long, hipStream_t);
template hipError_t convert<float, float>(const float*, float*, long, hipStream_t);

template <typename TI, typename TO>
__global__ void k_copy2d(int rows, int cols, const TI* in, int ldin, TO* out, int ldout, double scale) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)rows * cols) {
    int i = (int)(e % rows), j = (int)(e / rows);
    out[i + (long)ldout * j] = (TO)((double)in[i + (long)ldin * j] * scale);
  }
}
template <typename TI, typename TO>
hipError_t copy2d(int rows, int cols, const TI* in, int ldin, TO* out, int ldout, double scale, hipStream_t s) {
  long cnt = (long)rows * cols;
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy2d<TI, TO>), dim3((cnt + 255) / 256), dim3(256), 0, s, rows, cols, in, ldin, out, ldout, scale);
  return hipGetLastError();
}
template hipError_t copy2d<double, double>(int, int, const double*, int, double*, int, double, hipStream_t);
template hipError_t copy2d<float, float>(int, int, const float*, int, float*, int, double, hipStream_t);
template hipError_t copy2d<double, float>(int, int, const double*, int, float*, int, double, hipStream_t);
template hipError_t copy2d<float, double>(int, int, const float*, int, double*, int, double, hipStream_t);

template <typename T>
__global__ void k_permute3(const T* in, int d0, int d1, int d2, T* out, int p0, int p1, int p2) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long tot = (long)d0 * d1 * d2;
  if (e >= tot) return;
  int i = (int)(e % d0);
  int j = (int)((e / d0) % d1);
  int l = (int)(e / ((long)d0 * d1));
  int idx[3] = {i, j, l};
  int dims[3] = {d0, d1, d2};
  int o0 = idx[p0], o1 = idx[p1], o2 = idx[p2];
  int e0 = dims[p0], e1 = dims[p1];
  out[o0 + (long)e0 * (o1 + (long)e1 * o2)] = in[e];
}
template <typename T>
hipError_t permute3(const T* in, int d0, int d1, int d2, T* out, int p0, int p1, int p2, hipStream_t s) {
  long tot = (long)d0 * d1 * d2;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute3<T>, dim3((tot + 255) / 256), dim3(256), 0, s, in, d0, d1, d2, out, p0, p1, p2);
  return hipGetLastError();
}
template hipError_t permute3<double>(const double*, int, int, int, double*, int, int, int, hipStream_t);
template hipError_t permute3<float>(const float*, int, int, int, float*, int, int, int, hipStream_t);

__global__ void k_scale_cols(double* a, int rows, int cols, int ld, const double* scale) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)rows * cols) {
    int i = (int)(e % rows), j = (int)(e / rows);
    a[i + (long)ld * j] *= scale[j];
  }
}
hipError_t scale_cols_d(double* a, int rows, int cols, int ld, const double* scale, hipStream_t s) {
  long cnt = (long)rows * cols;
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols, dim3((cnt + 255) / 256), dim3(256), 0, s, a, rows, cols, ld, scale);
  return hipGetLastError();
}

__global__ void k_eig_inv_sqrt(const double* E, const double* w, int K, int q, double* W) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)K * q) {
    int i = (int)(e % K), j = (int)(e / K);
    W[i + (long)K * j] = E[i + (long)K * j] / sqrt(w[j]);
  }
}
hipError_t eig_inv_sqrt(const double* E, const double* w, int K, int q, double* W, hipStream_t s) {
  long cnt = (long)K * q;
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eig_inv_sqrt, dim3((cnt + 255) / 256), dim3(256), 0, s, E, w, K, q, W);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* a, const T* b, long count, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long i = threadIdx.x; i < count; i += 256) acc += (double)a[i] * (double)b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}
template <typename T>
hipError_t dot(const T* a, const T* b, long count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<T>, dim3(1), dim3(256), 0, s, a, b, count, out);
  return hipGetLastError();
}
template hipError_t dot<double>(const double*, const double*, long, double*, hipStream_t);
template hipError_t dot<float>(const float*, const float*, long, double*, hipStream_t);

__global__ void k_khatri_rao(const double* X2, int q2, const double* X3, int q3, int R, double* out) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long tot = (long)q2 * q3 * R;
  if (e < tot) {
    int b = (int)(e % q2);
    int c = (int)((e / q2) % q3);
    int k = (int)(e / ((long)q2 * q3));
    out[e] = X2[b + (long)q2 * k] * X3[c + (long)q3 * k];
  }
}
hipError_t khatri_rao_d(const double* X2, int q2, const double* X3, int q3, int R, double* out, hipStream_t s) {
  long tot = (long)q2 * q3 * R;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_khatri_rao, dim3((tot + 255) / 256), dim3(256), 0, s, X2, q2, X3, q3, R, out);
  return hipGetLastError();
}

template <typename T>
__global__ void k_contract_mid(const T* T1, const T* A, int rm, int ro, int ncol, T* t) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rm * ncol) return;
  int i = (int)(e % rm);
  long col = e / rm;
  const T* base = T1 + i + (long)rm * ro * col;
  const T* a = A + (long)ro * col;
  double acc = 0.0;
  for (int j = 0; j < ro; ++j) acc += (double)base[(long)rm * j] * (double)a[j];
  t[e] = (T)acc;
}
template <typename T>
hipError_t contract_mid(const T* T1, const T* A, int rm, int ro, int ncol, T* t, hipStream_t s) {
  long tot = (long)rm * ncol;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_contract_mid<T>, dim3((tot + 255) / 256), dim3(256), 0, s, T1, A, rm, ro, ncol, t);
  return hipGetLastError();
}
template hipError_t contract_mid<double>(const double*, const double*, int, int, int, double*, hipStream_t);
template hipError_t contract_mid<float>(const float*, const float*, int, int, int, float*, hipStream_t);

template <typename T>
__global__ void k_gather_rows(const T* in, int ld, const int* rows, int m, int cols, double* out) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)m * cols) {
    int p = (int)(e % m), c = (int)(e / m);
    out[e] = (double)in[rows[p] + (long)ld * c];
  }
}
template <typename T>
hipError_t gather_rows(const T* in, int ld, const int* rows, int m, int cols, double* out, hipStream_t s) {
  long tot = (long)m * cols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows<T>, dim3((tot + 255) / 256), dim3(256), 0, s, in, ld, rows, m, cols, out);
  return hipGetLastError();
}
template hipError_t gather_rows<double>(const double*, int, const int*, int, int, double*, hipStream_t);
template hipError_t gather_rows<float>(const float*, int, const int*, int, int, double*, hipStream_t);

// ---------------------------------------------------------------------------------------------
// Symbol construction
// ---------------------------------------------------------------------------------------------
__global__ void k_lambda(int n, double* out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    double h = 1.0 / (double)(n + 1);
    double s = sinpi(0.5 * (double)(k + 1) * h);
    out[k] = 4.0 / (h * h) * s * s;
  }
}
hipError_t lambda_1d(int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_lambda, dim3((n + 255) / 256), dim3(256), 0, s, n, out);
  return hipGetLastError();
}

template <typename T>
__global__ void k_expfactors(const double* lam, int n, const double* tau, int K, T* E, int ldE, int withLam) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)n * K) {
    int i = (int)(e % n), k = (int)(e / n);
    double v = exp(-tau[k] * lam[i]);
    E[i + (long)ldE * k] = (T)(withLam ? lam[i] * v : v);
  }
}
template <typename T>
hipError_t expfactors(const double* lam, int n, const double* tau, int K, T* E, int ldE, int withLam, hipStream_t s) {
  long tot = (long)n * K;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expfactors<T>, dim3((tot + 255) / 256), dim3(256), 0, s, lam, n, tau, K, E, ldE, withLam);
  return hipGetLastError();
}
template hipError_t expfactors<double>(const double*, int, const double*, int, double*, int, int, hipStream_t);
template hipError_t expfactors<float>(const double*, int, const double*, int, float*, int, int, hipStream_t);

// target function of the fits, in the scaled variable y = rho/rho0:
//   kind 0: g(y) = c_neg rho^-(1+alpha) + c_pos rho^-(1-alpha), rho = rho0*y
//   kind 1: p(y) = 1/s(rho) = 1/(c_neg rho^-alpha + c_pos rho^alpha)
//   kind 2: c_neg rho^-alpha (the state operator beta A^-alpha)
__device__ double fit_target(int kind, double alpha, double cn, double cp, double rho0, double y) {
  double rho = rho0 * y;
  double ra = pow(rho, alpha);
  if (kind == 0) return (cn / ra + cp * ra) / rho;
  if (kind == 2) return cn / ra;
  return 1.0 / (cn / ra + cp * ra);
}

__global__ void k_fit_design(int kind, double alpha, double cn, double cp, double rho0, double B, int K, int m,
                             const FitCand* cands, double* A, double* tvec) {
  int c = blockIdx.y;
  FitCand fc = cands[c];
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double lo = log(1.0 / B) + fc.a, hi = fc.b;
  if (e < K) {
    double t = exp(lo + (hi - lo) * (double)e / (double)(K > 1 ? K - 1 : 1));
    tvec[(long)c * K + e] = t;
  }
  if (e < (long)m * K) {
    int j = (int)(e % m), k = (int)(e / m);
    double t = exp(lo + (hi - lo) * (double)k / (double)(K > 1 ? K - 1 : 1));
    double y = exp(log(B) * (double)j / (double)(m > 1 ? m - 1 : 1));
    A[(long)c * m * K + e] = exp(-t * y) / fit_target(kind, alpha, cn, cp, rho0, y);
  }
}
hipError_t fit_design(int kind, double alpha, double cneg, double cpos, double rho0, double B, int K, int m,
                      const FitCand* cands_dev, int ncand, double* A, double* tvec, hipStream_t s) {
  long tot = (long)m * K;
  hipLaunchKernelGGL(k_fit_design, dim3((tot + 255) / 256, ncand), dim3(256), 0, s, kind, alpha, cneg, cpos, rho0,
                     B, K, m, cands_dev, A, tvec);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fit_error(int kind, double alpha, double cn, double cp, double rho0,
                                                   double B, int K, const double* t, const double* w, int m,
                                                   double* err) {
  __shared__ double red[256];
  int c = blockIdx.x;
  const double* tc = t + (long)c * K;
  const double* wc = w + (long)c * K;
  double mx = 0.0;
  for (int j = threadIdx.x; j < m; j += 256) {
    double y = exp(log(B) * (double)j / (double)(m - 1));
    double v = 0.0;
    for (int k = 0; k < K; ++k) v += wc[k] * exp(-tc[k] * y);
    double r = fabs(v / fit_target(kind, alpha, cn, cp, rho0, y) - 1.0);
    if (!(r <= mx)) mx = r;  // NaN propagates as "bad"
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double a = red[threadIdx.x], b = red[threadIdx.x + s];
      red[threadIdx.x] = (a >= b || isnan(a)) ? a : b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) err[c] = red[0];
}
hipError_t fit_error(int kind, double alpha, double cneg, double cpos, double rho0, double B, int K,
                     const double* t, const double* w, int ncand, int m, double* err, hipStream_t s) {
  hipLaunchKernelGGL(k_fit_error, dim3(ncand), dim3(256), 0, s, kind, alpha, cneg, cpos, rho0, B, K, t, w, m, err);
  return hipGetLastError();
}

// sinc nodes of g: u_k = k hh, t = log(1+e^u), phi' = 1/(1+e^-u);
// w_k = hh phi'(u) [c_neg rho0^-(1+a) t^a / Gamma(1+a) + c_pos rho0^-(1-a) t^-a / Gamma(1-a)], tau = t/rho0.
// alpha = 1 appends tau = 0 with weight c_pos.
__global__ void k_sinc_g(double alpha, double cn, double cp, double rho0, int kl, int kr, double hh, double* tau,
                         double* w) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = kl + kr + 1;
  bool one = fabs(1.0 - alpha) < 1e-15;
  if (idx < cnt) {
    double u = (double)(idx - kl) * hh;
    double e = exp(-fabs(u));
    double t = (u >= 0 ? u : 0.0) + log1p(e);
    double dph = u >= 0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
    double v = cn * pow(rho0, -(1.0 + alpha)) * pow(t, alpha) / tgamma(1.0 + alpha);
    if (!one) v += cp * pow(rho0, -(1.0 - alpha)) * pow(t, -alpha) / tgamma(1.0 - alpha);
    w[idx] = hh * dph * v;
    tau[idx] = t / rho0;
  } else if (idx == cnt && one) {
    w[idx] = cp;
    tau[idx] = 0.0;
  }
}
hipError_t sinc_g_nodes(double alpha, double cneg, double cpos, double rho0, int kl, int kr, double hh, double* tau,
                        double* w, hipStream_t s) {
  int cnt = kl + kr + 2;
  hipLaunchKernelGGL(k_sinc_g, dim3((cnt + 255) / 256), dim3(256), 0, s, alpha, cneg, cpos, rho0, kl, kr, hh, tau, w);
  return hipGetLastError();
}

// symbol value at index tuples: opkind 0 -> rho * sum w exp(-tau rho); 1 -> sum w exp(-tau rho)
__global__ void k_symbol_eval(int d, const int* idx, int count, const double* l0, const double* l1, const double* l2,
                              int opkind, int K, const double* tau, const double* w, double* out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  double rho = l0[idx[p * d + 0]] + l1[idx[p * d + 1]];
  if (d == 3) rho += l2[idx[p * d + 2]];
  double v = 0.0;
  for (int k = 0; k < K; ++k) v += w[k] * exp(-tau[k] * rho);
  out[p] = opkind == 0 ? rho * v : v;
}
hipError_t symbol_eval(int d, const int* idx, int count, const double* lam0, const double* lam1, const double* lam2,
                       int opkind, int K, const double* tau, const double* w, double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_symbol_eval, dim3((count + 255) / 256), dim3(256), 0, s, d, idx, count, lam0, lam1, lam2,
                     opkind, K, tau, w, out);
  return hipGetLastError();
}

// Column scaling of the least-squares normal equations: D_k = 1/sqrt(G_kk), G <- D G D, b <- D b.
__global__ void k_fit_scale(int K, double* G, double* b, double* D) {
  int c = blockIdx.x;
  double* Gc = G + (long)c * K * K;
  double* bc = b + (long)c * K;
  double* Dc = D + (long)c * K;
  __shared__ double dsh[64];
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double g = Gc[k + (long)K * k];
    dsh[k] = 1.0 / sqrt(g > 1e-300 ? g : 1e-300);
    Dc[k] = dsh[k];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    int i = e % K, j = e / K;
    Gc[e] *= dsh[i] * dsh[j];
  }
  for (int k = threadIdx.x; k < K; k += blockDim.x) bc[k] *= dsh[k];
}
hipError_t fit_scale(int K, int nc, double* G, double* b, double* D, hipStream_t s) {
  if (K > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fit_scale, dim3(nc), dim3(256), 0, s, K, G, b, D);
  return hipGetLastError();
}

// Pseudo-inverse solve in the eigenbasis: z = sum_{ev_j > cut ev_0} E_j (E_j . b)/ev_j, w = D z.
__global__ void k_fit_solve(int K, const double* ev, const double* E, const double* b, const double* D, double cut,
                            double* w) {
  int c = blockIdx.x;
  const double* evc = ev + (long)c * K;
  const double* Ec = E + (long)c * K * K;
  const double* bc = b + (long)c * K;
  __shared__ double proj[64];
  for (int j = threadIdx.x; j < K; j += blockDim.x) {
    double p = 0.0;
    if (evc[j] > cut * evc[0]) {
      for (int i = 0; i < K; ++i) p += Ec[i + (long)K * j] * bc[i];
      p /= evc[j];
    }
    proj[j] = p;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < K; i += blockDim.x) {
    double z = 0.0;
    for (int j = 0; j < K; ++j) z += Ec[i + (long)K * j] * proj[j];
    w[(long)c * K + i] = D[(long)c * K + i] * z;
  }
}
hipError_t fit_solve(int K, int nc, const double* ev, const double* E, const double* b, const double* D, double cut,
                     double* w, hipStream_t s) {
  if (K > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fit_solve, dim3(nc), dim3(64), 0, s, K, ev, E, b, D, cut, w);
  return hipGetLastError();
}

__global__ void k_scale(double* a, long n, double sc) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] *= sc;
}
hipError_t scale(double* a, long n, double sc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3((n + 255) / 256), dim3(256), 0, s, a, n, sc);
  return hipGetLastError();
}

}  // namespace tpk
