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

#include <algorithm>
#include <type_traits>

namespace tpk {

// ---------------------------------------------------------------------------------------------
// GEMM
// ---------------------------------------------------------------------------------------------
constexpr int GBM = 64, GBN = 64, GBK = 16, GTHREADS = 256;

// c = b * r1 + a for 0 <= c < 2^24: the float quotient is off by at most one, then corrected
// (an integer division per loaded element would dominate the tile load).
__device__ __forceinline__ void fast_divmod(int c, int r1, float inv, int& b, int& a) {
  b = (int)((float)c * inv);
  a = c - b * r1;
  if (a < 0) { --b; a += r1; } else if (a >= r1) { ++b; a -= r1; }
}

template <typename T>
__device__ __forceinline__ T fs_load(const FaceSplit<T>& F, int row, int c, float inv) {
  int a, b;
  fast_divmod(c, F.r1, inv, b, a);
  return F.x1[row + (long)F.ld1 * a] * F.x2[row + (long)F.ld2 * b];
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
  const float invA = g.fsA ? 1.0f / (float)FA.r1 : 0.0f, invB = g.fsB ? 1.0f / (float)FB.r1 : 0.0f;
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
        if (row < g.M && col < kend) v = g.fsA ? (Tacc)fs_load(FA, row, col, invA) : (Tacc)A[row + (long)g.lda * col];
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
        if (row < kend && col < g.N) v = g.fsB ? (Tacc)fs_load(FB, row, col, invB) : (Tacc)B[row + (long)g.ldb * col];
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
typedef double d2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Split-BF16 products of FP32 operands: x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi), both
// rounded to nearest even (8 significant bits each), so |x - hi| <= 2^-8 |x| and |r| <= 2^-16 |x|; a
// product is taken as hi*hi' + hi*lo' + lo*hi' (lo*lo' and the r terms dropped: relative error at
// most about 3 * 2^-16 per product), each term exact in the
// FP32 accumulation of the BF16 matrix cores.  The 16x16x16 BF16 instruction takes from lane l
// the 4 consecutive contraction slots 4 (l/16) .. 4 (l/16) + 3 of row (A) or column (B) l % 16 and
// leaves its 16x16 FP32 result in the layout of the FP32 16x16x4 instruction.
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef __bf16 b4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void bf16_split4(const float (&x)[4], s4_t& hi, s4_t& lo) {
  // FP32 -> BF16 conversions round to nearest even (two values per conversion instruction)
  const f4_t v = {x[0], x[1], x[2], x[3]};
  const b4_t h = __builtin_convertvector(v, b4_t);
  const b4_t l = __builtin_convertvector(v - __builtin_convertvector(h, f4_t), b4_t);
  hi = __builtin_bit_cast(s4_t, h);
  lo = __builtin_bit_cast(s4_t, l);
}
__device__ __forceinline__ f4_t mfma16_bf16(s4_t a, s4_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// One stage of the MFMA kernel covers MBK contraction indices; each thread loads MNE elements of
// the A tile and MNE of the B tile per stage.
constexpr int MBK = 16;
constexpr int MNE = MBK / 4;  // elements of each operand per thread per stage

// How an operand's tile elements are read: column-major, transposed, or face-split.
enum { OP_N = 0, OP_T = 1, OP_FS = 2 };

// The raw loads of one operand's share of a stage.  They are issued without a bounds branch
// (indices clamped into the matrix) and combined - bounds mask, face-split product, conversion
// to the accumulation type - only when the stage is written to LDS: a load under a
// divergent branch, or an arithmetic use of a loaded value, makes the compiler wait for it on the
// spot, while these stay in flight through the previous stage's MFMAs.
template <typename T, int KIND>
struct OpRegs {
  T x[MNE];
  T y[KIND == OP_FS ? MNE : 1];
  unsigned ok;
};

// Element i of the thread's share: A tiles are M x K, B tiles K x N.  For a column-major A tile
// (or a face-split one) lane groups run along M; for a transposed one along K; B the other way.
// Along M (or N) a thread takes the MNE consecutive contraction indices of its wave's quarter of the
// stage for one row, which it stores to LDS as one contiguous run.
template <bool IS_A, int KIND>
__device__ __forceinline__ void tile_pos(int tid, int i, int& outer, int& kk) {
  const bool alongK = IS_A ? (KIND == OP_T) : (KIND != OP_T);
  if (alongK) { kk = tid % MBK; outer = tid / MBK + (GTHREADS / MBK) * i; }
  else { outer = tid & 63; kk = MNE * (tid >> 6) + i; }
}

// LDS tile layout: row o of the tile (a row of A, a column of B) holds the stage's MBK contraction
// indices contiguously, rows padded to a multiple of 16 bytes that spreads the 16 rows a quarter
// wave reads over all banks.
template <typename Tacc>
struct LdsTile {
  static constexpr int RS = MBK + (sizeof(Tacc) == 4 ? 4 : 2);  // row stride in elements
};

// Loads op's stage at (o0 along M or N, k0 along K); nout is M or N, the contraction runs to kend.
// P: the operand's matrix (OP_N, OP_T), F: its face-split description (OP_FS).
template <bool IS_A, int KIND, typename T>
__device__ __forceinline__ void op_fetch(const T* P, int ld, const FaceSplit<T>& F, float inv, int o0, int nout,
                                         int k0, int kend, int tid, OpRegs<T, KIND>& r) {
  r.ok = 0;
#pragma unroll
  for (int i = 0; i < MNE; ++i) {
    int o, kk;
    tile_pos<IS_A, KIND>(tid, i, o, kk);
    const int oi = o0 + o, ki = k0 + kk;
    r.ok |= (unsigned)(oi < nout && ki < kend) << i;
    const int oc = min(oi, nout - 1), kc = min(ki, kend - 1);
    // row and column of the stored matrix
    const int row = IS_A ? (KIND == OP_T ? kc : oc) : (KIND == OP_T ? oc : kc);
    const int col = IS_A ? (KIND == OP_T ? oc : kc) : (KIND == OP_T ? kc : oc);
    if (KIND == OP_FS) {
      int a, b;
      fast_divmod(col, F.r1, inv, b, a);
      r.x[i] = F.x1[row + (long)F.ld1 * a];
      r.y[i] = F.x2[row + (long)F.ld2 * b];
    } else {
      r.x[i] = P[row + (long)ld * col];
    }
  }
}

template <typename Tacc, typename T, int KIND>
__device__ __forceinline__ Tacc op_value(const OpRegs<T, KIND>& r, int i) {
  Tacc v;
  if (KIND == OP_FS) {
    v = (Tacc)(r.x[i] * r.y[i]);
  } else {
    v = (Tacc)r.x[i];
  }
  return ((r.ok >> i) & 1u) ? v : (Tacc)0;
}

// Writes the stage to LDS as T[m][k] (A) or T[n][k] (B): a run of MNE values per thread along M,
// single values along K.
template <bool IS_A, int KIND, typename Tacc, typename T>
__device__ __forceinline__ void op_store(Tacc (*S)[LdsTile<Tacc>::RS], int tid, const OpRegs<T, KIND>& r) {
  const bool alongK = IS_A ? (KIND == OP_T) : (KIND != OP_T);
  if (alongK) {
#pragma unroll
    for (int i = 0; i < MNE; ++i) {
      int o, kk;
      tile_pos<IS_A, KIND>(tid, i, o, kk);
      S[o][kk] = op_value<Tacc>(r, i);
    }
  } else {
    typedef typename std::conditional<sizeof(Tacc) == 4, f4_t, d2_t>::type V;
    constexpr int W = 16 / sizeof(Tacc);
    V* dst = reinterpret_cast<V*>(&S[tid & 63][MNE * (tid >> 6)]);
#pragma unroll
    for (int c = 0; c < MNE / W; ++c) {
      V v;
#pragma unroll
      for (int e = 0; e < W; ++e) v[e] = op_value<Tacc>(r, W * c + e);
      dst[c] = v;
    }
  }
}

// MNE consecutive LDS values from a 16-byte aligned address as 16-byte reads.
__device__ __forceinline__ void lds_run(const float* p, float (&v)[MNE]) {
#pragma unroll
  for (int c = 0; c < MNE / 4; ++c) {
    const f4_t x = reinterpret_cast<const f4_t*>(p)[c];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[4 * c + e] = x[e];
  }
}
__device__ __forceinline__ void lds_run(const double* p, double (&v)[MNE]) {
#pragma unroll
  for (int c = 0; c < MNE / 2; ++c) {
    const d2_t x = reinterpret_cast<const d2_t*>(p)[c];
    v[2 * c] = x[0];
    v[2 * c + 1] = x[1];
  }
}

// SPLIT (FP32 operands and accumulation only): the products of a stage are split-BF16 products on
// the BF16 matrix cores instead of FP32 ones (the loads, LDS tiles and epilogue are the same).
template <typename TA, typename TB, typename TC, typename Tacc, int AK, int BK, bool SPLIT = false>
__global__ __launch_bounds__(GTHREADS) void k_gemm_mfma(GemmGroup<TA, TB, TC, Tacc> grp) {
  static_assert(!SPLIT || (std::is_same<Tacc, float>::value && MNE == 4), "split-BF16 takes FP32 16-deep stages");
  typedef typename std::conditional<std::is_same<Tacc, double>::value, d4_t, f4_t>::type V4;
  constexpr int RS = LdsTile<Tacc>::RS;
  __shared__ __align__(16) Tacc As[GBM][RS];
  __shared__ __align__(16) Tacc Bs[GBN][RS];
  // the product this workgroup belongs to: blockIdx.z runs over the products' batch x split ranges
  int z = blockIdx.z, j = 0;
  while (j + 1 < grp.count && z >= grp.z0[j + 1]) ++j;
  const GemmArgs<TA, TB, TC, Tacc>& g = grp.g[j];
  z -= grp.z0[j];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  if (m0 >= g.M || n0 >= g.N) return;  // the grid spans the largest product of the group
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int b = z / g.splits;
  const int sp = z - b * g.splits;
  const int kbeg = sp * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const TA* A = AK != OP_FS ? g.A + (long)(b / g.divA) * g.sA : nullptr;
  const TB* B = BK != OP_FS ? g.B + (long)(b / g.divB) * g.sB : nullptr;
  FaceSplit<TA> FA = g.FA;
  FaceSplit<TB> FB = g.FB;
  if (AK == OP_FS) { FA.x1 += (long)(b / g.divA) * g.sA; FA.x2 += (long)(b / g.divA) * g.sA; }
  if (BK == OP_FS) { FB.x1 += (long)(b / g.divB) * g.sB; FB.x2 += (long)(b / g.divB) * g.sB; }
  const float invA = AK == OP_FS ? 1.0f / (float)FA.r1 : 0.0f, invB = BK == OP_FS ? 1.0f / (float)FB.r1 : 0.0f;
  TC* C = g.C + (long)b * g.sC;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;

  OpRegs<TA, AK> ra;
  OpRegs<TB, BK> rb;
  if (kbeg < kend) {
    op_fetch<true, AK>(A, g.lda, FA, invA, m0, g.M, kbeg, kend, tid, ra);
    op_fetch<false, BK>(B, g.ldb, FB, invB, n0, g.N, kbeg, kend, tid, rb);
  }
  for (int k0 = kbeg; k0 < kend; k0 += MBK) {
    op_store<true, AK>(As, tid, ra);
    op_store<false, BK>(Bs, tid, rb);
    __syncthreads();
    if (k0 + MBK < kend) {
      op_fetch<true, AK>(A, g.lda, FA, invA, m0, g.M, k0 + MBK, kend, tid, ra);
      op_fetch<false, BK>(B, g.ldb, FB, invB, n0, g.N, k0 + MBK, kend, tid, rb);
    }
    // the blocks are formed transposed, D = (A B)^T = B^T A^T (B's values in the first operand):
    // a lane's results then lie along a column of C, so each store instruction writes runs of
    // 16 consecutive rows (64 or 128 contiguous bytes) instead of 16 different columns.  Lane
    // group g = lane / 16 supplies the contraction indices MNE g .. MNE g + MNE - 1 of the stage
    // (the instruction's k slot g of step t is index MNE g + t for both operands, so the products
    // are the same), read as 16-byte runs
    {
      const int c16 = lane & 15, kq = MNE * (lane >> 4);
      Tacc a0[MNE], a1[MNE], b0[MNE], b1[MNE];
      lds_run(&As[wm + c16][kq], a0);
      lds_run(&As[wm + 16 + c16][kq], a1);
      lds_run(&Bs[wn + c16][kq], b0);
      lds_run(&Bs[wn + 16 + c16][kq], b1);
      if constexpr (SPLIT) {
        // the stage's 16 indices in one instruction per term: lane group g holds indices 4g .. 4g+3
        s4_t ah0, al0, ah1, al1, bh0, bl0, bh1, bl1;
        bf16_split4(a0, ah0, al0);
        bf16_split4(a1, ah1, al1);
        bf16_split4(b0, bh0, bl0);
        bf16_split4(b1, bh1, bl1);
        acc[0][0] = mfma16_bf16(bl0, ah0, acc[0][0]);
        acc[0][1] = mfma16_bf16(bl1, ah0, acc[0][1]);
        acc[1][0] = mfma16_bf16(bl0, ah1, acc[1][0]);
        acc[1][1] = mfma16_bf16(bl1, ah1, acc[1][1]);
        acc[0][0] = mfma16_bf16(bh0, al0, acc[0][0]);
        acc[0][1] = mfma16_bf16(bh1, al0, acc[0][1]);
        acc[1][0] = mfma16_bf16(bh0, al1, acc[1][0]);
        acc[1][1] = mfma16_bf16(bh1, al1, acc[1][1]);
        acc[0][0] = mfma16_bf16(bh0, ah0, acc[0][0]);
        acc[0][1] = mfma16_bf16(bh1, ah0, acc[0][1]);
        acc[1][0] = mfma16_bf16(bh0, ah1, acc[1][0]);
        acc[1][1] = mfma16_bf16(bh1, ah1, acc[1][1]);
      } else {
#pragma unroll
        for (int t = 0; t < MNE; ++t) {
          acc[0][0] = mfma16(b0[t], a0[t], acc[0][0]);
          acc[0][1] = mfma16(b1[t], a0[t], acc[0][1]);
          acc[1][0] = mfma16(b0[t], a1[t], acc[1][0]);
          acc[1][1] = mfma16(b1[t], a1[t], acc[1][1]);
        }
      }
    }
    __syncthreads();
  }
  // element v of lane l of block (i, j) is C[16 i + l % 16][16 j + cbase + cstep v] of the wave's
  // quarter (the 16x16 result layouts of the FP32 and FP64 instructions, transposed)
  const bool f64 = std::is_same<Tacc, double>::value;
  const int cbase = f64 ? (lane >> 4) : 4 * (lane >> 4), cstep = f64 ? 4 : 1, rl = lane & 15;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row = m0 + wm + 16 * i + rl;
        int col = n0 + wn + 16 * j + cbase + cstep * v;
        if (row >= g.M || col >= g.N) continue;
        Tacc x = acc[i][j][v];
        if (g.part) {
          g.part[(long)z * g.M * g.N + row + (long)g.M * col] = x;
        } else {
          // FP64 results of FP32 accumulation are scaled and summed in FP64
          typedef typename std::conditional<std::is_same<TC, double>::value, double, Tacc>::type Te;
          long o = row + (long)g.ldc * col;
          Te y = (Te)g.alpha * (Te)x;
          if (g.beta != (Tacc)0) y += (Te)g.beta * (Te)C[o];
          C[o] = (TC)y;
        }
      }
}

// Split-K reduction of a group: blockIdx.y runs over the products' batches (z0 of the group's
// reduction offsets), blockIdx.x over the largest product's M x N elements.
template <typename TA, typename TB, typename TC, typename Tacc>
__global__ void k_gemm_reduce(GemmGroup<TA, TB, TC, Tacc> grp) {
  int y = blockIdx.y, j = 0;
  while (j + 1 < grp.count && y >= grp.r0[j + 1]) ++j;
  const GemmArgs<TA, TB, TC, Tacc>& g = grp.g[j];
  const int b = y - grp.r0[j];
  const long mn = (long)g.M * g.N;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mn || g.splits < 2) return;
  const int splits = g.splits;
  int row = (int)(e % g.M), col = (int)(e / g.M);
  const Tacc* p = g.part + (long)b * splits * mn + e;
  // the partial sums are added in FP64 when the result is FP64 (FP32 chunks of an FP32-accumulated
  // product); four independent sums keep four loads in flight (fixed order: deterministic)
  typedef typename std::conditional<std::is_same<TC, double>::value, double, Tacc>::type Te;
  Te a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int s = 0;
  for (; s + 4 <= splits; s += 4) {
    a0 += (Te)p[(long)s * mn];
    a1 += (Te)p[(long)(s + 1) * mn];
    a2 += (Te)p[(long)(s + 2) * mn];
    a3 += (Te)p[(long)(s + 3) * mn];
  }
  for (; s < splits; ++s) a0 += (Te)p[(long)s * mn];
  Te acc = (a0 + a1) + (a2 + a3);
  long o = (long)b * g.sC + row + (long)g.ldc * col;
  Te v = (Te)g.alpha * acc;
  if (g.beta != (Tacc)0) v += (Te)g.beta * (Te)g.C[o];
  g.C[o] = (TC)v;
}

// 0: plain FMA kernel, 1: FP32 / FP64 matrix cores, 2: as 1 with split-BF16 products for the
// contractions with FP32 operands, accumulation and result
static int g_use_mfma = 1;
bool gemm_use_mfma() { return g_use_mfma != 0; }
void gemm_set_mfma(int mode) { g_use_mfma = mode; }

// The operand kinds are template parameters: each kernel holds only its own loads and registers.
template <typename TA, typename TB, typename TC, typename Tacc, int AK, bool SPLIT>
static void launch_mfma_b(const GemmGroup<TA, TB, TC, Tacc>& h, bool fsB, bool tB, dim3 grid, hipStream_t s) {
  if (fsB)
    hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TC, Tacc, AK, OP_FS, SPLIT>), grid, dim3(GTHREADS), 0, s, h);
  else if (tB)
    hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TC, Tacc, AK, OP_T, SPLIT>), grid, dim3(GTHREADS), 0, s, h);
  else
    hipLaunchKernelGGL((k_gemm_mfma<TA, TB, TC, Tacc, AK, OP_N, SPLIT>), grid, dim3(GTHREADS), 0, s, h);
}
template <typename TA, typename TB, typename TC, typename Tacc, int AK>
static void launch_mfma_a(const GemmGroup<TA, TB, TC, Tacc>& h, bool fsB, bool tB, dim3 grid, hipStream_t s) {
  constexpr bool f32 = std::is_same<TA, float>::value && std::is_same<TB, float>::value &&
                       std::is_same<TC, float>::value && std::is_same<Tacc, float>::value;
  if constexpr (f32) {
    if (g_use_mfma == 2) {
      launch_mfma_b<TA, TB, TC, Tacc, AK, true>(h, fsB, tB, grid, s);
      return;
    }
  }
  launch_mfma_b<TA, TB, TC, Tacc, AK, false>(h, fsB, tB, grid, s);
}

template <typename TA, typename TB, typename TC, typename Tacc>
hipError_t gemm_group(const GemmArgs<TA, TB, TC, Tacc>* gs, int count, hipStream_t s, hipEvent_t mid) {
  if (count < 1 || count > kGemmGroup) return hipErrorInvalidValue;
  GemmGroup<TA, TB, TC, Tacc> h;
  h.count = 0;
  int gx = 0, gy = 0, z = 0, r = 0;
  bool split = false;
  for (int i = 0; i < count; ++i) {
    GemmArgs<TA, TB, TC, Tacc> a = gs[i];
    if (a.M <= 0 || a.N <= 0 || a.batch <= 0) continue;
    // one operand kind per launch: the kernels are specialised on it
    if (h.count > 0 && (a.fsA != h.g[0].fsA || a.tA != h.g[0].tA || a.fsB != h.g[0].fsB || a.tB != h.g[0].tB))
      return hipErrorInvalidValue;
    if (a.splits < 1 || !a.part) { a.splits = 1; a.part = nullptr; }
    // split chunks are multiples of the stage depth
    a.kchunk = a.splits > 1 ? ((a.K + a.splits - 1) / a.splits + MBK - 1) / MBK * MBK : a.K;
    gx = std::max(gx, (a.M + GBM - 1) / GBM);
    gy = std::max(gy, (a.N + GBN - 1) / GBN);
    h.z0[h.count] = z;
    h.r0[h.count] = r;
    z += a.batch * a.splits;
    if (a.splits > 1) { r += a.batch; split = true; }
    h.g[h.count++] = a;
  }
  if (h.count == 0) return hipSuccess;
  h.z0[h.count] = z;
  h.r0[h.count] = r;
  const GemmArgs<TA, TB, TC, Tacc>& f = h.g[0];
  dim3 grid(gx, gy, z);
  if (gemm_use_mfma()) {
    if (f.fsA)
      launch_mfma_a<TA, TB, TC, Tacc, OP_FS>(h, f.fsB, f.tB, grid, s);
    else if (f.tA)
      launch_mfma_a<TA, TB, TC, Tacc, OP_T>(h, f.fsB, f.tB, grid, s);
    else
      launch_mfma_a<TA, TB, TC, Tacc, OP_N>(h, f.fsB, f.tB, grid, s);
  } else {
    for (int i = 0; i < h.count; ++i) {
      const GemmArgs<TA, TB, TC, Tacc>& a = h.g[i];
      dim3 g1((a.M + GBM - 1) / GBM, (a.N + GBN - 1) / GBN, a.batch * a.splits);
      hipLaunchKernelGGL((k_gemm<TA, TB, TC, Tacc>), g1, dim3(GTHREADS), 0, s, a);
    }
  }
  if (split) {
    if (mid) {
      const hipError_t e = hipEventRecord(mid, s);
      if (e != hipSuccess) return e;
    }
    long mn = 0;
    for (int i = 0; i < h.count; ++i)
      if (h.g[i].splits > 1) mn = std::max(mn, (long)h.g[i].M * h.g[i].N);
    dim3 rg((mn + 255) / 256, r);
    hipLaunchKernelGGL((k_gemm_reduce<TA, TB, TC, Tacc>), rg, dim3(256), 0, s, h);
  }
  return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename Tacc>
hipError_t gemm(const GemmArgs<TA, TB, TC, Tacc>& g, hipStream_t s, hipEvent_t mid) {
  return gemm_group<TA, TB, TC, Tacc>(&g, 1, s, mid);
}

template hipError_t gemm<double, double, double, double>(const GemmArgs<double, double, double, double>&, hipStream_t, hipEvent_t);
template hipError_t gemm<float, float, float, float>(const GemmArgs<float, float, float, float>&, hipStream_t, hipEvent_t);
template hipError_t gemm_group<double, double, double, double>(const GemmArgs<double, double, double, double>*, int, hipStream_t, hipEvent_t);
template hipError_t gemm_group<float, float, float, float>(const GemmArgs<float, float, float, float>*, int, hipStream_t, hipEvent_t);
template hipError_t gemm_group<float, float, double, double>(const GemmArgs<float, float, double, double>*, int, hipStream_t, hipEvent_t);
template hipError_t gemm_group<double, double, float, double>(const GemmArgs<double, double, float, double>*, int, hipStream_t, hipEvent_t);
template hipError_t gemm_group<float, float, double, float>(const GemmArgs<float, float, double, float>*, int, hipStream_t, hipEvent_t);
template hipError_t gemm<float, float, double, double>(const GemmArgs<float, float, double, double>&, hipStream_t, hipEvent_t);
template hipError_t gemm<double, double, float, double>(const GemmArgs<double, double, float, double>&, hipStream_t, hipEvent_t);
template hipError_t gemm<float, float, double, float>(const GemmArgs<float, float, double, float>&, hipStream_t, hipEvent_t);

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

// TI: storage type of the columns; T: arithmetic type of the transform (T = double for FP32
// columns where the FP64 work array fits in LDS, see dst1).
// GLOBAL: the work array lives in `work` (one slice of cpw * N/2 complex values per workgroup,
// L2 resident) instead of LDS; the barriers order those global accesses within the workgroup.
// Several column blocks of one length share a launch: the workgroups of job i start at
// blockIdx.x = blk0 (increasing with i).
template <typename TI>
struct DstJobs { DstJob<TI> j[kDstJobs]; int count; };

template <typename TI, typename T, bool GLOBAL>
__global__ __launch_bounds__(256) void k_dst1(int N, int logL, int cpw, DstJobs<TI> jobs,
                                              const T* __restrict__ tab, T scale, C2<T>* work) {
  extern __shared__ char smem_raw[];
  const int L = N >> 1;
  const int tot = cpw * L;
  C2<T>* X = GLOBAL ? work + (long)blockIdx.x * tot : reinterpret_cast<C2<T>*>(smem_raw);
  double* partial = GLOBAL ? reinterpret_cast<double*>(smem_raw)
                           : reinterpret_cast<double*>(reinterpret_cast<C2<T>*>(smem_raw) + tot);  // 256 chunk totals
  const int tid = threadIdx.x;
  int jb = 0;
  while (jb + 1 < jobs.count && (int)blockIdx.x >= jobs.j[jb + 1].blk0) ++jb;
  const int cols = jobs.j[jb].cols, ldin = jobs.j[jb].ldin, ldout = jobs.j[jb].ldout;
  const TI* in = jobs.j[jb].in;
  TI* out = jobs.j[jb].out;
  const int col0 = ((int)blockIdx.x - jobs.j[jb].blk0) * cpw;

  auto xval = [&](int c, int j) -> T {  // x_j, 1-based, zero outside 1..N-1
    int col = col0 + c;
    if (j <= 0 || j >= N || col >= cols) return (T)0;
    return (T)in[(j - 1) + (long)ldin * col];
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
  // segmented inclusive scan of X[].re per column (odd outputs).  The running sum is kept in
  // double and each output is rounded once: in FP32 a running sum rounded at every step
  // carries the rounding of its largest partial sums into every later output (a random walk of
  // eps * max|y| over up to N/2 steps, 4e-4 relative at N = 32768 for a single high mode).
  const int chunk = tot / 256;  // >= 1, divides L
  {
    int beg = tid * chunk;
    double run = 0.0;
    for (int i = 0; i < chunk; ++i) run += (double)X[beg + i].re;
    partial[tid] = run;
  }
  __syncthreads();
  {
    int beg = tid * chunk;
    int cstart = (beg / L) * L;  // first element of this column
    int t0 = cstart / chunk;
    double run = 0.0;
    for (int t = t0; t < tid; ++t) run += partial[t];
    for (int i = 0; i < chunk; ++i) { run += (double)X[beg + i].re; X[beg + i].re = (T)run; }
  }
  __syncthreads();
  for (int e = tid; e < tot; e += 256) {
    int c = e / L, k = e - c * L;
    int col = col0 + c;
    if (col >= cols) continue;
    out[2 * k + (long)ldout * col] = (TI)(scale * X[e].re);              // y_{2k+1}
    if (k >= 1) out[2 * k - 1 + (long)ldout * col] = (TI)(scale * X[e].im);  // y_{2k}
  }
}

template <typename TI, typename T>
hipError_t dst1_launch(int N, const DstJob<TI>* jl, int count, const T* tab, void* work, hipStream_t s) {
  int L = N / 2;
  int logL = 0;
  while ((1 << logL) < L) ++logL;
  int cpw = L >= 256 ? 1 : 256 / L;
  T scale = (T)sqrt(2.0 / (double)N);
  DstJobs<TI> jobs;
  jobs.count = 0;
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    if (jl[i].cols <= 0) continue;
    DstJob<TI> j = jl[i];
    j.blk0 = blocks;
    blocks += (j.cols + cpw - 1) / cpw;
    jobs.j[jobs.count++] = j;
  }
  if (blocks == 0) return hipSuccess;
  if (work) {
    hipLaunchKernelGGL((k_dst1<TI, T, true>), dim3(blocks), dim3(256), 256 * sizeof(double), s, N, logL, cpw, jobs,
                       tab, scale, reinterpret_cast<C2<T>*>(work));
    return hipGetLastError();
  }
  size_t shm = (size_t)cpw * L * sizeof(C2<T>) + 256 * sizeof(double);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dst1<TI, T, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_dst1<TI, T, false>), dim3(blocks), dim3(256), shm, s, N, logL, cpw, jobs, tab, scale,
                     (C2<T>*)nullptr);
  return hipGetLastError();
}

// FP32 columns are transformed in FP64 arithmetic.  The pre-processing adds the small
// sin(pi j/N)-weighted symmetric part of x to its antisymmetric part, so in FP32 arithmetic the
// transform of a vector whose spectrum sits at either end (the smooth factors of the iterates)
// loses about eps N / pi relative accuracy (measured: 5e-5 for the inverse of the first mode at
// N = 8192, 7e-5 at N = 32768); the FP64 work array removes it.  It fits in LDS up to N = 16384;
// at N = 32768 it lives in `work` (cols * N/2 complex doubles, global, one job per launch).
template <typename T>
static hipError_t dst1_jobs(int N, const DstJob<T>* jobs, int count, const T* tab, const double* tab64, void* work,
                            hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kDstJobs) return hipErrorInvalidValue;
  if (std::is_same<T, float>::value && tab64 && (N <= 16384 || work))
    return dst1_launch<T, double>(N, jobs, count, tab64, N <= 16384 ? nullptr : work, s);
  return dst1_launch<T, T>(N, jobs, count, tab, N <= 16384 ? nullptr : work, s);
}

template <typename T>
hipError_t dst1(int N, int cols, const T* in, int ldin, T* out, int ldout, const T* tab, const double* tab64,
                void* work, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  const DstJob<T> j{in, out, cols, ldin, ldout, 0};
  return dst1_jobs<T>(N, &j, 1, tab, tab64, work, s);
}

template <typename T>
hipError_t dst1_batched(int N, const DstJob<T>* jobs, int count, const T* tab, const double* tab64, hipStream_t s) {
  if (N > 16384) return hipErrorInvalidValue;
  return dst1_jobs<T>(N, jobs, count, tab, tab64, nullptr, s);
}

template hipError_t dst1<double>(int, int, const double*, int, double*, int, const double*, const double*, void*,
                                 hipStream_t);
template hipError_t dst1<float>(int, int, const float*, int, float*, int, const float*, const double*, void*,
                                hipStream_t);
template hipError_t dst1_batched<double>(int, const DstJob<double>*, int, const double*, const double*, hipStream_t);
template hipError_t dst1_batched<float>(int, const DstJob<float>*, int, const float*, const double*, hipStream_t);

// ---------------------------------------------------------------------------------------------
// Cyclic Jacobi eigensolver (FP64), round-robin parallel ordering, A in LDS, V in global.
// ---------------------------------------------------------------------------------------------
constexpr int EIG_LDS_MAX = kGramLds;  // matrices up to this size live in LDS
constexpr int EIG_MAX = 256;       // larger ones (up to this) live in global scratch

__device__ __forceinline__ int rr_index(int j, int s, int Kp) {
  // circle method: position 0 fixed, others rotate by s
  return j == 0 ? 0 : ((j - 1 + s) % (Kp - 1)) + 1;
}

// One workgroup per matrix.  A (Kp x Kp) in LDS when SMEM, else in J.work (global, L2 resident).
template <bool SMEM>
__global__ __launch_bounds__(256) void k_syev(JobBatch<EigJob> jobs) {
  extern __shared__ double sm[];
  const EigJob J = jobs.j[blockIdx.x];
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

__global__ __launch_bounds__(EIG_NT) void k_syev_small(JobBatch<EigJob> jobs) {
  extern __shared__ double sm[];
  const EigJob J = jobs.j[blockIdx.x];
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

// DPP row permutations on doubles and sums over aligned lane groups of 4, 8 and 16 (quad
// xor 1, quad xor 2, half-row mirror, row mirror); every lane of a group receives its sum.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ double group_sum(double v, int lanes) {
  if (lanes >= 2) v += dpp_f64<0xB1>(v);
  if (lanes >= 4) v += dpp_f64<0x4E>(v);
  if (lanes >= 8) v += dpp_f64<0x141>(v);
  if (lanes >= 16) v += dpp_f64<0x140>(v);
  return v;
}
// Lanes per group for the DPP sums: the largest power of two <= 16 with lanes * groups <= nt
// (at least 1).
__device__ __forceinline__ int lanes_for(int nt, int groups) {
  int l = 16;
  while (l > 1 && l * groups > nt) l >>= 1;
  return l;
}

// Sum / maximum over the 64 lanes (DPP within rows of 16, then the four row results read into
// scalars); every lane receives the result, and the order of the additions is fixed.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  v = group_sum(v, 16);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// ---------------------------------------------------------------------------------------------
// Pivoted Cholesky of Gram matrices, shared by the orthonormalisation (k_pchol) and the Gram
// eigensolver (k_psd_eig).  G[P,P] = R^T R, the pivot of each step being the largest remaining
// diagonal entry; it stops once that entry is <= ctol * max diag(G).  The workgroup is sized to
// the matrix (256 threads up to K = 64, 512 up to 128, 1024 beyond); the thread grid of the
// trailing updates: thread (tx, ty) owns the elements (tx + TX a, ty + TY b).
// ---------------------------------------------------------------------------------------------
struct CholShared { double rest; int q; };

template <int NT> struct ChGrid;
template <> struct ChGrid<64> { static constexpr int TX = 8, NBI = 8, NBJ = 8, KMAX = 64; };
template <> struct ChGrid<256> { static constexpr int TX = 16, NBI = 4, NBJ = 4, KMAX = 64; };
template <> struct ChGrid<512> { static constexpr int TX = 32, NBI = 4, NBJ = 8, KMAX = 128; };
template <> struct ChGrid<1024> { static constexpr int TX = 32, NBI = 8, NBJ = 8, KMAX = 256; };


// The factorisation blocked (the pivoted scheme of LAPACK's dpstrf): panels of NB pivots are
// factored left-looking by wave 0 alone, lane i owning rows i + 64 r (r < RPL), with no barrier:
// the Schur diagonal lives in those lanes' registers, the pivot is the lane maximum of 32-bit
// keys (the diagonal relative to the largest initial one, as float bits, the low IB bits replaced
// by 2^IB - 1 - index: ties to 2^-(23-IB) relative go to the lower index), and column k is
// (S[:, p] - L[:, panel] L[p, panel]^T) / sqrt(d_p) with L[p, panel] read from lane p's registers.
// After each panel the whole workgroup applies it to the trailing matrix S (one barrier on each
// side), which is full and symmetric (in LDS, or in global memory for K > 128).  Output:
// Lc[k K + i] = L(i, k) (column k of L in the original row order, so R(k, l) = Lc[k K + perm[l]] in
// pivot order), dk[k] = sqrt(pivot k), perm (the pivots, then the unpivoted indices in increasing
// order), sh.rest (the Schur trace left).  S is overwritten.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false));
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0), r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32), r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(r0, r1), max(r2, r3));
}

// Panel width, rows per lane of wave 0 (K <= 64 RPL) and bits of the pivot index in the keys
template <int NT> struct CholBlk;
template <> struct CholBlk<256> { static constexpr int RPL = 1, NB = 16, IB = 6; };
template <> struct CholBlk<512> { static constexpr int RPL = 2, NB = 16, IB = 8; };
template <> struct CholBlk<1024> { static constexpr int RPL = 4, NB = 8, IB = 8; };

template <int IB>
__device__ __forceinline__ unsigned pivot_key_ib(double v, double scale, int i) {
  constexpr unsigned m = (1u << IB) - 1u;
  return v > 0.0 ? ((__float_as_uint((float)(v * scale)) & ~m) | (m - (unsigned)i)) : 0u;
}
// a[r] of lane `lane` for a uniform r < N: every a[i] is read from the lane and the choice is made
// among the (uniform) results, so the array is never indexed dynamically (a select among the
// elements themselves may be folded into an indexed access, which puts the array in scratch)
template <int N>
__device__ __forceinline__ double readlane_pick(const double (&a)[N], int r, int lane) {
  double v = readlane_f64(a[0], lane);
#pragma unroll
  for (int i = 1; i < N; ++i) {
    const double w = readlane_f64(a[i], lane);
    v = r == i ? w : v;
  }
  return v;
}

// Index of the trailing matrix entry S(i, j): column-major with leading dimension K, or (PACKED) the
// lower triangle by columns, K (K + 1) / 2 entries.
template <bool PACKED>
__device__ __forceinline__ int s_idx(int i, int j, int K) {
  if (!PACKED) return i + K * j;
  const int lo = min(i, j), hi = max(i, j);
  return lo * (2 * K - lo - 1) / 2 + hi;
}

template <int NT, bool PACKED = false>
__device__ __forceinline__ int chol_phase_blk(const double* G, int K, double ctol, double* S, double* Lc, double* dk,
                                              int* perm, int* mark, CholShared& sh) {
  constexpr int RPL = CholBlk<NT>::RPL, NB = CholBlk<NT>::NB, IB = CholBlk<NT>::IB;
  constexpr unsigned IM = (1u << IB) - 1u;
  constexpr int TX = ChGrid<NT>::TX, TY = NT / TX, NBI = ChGrid<NT>::NBI, NBJ = ChGrid<NT>::NBJ;
  __shared__ int pstate[2];  // rank so far, 1 once the factorisation has stopped
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < K * K; e += NT) {
    const int i = e % K, j = e / K;
    if (PACKED && i < j) continue;
    S[s_idx<PACKED>(i, j, K)] = G[min(i, j) + (long)K * max(i, j)];
  }
  // wave 0: the Schur diagonal of rows lane + 64 r, the scale of the pivot keys, the threshold
  double d[RPL];
  bool alive[RPL];  // row not pivoted yet
  double scale = 0.0, stop = 0.0;
#pragma unroll
  for (int r = 0; r < RPL; ++r) { d[r] = 0.0; alive[r] = false; }
  if (wave == 0) {
    double dm = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = lane + 64 * r;
      alive[r] = row < K;
      d[r] = alive[r] ? G[row + (long)K * row] : 0.0;
      dm = fmax(dm, d[r]);
    }
    const double dmax0 = wave_max_f64(dm);
    scale = dmax0 > 0.0 ? 1.0 / dmax0 : 0.0;
    stop = ctol * dmax0;
    if (lane == 0) { pstate[0] = 0; pstate[1] = dmax0 > 0.0 ? 0 : 1; }
  }
  __syncthreads();
  for (int kb = 0; kb < K; kb += NB) {
    if (wave == 0) {
      int k = kb;
      bool done = false;
      double lrow[NB][RPL];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) lrow[t][r] = 0.0;
        if (done || kb + t >= K) continue;  // uniform
        unsigned kl = 0u;
#pragma unroll
        for (int r = 0; r < RPL; ++r) kl = max(kl, alive[r] ? pivot_key_ib<IB>(d[r], scale, lane + 64 * r) : 0u);
        const unsigned key = wave_max_u32(kl);
        const int p = (int)(IM - (key & IM)), pr = p >> 6, pl = p & 63;
        const double dp = readlane_pick(d, pr, pl);
        if (!key || !(dp > stop)) { done = true; continue; }  // uniform
        const double sp = sqrt(dp), rs = 1.0 / sp;
        double lp[NB];  // L(p, kb + u), u < t
#pragma unroll
        for (int u = 0; u < t; ++u) lp[u] = readlane_pick(lrow[u], pr, pl);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int row = lane + 64 * r;
          double c = row < K ? S[s_idx<PACKED>(row, p, K)] : 0.0;
#pragma unroll
          for (int u = 0; u < t; ++u) c = fma(-lrow[u][r], lp[u], c);
          const double l = row == p ? sp : c * rs;
          lrow[t][r] = l;
          if (row < K) Lc[(kb + t) * K + row] = l;
          if (row == p) alive[r] = false;
          d[r] = alive[r] ? fma(-l, l, d[r]) : 0.0;
        }
        if (lane == 0) { perm[kb + t] = p; dk[kb + t] = sp; }
        k = kb + t + 1;
      }
      if (lane == 0) { pstate[0] = k; pstate[1] = done ? 1 : 0; }
    }
    __syncthreads();
    if (pstate[1] || pstate[0] >= K) break;  // uniform
    // trailing update S -= L_panel L_panel^T: thread (tx, ty) owns (tx + TX a, ty + TY b), taken
    // AC rows at a time (the 1024-thread grid holds 64 entries per thread: two rows and one panel
    // column at a time keep them in registers)
    {
      constexpr int AC = NT == 1024 ? 2 : NBI, UT = NT == 1024 ? 1 : 4;
      const int tx = tid % TX, ty = tid / TX;
#pragma unroll
      for (int a0 = 0; a0 < NBI; a0 += AC) {
        double acc[AC][NBJ];
#pragma unroll
        for (int a = 0; a < AC; ++a)
#pragma unroll
          for (int b = 0; b < NBJ; ++b) acc[a][b] = 0.0;
#pragma unroll UT
        for (int t = 0; t < NB; ++t) {
          const double* Lt = Lc + (kb + t) * K;
          double li[AC], lj[NBJ];
#pragma unroll
          for (int a = 0; a < AC; ++a) li[a] = tx + TX * (a0 + a) < K ? Lt[tx + TX * (a0 + a)] : 0.0;
#pragma unroll
          for (int b = 0; b < NBJ; ++b) lj[b] = ty + TY * b < K ? Lt[ty + TY * b] : 0.0;
#pragma unroll
          for (int b = 0; b < NBJ; ++b)
#pragma unroll
            for (int a = 0; a < AC; ++a) acc[a][b] = fma(li[a], lj[b], acc[a][b]);
        }
#pragma unroll
        for (int b = 0; b < NBJ; ++b)
#pragma unroll
          for (int a = 0; a < AC; ++a) {
            const int i = tx + TX * (a0 + a), j = ty + TY * b;
            if (i < K && j < K && (!PACKED || i >= j)) S[s_idx<PACKED>(i, j, K)] -= acc[a][b];
          }
      }
    }
    __syncthreads();
  }
  const int q = pstate[0];
  // unpivoted indices (in increasing order) after the pivots, and their remaining trace
  for (int i = tid; i < K; i += NT) mark[i] = 0;
  __syncthreads();
  for (int k = tid; k < q; k += NT) mark[perm[k]] = 1;
  if (wave == 0) {
    double r2 = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) r2 += alive[r] ? fmax(d[r], 0.0) : 0.0;
    for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o);
    if (lane == 0) { sh.rest = r2; sh.q = q; }
  }
  __syncthreads();
  for (int i = tid; i < K; i += NT)
    if (!mark[i]) {
      int c = 0;
      for (int j = 0; j < i; ++j) c += mark[j] ? 0 : 1;
      perm[q + c] = i;
    }
  __syncthreads();
  return q;
}



// Rank-revealing orthonormalisation factor: W (K x q, ld K) = P[:, :q] R^-1, so that V W has
// orthonormal columns spanning V's numerically independent columns (G = V^T V); q to *J.q.
// R is gathered into pivot order (through registers when it overwrites the LDS copy of S).
// X = R^-1 column by column, 4 to 16 lanes per column: row i of column j needs
// sum_{i<l<=j} R(i, l) X(l, j), which the lanes split by l mod (lanes) and add with DPP; each
// lane keeps the X(l, j) of its own residue class, so no barrier is needed.
// K <= 64 on 256 threads: the blocked factorisation, then X = R^-1 with R transposed in pivot
// order (RT[l + K i] = R(i, l)).  Four lanes per column j of X, lane li holding the rows
// l = li (mod 4) in registers; the rows i are taken bottom-up in the same order by every column,
// so row i of R is a broadcast read, and X(i, j) = -(sum_{i<l<=j} R(i, l) X(l, j)) / R(i, i)
// needs only the X(l, j) the lane holds itself.  LDS: S and L (2 K^2), then dk, 1/R(i,i), perm.
__device__ __forceinline__ void pchol64(const CholJob& J, double* sm) {
  const int K = J.K, tid = threadIdx.x;
  double* S = sm;
  double* Lc = S + K * K;
  double* dk = Lc + K * K;
  double* xd = dk + K;
  int* perm = reinterpret_cast<int*>(xd + K);
  int* mark = reinterpret_cast<int*>(xd);  // free until the inverse
  __shared__ CholShared sh;
  const int q = chol_phase_blk<256>(J.g, K, J.tol, S, Lc, dk, perm, mark, sh);
  for (int e = tid; e < q * q; e += 256) {
    const int l = e % q, i = e / q;
    S[l + K * i] = l >= i ? Lc[i * K + perm[l]] : 0.0;
  }
  for (int i = tid; i < q; i += 256) xd[i] = 1.0 / Lc[i * K + perm[i]];
  __syncthreads();
  // X(li + 4 t, j) in xr[t]; the row loop is unrolled so that the owner's write has a fixed index
  const int j = tid >> 2, li = tid & 3;
  double xr[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) xr[t] = 0.0;
#pragma unroll
  for (int i = 63; i >= 0; --i) {
    if (i < q && j < q && i <= j) {  // the same for the four lanes of a column
      double part = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        if (4 * t + 3 > i) {  // rows l = li + 4 t <= i never contribute
          const int l = li + 4 * t;
          const double rv = S[min(l, j) + K * i];
          part = (l > i && l <= j) ? fma(rv, xr[t], part) : part;
        }
      }
      part += dpp_f64<0xB1>(part);
      part += dpp_f64<0x4E>(part);
      const double x = i == j ? xd[i] : -part * xd[i];
      if (li == (i & 3)) xr[i >> 2] = x;
    }
  }
  // W = P X: every row of column j written once (perm is a permutation of 0..K-1)
  if (j < q) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int l = li + 4 * t;
      if (l < K) J.w[perm[l] + (long)K * j] = l <= j ? xr[t] : 0.0;
    }
  }
  if (tid == 0 && J.q) *J.q = q;
}

template <bool SMEM, int NT>
__global__ __launch_bounds__(NT) void k_pchol(JobBatch<CholJob> jobs) {
  extern __shared__ double sm[];
  constexpr int KMAX = ChGrid<NT>::KMAX, NW = NT / 64;
  const CholJob J = jobs.j[blockIdx.x];
  const int K = J.K;
  const int tid = threadIdx.x;
  if (K <= 0) { if (tid == 0 && J.q) *J.q = 0; return; }
  if constexpr (NT == 256) {
    pchol64(J, sm);
    return;
  }
  // L in the job's global scratch (first K^2), the trailing matrix in LDS (K <= 128) or after L;
  // R and X = R^-1 then take the trailing matrix's place
  double* Lc = J.work;
  double* S = SMEM ? sm : J.work + (size_t)K * K;
  double* Rp = S;  // R (q x q, ld K, upper) then X = R^-1 below it
  double* base = SMEM ? sm + (size_t)K * K : sm;
  double* dk = base;
  double* xd = dk + K;
  int* perm = reinterpret_cast<int*>(xd + K + 2 * NW);
  __shared__ CholShared sh;
  int* mark = reinterpret_cast<int*>(xd);  // free until the inverse
  const int q = chol_phase_blk<NT>(J.g, K, J.tol, S, Lc, dk, perm, mark, sh);
  for (int e = tid; e < q * q; e += NT) {
    const int i = e % q, l = e / q;
    Rp[i + K * l] = i <= l ? Lc[i * K + perm[l]] : 0.0;
  }
  __syncthreads();
  // X(i, j) = -(sum_{i<l<=j} R(i, l) X(l, j)) / R(i, i), bottom-up; X(l, j), l < j, at Rp[j + K l]
  {
    const int lc = lanes_for(NT, q);
    const int lg = lc == 16 ? 4 : (lc == 8 ? 3 : (lc == 4 ? 2 : (lc == 2 ? 1 : 0)));
    for (int j0 = 0; j0 < q; j0 += NT / lc) {
      const int j = j0 + (tid >> lg), li = tid & (lc - 1);
      if (j < q) {
        const double xjj = 1.0 / Rp[j + K * j];
        if (li == 0) xd[j] = xjj;
        for (int i = j - 1; i >= 0; --i) {
          // lane li takes the l = i+1 .. j with l = li (mod lc): exactly the X(l, j) it wrote
          double part = 0.0;
#pragma unroll 4
          for (int l = i + 1 + ((li - i - 1) & (lc - 1)); l <= j; l += lc)
            part += Rp[i + K * l] * (l == j ? xjj : Rp[j + K * l]);
          const double acc = group_sum(part, lc);
          if ((i & (lc - 1)) == li) Rp[j + K * i] = -acc / Rp[i + K * i];
        }
      }
    }
  }
  for (int e = tid; e < K * q; e += NT) J.w[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < q * q; e += NT) {
    const int l = e % q, j = e / q;
    if (l > j) continue;
    J.w[perm[l] + (long)K * j] = (l == j) ? xd[l] : Rp[j + K * l];
  }
  if (tid == 0 && J.q) *J.q = q;
}

template <bool SMEM, int NT, typename Job>
hipError_t launch_gram(void (*kern)(JobBatch<Job>), const JobBatch<Job>& jobs, int count, size_t shm, hipStream_t s) {
  if (SMEM) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(count), dim3(NT), shm, s, jobs);
  return hipGetLastError();
}

// Orders 128 < K <= 192 on 1024 threads with everything in LDS but L: the trailing matrix as its
// packed lower triangle (K (K + 1) / 2 doubles, 148 KB at K = 192), L in the job's global scratch.
// R (pivot order) then takes the same place as a packed upper triangle by columns, and X = R^-1 is
// formed there by blocks of 64 rows and columns: the diagonal blocks X_II = R_II^-1 by the register
// scheme of pchol64 (256 threads each, all blocks at once), then
//   X_IJ = -X_II (sum_{I < L <= J} R_IL X_LJ),  I < J,
// every block product held in registers and written over the R block it replaces once no thread
// reads that block any more (the barriers between the steps).
constexpr int CHOL_PACKED_MAX = 192;

__device__ __forceinline__ int up_idx(int i, int l) { return l * (l + 1) / 2 + i; }

// Entries (a, c + 16 u), u < 4, of the product of the 64-blocks (ra, ca) and (rb, cb) of the
// packed upper triangle Rp (q x q) over the first kn indices; a diagonal block contributes its
// upper triangle only.  Out-of-range rows and columns are clamped into the matrix (their results
// are not used).
__device__ __forceinline__ void blk_mm4(const double* Rp, int q, int ra, int ca, int rb, int cb, int kn, int a, int c,
                                        double (&out)[4]) {
  const int gi = min(64 * ra + a, q - 1);
  for (int b = 0; b < kn; ++b) {
    const int gl = 64 * ca + b, gr = 64 * rb + b;
    const double av = gi <= gl ? Rp[up_idx(gi, gl)] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gc = min(64 * cb + c + 16 * u, q - 1);
      const double bv = gr <= gc ? Rp[up_idx(gr, gc)] : 0.0;
      out[u] = fma(av, bv, out[u]);
    }
  }
}
// Writes s * v[u] to the entries (a, c + 16 u) of the 64-block (rb, cb) that lie inside it.
__device__ __forceinline__ void blk_put4(double* Rp, int rb, int cb, int nr, int nc, int a, int c, double sgn,
                                         const double (&v)[4]) {
  if (a >= nr) return;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (c + 16 * u < nc) Rp[up_idx(64 * rb + a, 64 * cb + c + 16 * u)] = sgn * v[u];
}

__global__ __launch_bounds__(1024) void k_pchol_packed(JobBatch<CholJob> jobs) {
  extern __shared__ double sm[];
  constexpr int NT = 1024, NW = NT / 64;
  const CholJob J = jobs.j[blockIdx.x];
  const int K = J.K;
  const int tid = threadIdx.x;
  if (K <= 0) { if (tid == 0 && J.q) *J.q = 0; return; }
  double* Lc = J.work;
  double* S = sm;
  double* dk = sm + (size_t)K * (K + 1) / 2;
  double* xd = dk + K;
  int* perm = reinterpret_cast<int*>(xd + K + 2 * NW);
  int* mark = reinterpret_cast<int*>(xd);  // free until the inverse
  __shared__ CholShared sh;
  const int q = chol_phase_blk<NT, true>(J.g, K, J.tol, S, Lc, dk, perm, mark, sh);
  double* Rp = S;
  for (int e = tid; e < q * q; e += NT) {
    const int i = e % q, l = e / q;
    if (i <= l) Rp[up_idx(i, l)] = Lc[i * K + perm[l]];
  }
  for (int i = tid; i < q; i += NT) xd[i] = 1.0 / Lc[i * K + perm[i]];
  __syncthreads();
  const int nb = (q + 63) / 64;
  const int n0 = min(q, 64), n1 = max(0, min(q - 64, 64)), n2 = max(0, q - 128);
  // diagonal blocks: 256 threads per block, four lanes per column jj, lane li holding the rows
  // li (mod 4) of X(:, jj) in registers (rows bottom-up)
  {
    const int bI = tid >> 8, jj = (tid & 255) >> 2, li = tid & 3;
    const int o = 64 * bI, n = bI < nb ? min(64, q - o) : 0;
    double xr[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) xr[t] = 0.0;
#pragma unroll
    for (int i = 63; i >= 0; --i) {
      if (i < n && jj < n && i <= jj) {  // the same for the four lanes of a column
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          if (4 * t + 3 > i) {  // rows l = li + 4 t <= i never contribute
            const int l = li + 4 * t;
            const double rv = Rp[up_idx(o + i, o + min(l, n - 1))];
            part = (l > i && l <= jj) ? fma(rv, xr[t], part) : part;
          }
        }
        part += dpp_f64<0xB1>(part);
        part += dpp_f64<0x4E>(part);
        const double x = i == jj ? xd[o + i] : -part * xd[o + i];
        if (li == (i & 3)) xr[i >> 2] = x;
      }
    }
    __syncthreads();
    if (jj < n) {
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int l = li + 4 * t;
        if (l <= jj) Rp[up_idx(o + l, o + jj)] = xr[t];
      }
    }
    __syncthreads();
  }
  // off-diagonal blocks: thread (a, c) forms the entries (a, c + 16 u) of a block product
  const int a = tid & 63, c = tid >> 6;
  if (nb == 3) {
    double t23[4] = {0.0, 0.0, 0.0, 0.0};
    blk_mm4(Rp, q, 1, 2, 2, 2, n2, a, c, t23);           // R23 X33
    __syncthreads();
    blk_put4(Rp, 1, 2, n1, n2, a, c, 1.0, t23);
    __syncthreads();
    double x23[4] = {0.0, 0.0, 0.0, 0.0};
    blk_mm4(Rp, q, 1, 1, 1, 2, n1, a, c, x23);           // X22 (R23 X33)
    __syncthreads();
    blk_put4(Rp, 1, 2, n1, n2, a, c, -1.0, x23);        // X23
    __syncthreads();
    double t13[4] = {0.0, 0.0, 0.0, 0.0}, s12[4] = {0.0, 0.0, 0.0, 0.0};
    blk_mm4(Rp, q, 0, 1, 1, 2, n1, a, c, t13);           // R12 X23
    blk_mm4(Rp, q, 0, 2, 2, 2, n2, a, c, t13);           //   + R13 X33
    blk_mm4(Rp, q, 0, 1, 1, 1, n1, a, c, s12);           // R12 X22
    __syncthreads();
    blk_put4(Rp, 0, 2, n0, n2, a, c, 1.0, t13);
    blk_put4(Rp, 0, 1, n0, n1, a, c, 1.0, s12);
    __syncthreads();
    double x13[4] = {0.0, 0.0, 0.0, 0.0}, x12[4] = {0.0, 0.0, 0.0, 0.0};
    blk_mm4(Rp, q, 0, 0, 0, 2, n0, a, c, x13);
    blk_mm4(Rp, q, 0, 0, 0, 1, n0, a, c, x12);
    __syncthreads();
    blk_put4(Rp, 0, 2, n0, n2, a, c, -1.0, x13);        // X13
    blk_put4(Rp, 0, 1, n0, n1, a, c, -1.0, x12);        // X12
    __syncthreads();
  } else if (nb == 2) {
    double s12[4] = {0.0, 0.0, 0.0, 0.0};
    blk_mm4(Rp, q, 0, 1, 1, 1, n1, a, c, s12);           // R12 X22
    __syncthreads();
    blk_put4(Rp, 0, 1, n0, n1, a, c, 1.0, s12);
    __syncthreads();
    double x12[4] = {0.0, 0.0, 0.0, 0.0};
    blk_mm4(Rp, q, 0, 0, 0, 1, n0, a, c, x12);
    __syncthreads();
    blk_put4(Rp, 0, 1, n0, n1, a, c, -1.0, x12);        // X12
    __syncthreads();
  }
  // W = P X: every row of column j written once (perm is a permutation of 0..K-1)
  for (int e = tid; e < K * q; e += NT) J.w[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < q * q; e += NT) {
    const int l = e % q, j = e / q;
    if (l <= j) J.w[perm[l] + (long)K * j] = Rp[up_idx(l, j)];
  }
  if (tid == 0 && J.q) *J.q = q;
}

hipError_t pchol_batched(const JobBatch<CholJob>& jobs_dev, int count, int Kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kBatchJobs) return hipErrorInvalidValue;
  if (Kmax > EIG_MAX) return hipErrorInvalidValue;
  const size_t extra = (size_t)Kmax * 16 + 32 * 8 + (size_t)Kmax * 4 + 64;
  const size_t shm = (size_t)Kmax * Kmax * 8 + extra;
  if (Kmax <= 64)
    return launch_gram<true, 256>(k_pchol<true, 256>, jobs_dev, count, (size_t)Kmax * Kmax * 16 + (size_t)Kmax * 20 + 64, s);
  if (Kmax <= EIG_LDS_MAX) return launch_gram<true, 512>(k_pchol<true, 512>, jobs_dev, count, shm, s);
  if (Kmax <= CHOL_PACKED_MAX)
    return launch_gram<true, 1024>(k_pchol_packed, jobs_dev, count, (size_t)Kmax * (Kmax + 1) / 2 * 8 + extra, s);
  return launch_gram<false, 1024>(k_pchol<false, 1024>, jobs_dev, count, extra, s);
}

// ---------------------------------------------------------------------------------------------
// Inverse square root of Gram matrices near the identity (the second pass of an orthonormalisation,
// whose Gram is I + E with E of the order of the first pass's loss of orthogonality) by the coupled
// Newton-Schulz iteration (Higham, Functions of Matrices, Sec. 6.3): Y0 = G, Z0 = I,
// T = (3 I - Z Y) / 2, Y <- Y T, Z <- T Z, which converges quadratically to Y = G^(1/2),
// Z = G^(-1/2) when ||I - G||_2 < 1.  One workgroup per matrix, Y, Z, T in LDS (K <= kNsMax).
// ok = 0 (W untouched) when ||G - I||_F > 1/2 or the iteration has not converged in 10 steps.
// ---------------------------------------------------------------------------------------------
__device__ double block_max256(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// The iterates are padded to 64 x 64 (G with the identity, so the padding stays the identity)
// and kept in LDS with leading dimension NS_LD; the 64 x 64 x 64 products run on the FP64 matrix
// cores, wave w computing rows 16 w .. 16 w + 15 as four 16 x 16 blocks.  Y, Z and T are
// functions of G, so they are symmetric and commute: the second factor is read as its transpose
// and the product is stored transposed, which keeps every LDS access contiguous along the 16
// lanes of a block row (the difference is of the order of the rounding of the products).
constexpr int NS_LD = 72;  // 144 dwords: the four lane groups of a read start 16 banks apart

// acc[cb][v] = (A B)[16 w + c + 4 v][16 cb + r] for lane (r, c) = (lane % 16, lane / 16)
__device__ __forceinline__ void ns_mm64(const double* A, const double* B, d4_t acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, c = lane >> 4;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < 64; k0 += 4) {
    const double a = A[(16 * w + r) + NS_LD * (k0 + c)];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma16(a, B[(16 * cb + r) + NS_LD * (k0 + c)], acc[cb]);
  }
}
// stores acc transposed: M[16 cb + r][16 w + c + 4 v] (column-major, ld NS_LD)
__device__ __forceinline__ void ns_store(double* M, const d4_t acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, c = lane >> 4;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) M[(16 * cb + r) + NS_LD * (16 * w + c + 4 * v)] = acc[cb][v];
}

__global__ __launch_bounds__(256) void k_ns_isqrt(JobBatch<NsJob> jobs) {
  extern __shared__ double sm[];
  __shared__ double red[4];
  const NsJob J = jobs.j[blockIdx.x];
  const int K = J.K, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, r = lane & 15, c = lane >> 4;
  double* Y = sm;
  double* Z = sm + 64 * NS_LD;
  double* T = sm + 2 * 64 * NS_LD;
  if (K <= 0) {
    if (tid == 0) *J.ok = 1;
    return;
  }
  double e2 = 0.0;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e & 63, j = e >> 6;
    const double id = i == j ? 1.0 : 0.0;
    const double g = (i < K && j < K) ? J.g[i + K * j] : id;
    Y[i + NS_LD * j] = g;
    Z[i + NS_LD * j] = id;
    e2 += (g - id) * (g - id);
  }
  // ||G - I||_F^2 as a block sum
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o);
  if (lane == 0) red[w] = e2;
  __syncthreads();
  const double fro2 = red[0] + red[1] + red[2] + red[3];
  if (!(fro2 <= 0.25)) {  // uniform
    if (tid == 0) *J.ok = 0;
    return;
  }
  bool done = false;
  for (int it = 0; it < 10 && !done; ++it) {
    d4_t o[4];
    ns_mm64(Z, Y, o);  // T = 1.5 I - 0.5 Z Y
    double dev = 0.0;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool dg = (16 * w + c + 4 * v) == (16 * cb + r);
        const double t = (dg ? 1.5 : 0.0) - 0.5 * o[cb][v];
        o[cb][v] = t;
        dev = fmax(dev, fabs(t - (dg ? 1.0 : 0.0)));
      }
    ns_store(T, o);
    for (int s2 = 32; s2 > 0; s2 >>= 1) dev = fmax(dev, __shfl_xor(dev, s2));
    __syncthreads();  // T published; every wave is done with this iteration's reads of red
    if (lane == 0) red[w] = dev;
    d4_t y[4], z[4];
    ns_mm64(Y, T, y);
    ns_mm64(T, Z, z);
    __syncthreads();  // every read of Y, Z, T is done, and red is published
    dev = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    ns_store(Y, y);
    ns_store(Z, z);
    __syncthreads();
    // T - I is of the order of the remaining error and the step squares it: from 1e-10 this step
    // has brought Z to G^(-1/2) to working precision (the products' rounding, ~K eps, is larger
    // than what a further step would remove)
    done = dev <= 1e-10;
  }
  for (int e = tid; e < K * K; e += 256) J.w[e] = Z[(e % K) + NS_LD * (e / K)];
  if (tid == 0) *J.ok = done ? 1 : 0;
}

hipError_t ns_isqrt_batched(const JobBatch<NsJob>& jobs, int count, int Kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kBatchJobs || Kmax > kNsMax) return hipErrorInvalidValue;
  const size_t shm = (size_t)3 * 64 * NS_LD * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_ns_isqrt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ns_isqrt, dim3(count), dim3(256), shm, s, jobs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Eigenpairs of a positive semidefinite Gram matrix G (K x K) by the preconditioned one-sided
// Jacobi method: pivoted Cholesky G[P,P] = R^T R, then Jacobi rotations orthogonalise the
// columns of X = R^T (K x q).  At convergence X = V Sigma with V the eigenvectors of G[P,P]
// and Sigma^2 its eigenvalues, so no rotation needs to be accumulated.  One barrier per
// Jacobi step: the column pairs of a step are disjoint, the 4 to 16 lanes that share a pair
// hold its rows in registers and add their partial dot products with DPP.
// ---------------------------------------------------------------------------------------------
// One-sided Jacobi on the q <= 32 columns of X (K <= 4 RT rows, ld K) by one wave: 4 lanes per
// column pair hold the rows li + 4 t (t < RT) of both columns in registers and add their partial
// dot products with two quad DPP steps.  A wave's LDS accesses are performed in order, so the
// rounds need no barrier (the pairs of a round are disjoint).  The same rotation rule and stopping
// test as the workgroup version; returns when the sweeps have converged.
template <int RT>
__device__ __forceinline__ void jacobi_wave(double* X, int K, int q, double jtol) {
  const int lane = threadIdx.x & 63;
  const int qp = q + (q & 1), np = qp / 2;
  const int pr = lane >> 2, li = lane & 3;
  const double jtol2 = jtol * jtol;
  for (int sweep = 0; sweep < 40 && q > 1; ++sweep) {
    float mx = 0.0f;  // the largest squared relative off-diagonal rotated away in this sweep
    for (int st = 0; st < qp - 1; ++st) {
      int p = 0, r = 0;
      bool valid = pr < np;
      if (valid) {
        p = rr_index(pr, st, qp);
        r = rr_index(qp - 1 - pr, st, qp);
        if (p > r) { const int t = p; p = r; r = t; }
        valid = r < q;
      }
      double xa[RT], xb[RT], al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int i = li + 4 * t;
        const bool in = valid && i < K;
        const int ic = min(i, K - 1);
        const double a = X[ic + K * p], b = X[ic + K * r];
        xa[t] = in ? a : 0.0;
        xb[t] = in ? b : 0.0;
      }
#pragma unroll
      for (int t = 0; t < RT; ++t) { al += xa[t] * xa[t]; be += xb[t] * xb[t]; ga += xa[t] * xb[t]; }
      al += dpp_f64<0xB1>(al); be += dpp_f64<0xB1>(be); ga += dpp_f64<0xB1>(ga);
      al += dpp_f64<0x4E>(al); be += dpp_f64<0x4E>(be); ga += dpp_f64<0x4E>(ga);
      const double ab = al * be;
      if (valid && ga * ga > jtol2 * ab) {  // the same for the four lanes of a pair
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = rsqrt(1.0 + t * t), sn = c * t;
#pragma unroll
        for (int u = 0; u < RT; ++u) {
          const int i = li + 4 * u;
          if (i < K) {
            X[i + K * p] = c * xa[u] - sn * xb[u];
            X[i + K * r] = sn * xa[u] + c * xb[u];
          }
        }
        mx = fmaxf(mx, (float)((ga * ga) / ab));
      }
      __builtin_amdgcn_wave_barrier();
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (mx == 0.0f || (double)mx * (double)q <= jtol) break;  // uniform
  }
}

// PACKED (orders 129..CHOL_PACKED_MAX): the factorisation's trailing matrix packed in LDS, X in
// global memory.
template <bool SMEM, int NT, bool PACKED = false>
__global__ __launch_bounds__(NT) void k_psd_eig(JobBatch<PsdJob> jobs) {
  extern __shared__ double sm[];
  constexpr int KMAX = ChGrid<NT>::KMAX, NW = NT / 64;
  const PsdJob J = jobs.j[blockIdx.x];
  const int K = J.K;
  const int tid = threadIdx.x;
  if (K <= 0) {
    if (tid == 0) { *J.q = 0; *J.rest = 0.0; }
    return;
  }
  // K > 64: L in the job's global scratch (first K^2), the trailing matrix in LDS (K <= 128, or
  // packed) or after L, and X in the trailing matrix's place (after L when it was packed)
  double* S = (SMEM || PACKED) ? sm : J.work + (size_t)K * K;
  double* X = PACKED ? J.work + (size_t)K * K : S;     // K x q, ld K
  double* base = SMEM ? sm + (size_t)K * K : (PACKED ? sm + (size_t)K * (K + 1) / 2 : sm);
  double* dk = base;                                   // K pivots; later column norms^2
  unsigned long long* slot = reinterpret_cast<unsigned long long*>(dk + K);  // 2 x NW keys
  int* perm = reinterpret_cast<int*>(slot + 2 * NW);   // K
  int* rank = perm + K;                                // K: output position of each column
  __shared__ CholShared sh;
  // per sweep: the largest squared relative off-diagonal (x_p.x_r)^2 / (|x_p|^2 |x_r|^2) that
  // was rotated away, as float bits (non-negative floats order like their bit patterns)
  __shared__ unsigned int offmax[3];
  if (tid == 0) offmax[0] = offmax[1] = offmax[2] = 0u;
  int q;
  if constexpr (NT == 256) {
    // blocked factorisation with L in its own LDS block (after the job's scratch), then
    // X = R^T in pivot order: X[l][k] = R(k, l) = L(perm[l], k) (l >= k), 0 above the diagonal
    double* Lc = base + 2 * K + 32;
    q = chol_phase_blk<256>(J.g, K, J.ctol, S, Lc, dk, perm, rank, sh);
    for (int e = tid; e < K * q; e += NT) {
      const int l = e % K, k = e / K;
      X[e] = l >= k ? Lc[k * K + perm[l]] : 0.0;
    }
  } else {
    double* Lc = J.work;
    q = chol_phase_blk<NT, PACKED>(J.g, K, J.ctol, S, Lc, dk, perm, rank, sh);
    for (int e = tid; e < K * q; e += NT) {
      const int l = e % K, k = e / K;
      X[e] = l >= k ? Lc[k * K + perm[l]] : 0.0;
    }
  }
  __syncthreads();
  // one-sided Jacobi on the q columns of X (round-robin pairs, L lanes per pair); up to 32 columns
  // of up to 64 rows (the least-squares fits of the symbols) by one wave without barriers
  bool jdone = false;
  if constexpr (NT == 256) {
    if (q <= 32 && K <= 64) {
      if ((tid >> 6) == 0) {
        if (K <= 32) jacobi_wave<8>(X, K, q, J.jtol);
        else jacobi_wave<16>(X, K, q, J.jtol);
      }
      jdone = true;
    }
  }
  const int qp = q + (q & 1), np = qp / 2;
  const int L = lanes_for(NT, np);
  const int lg = L == 16 ? 4 : (L == 8 ? 3 : (L == 4 ? 2 : (L == 2 ? 1 : 0)));
  const int pr = tid >> lg, li = tid & (L - 1);
  // rows per lane held in registers: KMAX / (lanes per pair), the lanes being at least
  // NT / (KMAX / 2) (or 1)
  constexpr int LMIN = (2 * NT) / KMAX > 0 ? (2 * NT) / KMAX : 1;
  constexpr int RMAX = SMEM ? (KMAX + LMIN - 1) / LMIN : 1;
  static_assert((RMAX & (RMAX - 1)) == 0, "row blocks per lane: a power of two");
  // The columns lie K doubles apart, a multiple of the LDS bank period when K is a multiple of
  // 16, so pairs that read the same rows of their columns hit the same banks.  Each pair walks
  // its row blocks from a different start (pr mod RMAX): the pairs of a wave then touch disjoint
  // row blocks at every load and store.  A lane still covers the rows li + L t, t < RMAX.
  const int rot = pr & (RMAX - 1);
  const double jtol2 = J.jtol * J.jtol;
  for (int sweep = 0; sweep < 40 && q > 1 && !jdone; ++sweep) {
    unsigned int* chg = &offmax[sweep % 3];
    if (tid == 0) offmax[(sweep + 1) % 3] = 0u;  // last read two sweeps ago
    for (int st = 0; st < qp - 1; ++st) {
      int p = 0, r = 0;
      bool valid = pr < np;
      if (valid) {
        p = rr_index(pr, st, qp);
        r = rr_index(qp - 1 - pr, st, qp);
        if (p > r) { const int t = p; p = r; r = t; }
        valid = r < q;
      }
      double al = 0.0, be = 0.0, ga = 0.0;
      double xa[RMAX], xb[RMAX];
      if (SMEM) {
#pragma unroll
        for (int t = 0; t < RMAX; ++t) {
          const int i = li + L * ((t + rot) & (RMAX - 1));
          const bool in = valid && i < K;
          xa[t] = in ? X[i + K * p] : 0.0;
          xb[t] = in ? X[i + K * r] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < RMAX; ++t) { al += xa[t] * xa[t]; be += xb[t] * xb[t]; ga += xa[t] * xb[t]; }
      } else if (valid) {
        for (int i = li; i < K; i += L) {
          const double a = X[i + K * p], b = X[i + K * r];
          al += a * a; be += b * b; ga += a * b;
        }
      }
      al = group_sum(al, L);
      be = group_sum(be, L);
      ga = group_sum(ga, L);
      // rotate while |ga| / sqrt(al be) > jtol, tested on the squares (no square root)
      const double ab = al * be;
      if (valid && ga * ga > jtol2 * ab) {
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = rsqrt(1.0 + t * t), sn = c * t;
        if (SMEM) {
#pragma unroll
          for (int u = 0; u < RMAX; ++u) {
            const int i = li + L * ((u + rot) & (RMAX - 1));
            if (i < K) {
              X[i + K * p] = c * xa[u] - sn * xb[u];
              X[i + K * r] = sn * xa[u] + c * xb[u];
            }
          }
        } else {
          for (int i = li; i < K; i += L) {
            const double a = X[i + K * p], b = X[i + K * r];
            X[i + K * p] = c * a - sn * b;
            X[i + K * r] = sn * a + c * b;
          }
        }
        // the squared relative off-diagonal that was rotated away
        if (li == 0) atomicMax(chg, __float_as_uint((float)((ga * ga) / ab)));
      }
      __syncthreads();
    }
    // read by every thread after the sweep's last barrier.  Stop when nothing was rotated, or
    // when every rotation was so small that the sweep's quadratic convergence leaves the
    // columns orthogonal to jtol: off-diagonals after a sweep are O(K max^2).
    const float mx2 = __uint_as_float(*chg);
    if (mx2 == 0.0f || (double)mx2 * (double)q <= J.jtol) break;
  }
  __syncthreads();
  // eigenvalues = squared column norms (16 lanes per column), sorted descending;
  // eigenvectors = normalised columns
  for (int c0 = 0; c0 < q; c0 += NT / 16) {
    const int i = c0 + (tid >> 4), l0 = tid & 15;
    double s2 = 0.0;
    if (i < q)
      for (int l = l0; l < K; l += 16) s2 += X[l + K * i] * X[l + K * i];
    s2 = group_sum(s2, 16);
    if (i < q && l0 == 0) dk[i] = s2;
  }
  __syncthreads();
  for (int i = tid; i < q; i += NT) {
    const double di = dk[i];
    int rk = 0;
    for (int j = 0; j < q; ++j) {
      const double dj = dk[j];
      if (dj > di || (dj == di && j < i)) ++rk;
    }
    rank[i] = rk;
  }
  for (int i = tid; i < K; i += NT) J.w[i] = 0.0;
  __syncthreads();
  for (int e = tid; e < K * K; e += NT) {
    const int l = e % K, i = e / K;
    if (i >= q) { J.v[e] = 0.0; continue; }
    const double nrm = sqrt(dk[i]);
    J.v[perm[l] + (long)K * rank[i]] = nrm > 0.0 ? X[l + K * i] / nrm : 0.0;
  }
  for (int i = tid; i < q; i += NT) J.w[rank[i]] = dk[i];
  if (tid == 0) { *J.q = q; *J.rest = sh.rest; }
}

hipError_t psd_eig_batched(const JobBatch<PsdJob>& jobs_dev, int count, int Kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kBatchJobs) return hipErrorInvalidValue;
  if (Kmax > EIG_MAX) return hipErrorInvalidValue;
  const size_t extra = (size_t)Kmax * 8 + 32 * 8 + (size_t)Kmax * 8 + 64;
  const size_t shm = (size_t)Kmax * Kmax * 8 + extra;
  // K <= 64: the factor L in its own block after the scratch
  if (Kmax <= 64) return launch_gram<true, 256>(k_psd_eig<true, 256>, jobs_dev, count, shm + (size_t)Kmax * Kmax * 8, s);
  if (Kmax <= EIG_LDS_MAX) return launch_gram<true, 512>(k_psd_eig<true, 512>, jobs_dev, count, shm, s);
  if (Kmax <= CHOL_PACKED_MAX)
    return launch_gram<true, 1024>(k_psd_eig<false, 1024, true>, jobs_dev, count,
                                   (size_t)Kmax * (Kmax + 1) / 2 * 8 + extra, s);
  return launch_gram<false, 1024>(k_psd_eig<false, 1024>, jobs_dev, count, extra, s);
}

// ---------------------------------------------------------------------------------------------
// Gram eigenpairs by reduction to tridiagonal form, K <= kTriMax, one workgroup of 512 threads
// (8 waves) per matrix, in registers and LDS:
//  1. Householder reduction G = Q T Q^T with Q accumulated.  Thread (l, c) = (tid % 64, tid / 64)
//     holds row l, columns = c (mod 8), of A and of Q in registers; every wave forms the reflector
//     from the published row by itself, and two barriers per step separate the products B v, Q v
//     from the rank-2 and rank-1 updates.
//  2. T + sigma I = L D L^T with every pivot positive (sigma = 0, or a multiple of eps ||T|| when
//     rounding left T without a positive definite factorisation): a representation that fixes
//     its eigenvalues to high relative accuracy.
//  3. Eigenvalue i by multisection: four lanes per eigenvalue with two points each (nine
//     subintervals per step, geometric while the interval spans more than a factor two), every
//     point counted by the stationary qd transform L D L^T - x I = L+ D+ L+^T (the number of
//     negative D+), down to a relative width of 2^-46.
//  4. Eigenvector i (lane i of wave 0) from the twisted factorisation at its eigenvalue: the
//     stationary transform from the top and the progressive one from the bottom meet at the index
//     r of smallest |gamma_r|; z_r = 1 and the multipliers of the two factorisations give the rest.
//     For a positive definite L D L^T these vectors are accurate to about eps / (relative gap).
//  5. Check |Z^T Z - I| over the kept eigenvectors (eigenvalue > ctol * trace) where the theory
//     does not already bound it (eigenvalues within 1 % of each other, and every norm): above jtol
//     (clustered eigenvalues) the job reports q = -1 and writes nothing else.
//  6. V = Q Z, kept eigenvectors in descending order of eigenvalue, zero columns after them.
// ---------------------------------------------------------------------------------------------
constexpr int TRI_NT = 512;                  // 8 waves: column classes of the reduction
constexpr int TRI_NW = TRI_NT / 64;
constexpr int TRI_CPT = kTriMax / TRI_NW;    // columns of A and Q per thread
constexpr int TRI_LD = kTriMax + 1;   // odd leading dimension: the rows of a column sit in distinct banks
constexpr double kTiny = 2.2250738585072014e-308;

// Minimum over the four lanes of a quad (DPP quad permutations).
__device__ __forceinline__ int quad_min(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));
  return min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
}
// 1/p from the hardware reciprocal and one Newton step (a few ulps).
__device__ __forceinline__ double recip(double p) {
  const double r = __builtin_amdgcn_rcp(p);
  return r * fma(-p, r, 2.0);
}

// Orders this wave's LDS writes before its later LDS reads of other lanes' entries.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Negative pivots of L D L^T - x I at two points at once (independent chains): the stationary qd
// transform D+_k = D_k + s_k, s_{k+1} = (s_k / D+_k) D_k L_k^2 - x, the quotient from the refined
// hardware reciprocal (an error of a few ulps in it is a perturbation of the representation of that
// relative size).  The loop carries no guard; a zero pivot or an overflow ends in a non-finite s, and
// that chain is counted again with a zero pivot taken as the smallest negative number and a
// quotient inf / inf as 1.
__device__ __forceinline__ int sturm_guarded(const double* D, const double* DL2, int K, double x) {
  double s = -x;
  int n = 0;
  for (int k = 0; k + 1 < K; ++k) {
    double p = D[k] + s;
    if (p == 0.0) p = -kTiny;
    n += p < 0.0 ? 1 : 0;
    double t = s * recip(p);
    if (t != t) t = 1.0;
    s = t * DL2[k] - x;
  }
  return n + ((D[K - 1] + s) < 0.0 ? 1 : 0);
}
__device__ __forceinline__ void sturm2(const double* D, const double* DL2, int K, double x0, double x1, int& c0,
                                       int& c1) {
  double s0 = -x0, s1 = -x1;
  int n0 = 0, n1 = 0;
#pragma unroll 8
  for (int k = 0; k + 1 < K; ++k) {
    const double dk = D[k], dl = DL2[k];
    const double p0 = dk + s0, p1 = dk + s1;
    n0 += p0 < 0.0 ? 1 : 0;
    n1 += p1 < 0.0 ? 1 : 0;
    s0 = (s0 * recip(p0)) * dl - x0;
    s1 = (s1 * recip(p1)) * dl - x1;
  }
  c0 = n0 + ((D[K - 1] + s0) < 0.0 ? 1 : 0);
  c1 = n1 + ((D[K - 1] + s1) < 0.0 ? 1 : 0);
  if (!isfinite(s0)) c0 = sturm_guarded(D, DL2, K, x0);
  if (!isfinite(s1)) c1 = sturm_guarded(D, DL2, K, x1);
}

// Point k (0..TRI_SEC) of the multisection of [a, b] into TRI_SEC parts: geometric while
// b > 2a > 0, else equidistant.
constexpr int TRI_SEC = 9;
// The geometric grid of the initial Sturm counts over [2^-60 T0, T0].
constexpr int TRI_GRID = 512;
__device__ __forceinline__ double tri_grid(double T0, int t) {
  return T0 * exp2(60.0 * ((double)t / (double)(TRI_GRID - 1) - 1.0));
}
__device__ __forceinline__ double tri_split(double a, double b, int k) {
  if (k <= 0) return a;
  if (k >= TRI_SEC) return b;
  if (a > 0.0 && b > 2.0 * a) {
    const double la = log2(a), lb = log2(b);
    return exp2(la + (lb - la) * (k * (1.0 / TRI_SEC)));
  }
  return a + (b - a) * (k * (1.0 / TRI_SEC));
}

// C (K x K) = X^T Y or X Y over LDS operands with leading dimension TRI_LD, 4 x 4 outputs per
// thread (rows 4 (tid % 16) .., columns 4 (tid / 16) ..).  TX: X is read transposed (X^T Y).
template <bool TX>
__device__ __forceinline__ void tri_mm44(const double* X, const double* Y, int K, double acc[4][4]) {
  const int r0 = 4 * (threadIdx.x % 16), c0 = 4 * (threadIdx.x / 16);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k = 0; k < K; ++k) {
    double x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = min(r0 + a, K - 1);
      x[a] = TX ? X[k + TRI_LD * r] : X[r + TRI_LD * k];
      y[a] = Y[k + TRI_LD * min(c0 + a, K - 1)];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
  }
}

__global__ __launch_bounds__(TRI_NT) void k_psd_tri(JobBatch<PsdJob> jobs) {
  extern __shared__ double sm[];
  const PsdJob J = jobs.j[blockIdx.x];
  const int K = J.K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (K <= 0) {
    if (tid == 0) { *J.q = 0; *J.rest = 0.0; }
    return;
  }
  double* A = sm;                          // Z (eigenvectors of T)
  double* Q = A + kTriMax * TRI_LD;        // K x K: the accumulated reflections, after the reduction
  double* Lp = Q + kTriMax * TRI_LD;       // [k][lane]: multipliers of the eigenvector phase
  double* Um = Lp + kTriMax * 64;
  double* dv = Um + kTriMax * 64;          // diagonal of T
  double* ev = dv + kTriMax;               // off-diagonal of T
  double* D = ev + kTriMax;                // T + sigma I = L D L^T
  double* L = D + kTriMax;
  double* DL2 = L + kTriMax;               // D_k L_k^2
  double* lam = DL2 + kTriMax;             // eigenvalues of T + sigma I, ascending
  double* vw = lam + kTriMax;              // per-wave copies of the reflector v (by absolute index), 8 x 64
  double* ww = vw + TRI_NW * 64;           // per-wave copies of w, 8 x 64
  double* pw = ww + TRI_NW * 64;           // partial B v per column class, 8 x 64
  double* qw = pw + TRI_NW * 64;           // partial Q v per column class, 8 x 64
  double* xb = qw + TRI_NW * 64;           // the row of A that the next reflection starts from, 64
  double* red = xb + 64;                   // 16 scalars
  // ---- 1. Householder reduction.  Thread (l, w) keeps A[l][w + 8t] and Q[l][w + 8t], t < 8, in
  // registers; the reflector of step j comes from row j (= column j), which the owners of that row
  // publish in xb at the end of the previous step.
  double ar[TRI_CPT], qr[TRI_CPT];
#pragma unroll
  for (int t = 0; t < TRI_CPT; ++t) {
    const int k = wave + TRI_NW * t;
    ar[t] = (lane < K && k < K) ? J.g[lane + (long)K * k] : 0.0;
    qr[t] = (lane == k && k < K) ? 1.0 : 0.0;
  }
  if (lane == 0)
#pragma unroll
    for (int t = 0; t < TRI_CPT; ++t)
      if (wave + TRI_NW * t < K) xb[wave + TRI_NW * t] = ar[t];
  __syncthreads();
  for (int j = 0; j + 2 < K; ++j) {
    const int o = j + 1;
    const double xl = (lane >= o && lane < K) ? xb[lane] : 0.0;   // A[l][j], l > j
    const double a2 = wave_sum_f64(xl * xl);
    const double x0 = readlane_f64(xl, o);
    const double al = sqrt(a2);
    const double beta = x0 >= 0.0 ? -al : al;
    const double tau = a2 > 0.0 ? 1.0 / (al * (al + fabs(x0))) : 0.0;
    const double vl = lane == o ? x0 - beta : xl;                  // v by absolute index, zero above o
    double* v = vw + 64 * wave;
    double* w = ww + 64 * wave;
    v[lane] = vl;
    wave_lds_sync();
    double pb = 0.0, pq = 0.0;
#pragma unroll
    for (int t = 0; t < TRI_CPT; ++t) {
      const double vk = v[wave + TRI_NW * t];
      pb += ar[t] * vk;
      pq += qr[t] * vk;
    }
    pw[64 * wave + lane] = pb;
    qw[64 * wave + lane] = pq;
    if (tid == 0) {
      dv[j] = xb[j];
      ev[j] = a2 > 0.0 ? beta : x0;
    }
    __syncthreads();
    // p = tau B v on the trailing rows, w = p - (tau/2)(p.v) v; every wave forms all of w
    double sp = 0.0, sq = 0.0;
#pragma unroll
    for (int c = 0; c < TRI_NW; ++c) {
      sp += pw[64 * c + lane];
      sq += qw[64 * c + lane];
    }
    const double pl = lane >= o ? tau * sp : 0.0;
    const double ql = tau * sq;
    const double k2 = wave_sum_f64(pl * vl);
    const double wl = pl - 0.5 * tau * k2 * vl;
    w[lane] = wl;
    wave_lds_sync();
    // B -= v w^T + w v^T, Q -= (Q v) tau v^T: v and w vanish outside the trailing block
#pragma unroll
    for (int t = 0; t < TRI_CPT; ++t) {
      const int k = wave + TRI_NW * t;
      const double vk = v[k], wk = w[k];
      ar[t] -= vl * wk + wl * vk;
      qr[t] -= ql * vk;
    }
    if (lane == o)
#pragma unroll
      for (int t = 0; t < TRI_CPT; ++t)
        if (wave + TRI_NW * t < K) xb[wave + TRI_NW * t] = ar[t];
    __syncthreads();
  }
  // Q to LDS for the back transformation
#pragma unroll
  for (int t = 0; t < TRI_CPT; ++t)
    if (lane < K && wave + TRI_NW * t < K) Q[lane + TRI_LD * (wave + TRI_NW * t)] = qr[t];
  // ---- 2. the last 2 x 2 block (row K-2 is in xb; A[K-1][K-1] is in its owner's registers), then
  // L D L^T of T + sigma I (one thread)
  if (lane == K - 1)
#pragma unroll
    for (int t = 0; t < TRI_CPT; ++t)
      if (wave + TRI_NW * t == K - 1) red[4] = ar[t];
  __syncthreads();
  if (wave == 0) {
    // lane i holds d_i and e_i; the factorisation runs through them with readlane / writelane
    double di = lane < K - 2 ? dv[lane] : 0.0;
    double ei = lane < K - 2 ? ev[lane] : 0.0;
    if (K >= 2) {
      if (lane == K - 2) { di = xb[K - 2]; ei = xb[K - 1]; }
      if (lane == K - 1) di = red[4];
    } else if (lane == 0) {
      di = xb[0];
    }
    const double eim1 = __shfl_up(ei, 1);
    const double off = (lane > 0 ? fabs(eim1) : 0.0) + (lane + 1 < K ? fabs(ei) : 0.0);
    const double tn = wave_max_f64(lane < K ? fabs(di) + off : 0.0);
    const double tr = wave_sum_f64(lane < K ? di : 0.0);
    double sigma = 0.0, Di = 0.0, Li = 0.0, DLi = 0.0;
    bool ok = false;
    for (int tries = 0; tries < 24 && !ok && tn > 0.0; ++tries) {
      double dp = readlane_f64(di, 0) + sigma;
      ok = dp > 0.0;
      if (lane == 0) Di = dp;
      for (int i = 0; i + 1 < K && ok; ++i) {
        const double e = readlane_f64(ei, i);
        const double li = e * recip(dp);
        if (lane == i) { Li = li; DLi = e * li; }
        dp = readlane_f64(di, i + 1) + sigma - li * e;
        if (lane == i + 1) Di = dp;
        ok = dp > 0.0;
      }
      if (!ok) sigma = sigma == 0.0 ? 2.220446049250313e-16 * tn : 4.0 * sigma;
    }
    if (lane < K) {
      dv[lane] = di;
      D[lane] = Di;
      L[lane] = Li;
      DL2[lane] = DLi;
    }
    if (lane == 0) {
      red[0] = sigma;
      red[1] = tn;
      red[2] = tr;
      red[3] = ok ? 1.0 : (tn > 0.0 ? -1.0 : 0.0);
    }
  }
  __syncthreads();
  const double sigma = red[0], tn = red[1], tr = red[2], st = red[3];
  if (st <= 0.0) {
    // zero matrix: no eigenpair kept; no positive definite shift found: let the caller decide
    if (st == 0.0) {
      for (int e = tid; e < K * K; e += TRI_NT) J.v[e] = 0.0;
      for (int o = tid; o < K; o += TRI_NT) J.w[o] = 0.0;
    }
    if (tid == 0) {
      *J.q = st == 0.0 ? 0 : -1;
      if (st == 0.0) *J.rest = 0.0;
    }
    return;
  }
  // ---- 3. eigenvalues of T + sigma I by multisection (eigenvalue tid / 4, ascending).  First the
  // Sturm counts at TRI_GRID geometric points x_t = ||T|| 2^(60 (t / (TRI_GRID - 1) - 1)), two per
  // thread of the first half; each eigenvalue i then starts from the bracket [x_lo, x_hi) with
  // count(x_lo) <= i < count(x_hi), hi = lo + 1 (a ratio of 2^(60 / 511), about 1.085), found by
  // bisection over t, and the four lanes of a quad count at the 8 interior points of TRI_SEC
  // subintervals of it.
  const double T0 = tn + sigma;
  int* cnt = reinterpret_cast<int*>(pw);  // free after the reduction: TRI_GRID counts
  if (tid < TRI_GRID / 2) {
    int c0, c1;
    sturm2(D, DL2, K, tri_grid(T0, 2 * tid), tri_grid(T0, 2 * tid + 1), c0, c1);
    cnt[2 * tid] = c0;
    cnt[2 * tid + 1] = c1;
  }
  __syncthreads();
  {
    const int i = tid >> 2, qd = tid & 3;
    double a = 0.0, b = 0.0;
    bool done = i >= K;   // the second half of the workgroup has no eigenvalue
    if (!done) {
      if (cnt[0] > i) {
        b = tri_grid(T0, 0);  // below 2^-60 ||T||: zero for every use here
        done = true;
      } else if (cnt[TRI_GRID - 1] <= i) {
        a = tri_grid(T0, TRI_GRID - 1);
        b = 2.0 * T0;
      } else {
        int lo = 0, hi = TRI_GRID - 1;  // cnt[lo] <= i < cnt[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (cnt[mid] > i) hi = mid; else lo = mid;
        }
        a = tri_grid(T0, lo);
        b = tri_grid(T0, hi);
      }
    }
    int iters = 0;
    while (!done) {
      const int k0 = 2 * qd + 1;
      int c0, c1;
      sturm2(D, DL2, K, tri_split(a, b, k0), tri_split(a, b, k0 + 1), c0, c1);
      int kf = c0 > i ? k0 : (c1 > i ? k0 + 1 : TRI_SEC);
      kf = quad_min(kf);
      const double na = tri_split(a, b, kf - 1), nb = tri_split(a, b, kf);
      a = na;
      b = nb;
      done = (b - a) <= 0x1p-46 * b || ++iters >= 64;
    }
    if (i < K && qd == 0) lam[i] = 0.5 * (a + b);
  }
  __syncthreads();
  // ---- 4. eigenvectors by twisted factorisations (lane i of wave 0), Z in A
  if (tid == 0) red[15] = 0.0;
  if (wave == 0 && lane < K) {
    const int i = lane;
    const double lm = lam[i];
    double* z = A + TRI_LD * i;
    double s = -lm;
#pragma unroll 8
    for (int k = 0; k + 1 < K; ++k) {
      z[k] = s;                                  // s_k, kept for gamma
      double dp = D[k] + s;
      if (dp == 0.0) dp = -kTiny;
      const double lpk = D[k] * L[k] * recip(dp);
      Lp[64 * k + i] = lpk;
      s = lpk * L[k] * s - lm;
    }
    z[K - 1] = s;
    double p = D[K - 1] - lm;
    int r = K - 1;
    double gmin = fabs(s + p + lm);
#pragma unroll 8
    for (int k = K - 2; k >= 0; --k) {
      double dm = DL2[k] + p;
      if (dm == 0.0) dm = -kTiny;
      const double t = D[k] * recip(dm);
      Um[64 * k + i] = L[k] * t;
      p = p * t - lm;
      const double g = fabs(z[k] + p + lm);
      if (g < gmin) { gmin = g; r = k; }
    }
    double zz = 1.0, nrm = 1.0;
    z[r] = 1.0;
    for (int k = r - 1; k >= 0; --k) {
      zz = -Lp[64 * k + i] * zz;
      z[k] = zz;
      nrm += zz * zz;
    }
    zz = 1.0;
    for (int k = r; k + 1 < K; ++k) {
      zz = -Um[64 * k + i] * zz;
      z[k + 1] = zz;
      nrm += zz * zz;
    }
    const double sc = 1.0 / sqrt(nrm);
    for (int k = 0; k < K; ++k) z[k] *= sc;
    if (!isfinite(sc) || !(sc > 0.0)) red[15] = 1.0;   // a vector the recurrences could not form
  }
  __syncthreads();
  // ---- 5. orthogonality of the kept eigenvectors (indices K - q .. K - 1).  Twisted-factorisation
  // vectors of an L D L^T whose eigenvalues are resolved to relative width 2^-46 differ from exact
  // ones by about K eps / relgap, so pairs whose eigenvalues differ by more than 1 % are orthogonal to
  // far below the tolerance; the other pairs are checked by dot products (and every vector was
  // normalised, non-finite ones flagged).
  const double cut = J.ctol * tr;
  int q = 0;
  for (int i = 0; i < K; ++i) q += (lam[i] - sigma > cut) ? 1 : 0;
  const int i0 = K - q;
  {
    double dev = red[15];
    for (int e = tid; e < q * q; e += TRI_NT) {
      const int ia = i0 + e % q, ib = i0 + e / q;
      if (ia >= ib) continue;
      const double la = lam[ia], lb = lam[ib];
      if (fabs(la - lb) > 0.01 * fmax(la, lb)) continue;
      double g = 0.0;
      for (int k = 0; k < K; ++k) g += A[k + TRI_LD * ia] * A[k + TRI_LD * ib];
      dev = fmax(dev, g != g ? 1.0 : fabs(g));
    }
    dev = wave_max_f64(dev);
    if (lane == 0) red[4 + wave] = dev;
  }
  __syncthreads();
  double dev = 0.0;
  for (int c = 0; c < TRI_NW; ++c) dev = fmax(dev, red[4 + c]);
  if (!(dev <= J.jtol)) {
    if (tid == 0) *J.q = -1;
    return;
  }
  // ---- 6. V = Q Z, column o = eigenvector K - 1 - o
  if (tid < 256) {
    double acc[4][4];
    tri_mm44<false>(Q, A, K, acc);
    const int r0 = 4 * (tid % 16), c0 = 4 * (tid / 16);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = r0 + a, i = c0 + b;
        if (r < K && i < K) {
          const int o = K - 1 - i;
          J.v[r + (long)K * o] = o < q ? acc[a][b] : 0.0;
        }
      }
  }
  for (int o = tid; o < K; o += TRI_NT) J.w[o] = o < q ? lam[K - 1 - o] - sigma : 0.0;
  if (tid == 0) {
    double rest = 0.0;
    for (int i = 0; i < i0; ++i) rest += fmax(lam[i] - sigma, 0.0);
    *J.q = q;
    *J.rest = rest;
  }
}

hipError_t psd_tri_batched(const JobBatch<PsdJob>& jobs_dev, int count, int Kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kBatchJobs || Kmax > kTriMax) return hipErrorInvalidValue;
  const size_t shm = sizeof(double) * ((size_t)2 * kTriMax * TRI_LD + 2 * kTriMax * 64 + 6 * kTriMax + 4 * TRI_NW * 64 + 64 + 16);
  return launch_gram<true, TRI_NT>(k_psd_tri, jobs_dev, count, shm, s);
}

hipError_t syev_batched(const JobBatch<EigJob>& jobs_dev, int count, int Kmax, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kBatchJobs) return hipErrorInvalidValue;
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

// blockIdx.y is the job; the workgroups of a job stride over its elements
template <typename TI, typename TO>
__global__ void k_convert_batch(ConvBatch<TI, TO> b) {
  const int j = blockIdx.y;
  const long cnt = b.count[j];
  const TI* in = b.in[j];
  TO* out = b.out[j];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (long)gridDim.x * blockDim.x)
    out[i] = (TO)in[i];
}
template <typename TI, typename TO>
hipError_t convert_batch(const ConvBatch<TI, TO>& b, hipStream_t s) {
  if (b.n < 1 || b.n > kConvJobs) return b.n == 0 ? hipSuccess : hipErrorInvalidValue;
  long mx = 0;
  for (int j = 0; j < b.n; ++j) mx = std::max(mx, b.count[j]);
  if (mx <= 0) return hipSuccess;
  const long blocks = std::min<long>((mx + 255) / 256, 2048);
  hipLaunchKernelGGL((k_convert_batch<TI, TO>), dim3((unsigned)blocks, b.n), dim3(256), 0, s, b);
  return hipGetLastError();
}
template hipError_t convert_batch<double, float>(const ConvBatch<double, float>&, hipStream_t);
template hipError_t convert_batch<float, double>(const ConvBatch<float, double>&, hipStream_t);
template hipError_t convert_batch<double, double>(const ConvBatch<double, double>&, hipStream_t);
template hipError_t convert_batch<float, float>(const ConvBatch<float, float>&, hipStream_t);

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

template <typename T>
__global__ void k_scale_cols_copy(const T* in, int rows, int cols, const double* w, T* out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  out[e] = (T)((double)in[e] * w[e / rows]);
}
template <typename T>
hipError_t scale_cols_copy(const T* in, int rows, int cols, const double* w, T* out, hipStream_t s) {
  const long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_scale_cols_copy<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, rows, cols, w, out);
  return hipGetLastError();
}
template hipError_t scale_cols_copy<float>(const float*, int, int, const double*, float*, hipStream_t);
template hipError_t scale_cols_copy<double>(const double*, int, int, const double*, double*, hipStream_t);

template <typename T>
__global__ void k_scale_cols_copy_batch(ScaleBatch<T> b) {
  const int j = blockIdx.y;
  const int rows = b.rows[j];
  const long tot = (long)rows * b.cols[j];
  const T* in = b.in[j];
  T* out = b.out[j];
  const double* w = b.w[j];
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
    out[e] = (T)((double)in[e] * w[e / rows]);
}
template <typename T>
hipError_t scale_cols_copy_batch(const ScaleBatch<T>& b, hipStream_t s) {
  if (b.count <= 0 || b.count > 3) return b.count == 0 ? hipSuccess : hipErrorInvalidValue;
  long mx = 0;
  for (int j = 0; j < b.count; ++j) mx = std::max(mx, (long)b.rows[j] * b.cols[j]);
  if (mx <= 0) return hipSuccess;
  const long blocks = std::min<long>((mx + 255) / 256, 1024);
  hipLaunchKernelGGL((k_scale_cols_copy_batch<T>), dim3((unsigned)blocks, b.count), dim3(256), 0, s, b);
  return hipGetLastError();
}
template hipError_t scale_cols_copy_batch<float>(const ScaleBatch<float>&, hipStream_t);
template hipError_t scale_cols_copy_batch<double>(const ScaleBatch<double>&, hipStream_t);

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

// <a, b> accumulated in double: up to 256 workgroups write partial sums to `part`, a
// single workgroup adds them (fixed order, so the result does not depend on timing).
template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* a, const T* b, long count, double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256)
    acc += (double)a[i] * (double)b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void k_sum(const double* part, int cnt, double* out) {
  __shared__ double red[256];
  red[threadIdx.x] = (int)threadIdx.x < cnt ? part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}
template <typename T>
hipError_t dot(const T* a, const T* b, long count, double* out, double* part, hipStream_t s) {
  int nb = (int)std::min<long>(256, std::max<long>(1, (count + 2047) / 2048));
  if (nb == 1) {
    hipLaunchKernelGGL(k_dot<T>, dim3(1), dim3(256), 0, s, a, b, count, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_dot<T>, dim3(nb), dim3(256), 0, s, a, b, count, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, (const double*)part, nb, out);
  return hipGetLastError();
}
template hipError_t dot<double>(const double*, const double*, long, double*, double*, hipStream_t);
template hipError_t dot<float>(const float*, const float*, long, double*, double*, hipStream_t);

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
    const int r = rows[p];  // the factor has ld = n rows: indices outside give NaN, no read
    out[e] = (r >= 0 && r < ld) ? (double)in[r + (long)ld * c] : __longlong_as_double(0x7ff8000000000000LL);
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
__global__ void k_lambda(int n, double power, double* out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    double h = 1.0 / (double)(n + 1);
    double s = sinpi(0.5 * (double)(k + 1) * h);
    double lam = 4.0 / (h * h) * s * s;
    out[k] = power == 1.0 ? lam : pow(lam, power);
  }
}
hipError_t lambda_1d(int n, double* out, hipStream_t s, double power) {
  hipLaunchKernelGGL(k_lambda, dim3((n + 255) / 256), dim3(256), 0, s, n, power, out);
  return hipGetLastError();
}
__global__ void k_lambda_batch(LamBatch b) {
  const int j = blockIdx.y, n = b.n[j];
  const double power = b.power[j];
  double* out = b.out[j];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double h = 1.0 / (double)(n + 1);
    const double sv = sinpi(0.5 * (double)(k + 1) * h);
    const double lam = 4.0 / (h * h) * sv * sv;
    out[k] = power == 1.0 ? lam : pow(lam, power);
  }
}
hipError_t lambda_batch(const LamBatch& b, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  int mx = 0;
  for (int j = 0; j < b.count; ++j) mx = std::max(mx, b.n[j]);
  if (mx <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lambda_batch, dim3((unsigned)std::min(128, (mx + 255) / 256), b.count), dim3(256), 0, s, b);
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

// blockIdx.y is the job; the workgroups of a job stride over its n x K elements
template <typename T>
__global__ void k_expfactors_batch(ExpBatch<T> b) {
  const ExpJob<T>& J = b.j[blockIdx.y];
  const long tot = (long)J.n * J.K;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % J.n), k = (int)(e / J.n);
    const double v = exp(-J.tau[k] * J.lam[i]);
    J.E[i + (long)J.ldE * k] = (T)(J.withLam ? J.lam[i] * v : v);
  }
}
template <typename T>
hipError_t expfactors_batch(const ExpBatch<T>& b, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  long mx = 0;
  for (int j = 0; j < b.count; ++j) mx = std::max(mx, (long)b.j[j].n * b.j[j].K);
  if (mx <= 0) return hipSuccess;
  const long blocks = std::min<long>((mx + 255) / 256, 1024);
  hipLaunchKernelGGL(k_expfactors_batch<T>, dim3((unsigned)blocks, b.count), dim3(256), 0, s, b);
  return hipGetLastError();
}
template hipError_t expfactors_batch<double>(const ExpBatch<double>&, hipStream_t);
template hipError_t expfactors_batch<float>(const ExpBatch<float>&, hipStream_t);

// target function of the fits, in the scaled variable y = rho/rho0:
//   kind 0: g(y) = c_neg rho^-(1+alpha) + c_pos rho^-(1-alpha), rho = rho0*y
//   kind 1: p(y) = 1/s(rho) = 1/(c_neg rho^-alpha + c_pos rho^alpha)
//   kind 2: c_neg rho^-alpha (the state operator beta A^-alpha)
__device__ double fit_target(int kind, const SymFn& f, double rho0, double y) {
  const double rho = rho0 * y;
  const double neg = f.cn > 0.0 ? f.cn * pow(rho, -f.alpha) : 0.0;
  const double pos = f.cp > 0.0 ? f.cp * pow(rho, f.beta) : 0.0;
  if (kind == 0) return (neg + (f.fitpos ? pos : 0.0)) / rho;
  if (kind == 2) return neg;
  return 1.0 / (f.c0 + neg + pos);
}

__global__ void k_fit_design(int kind, SymFn f, double rho0, double B, int K, int m, const FitCand* cands, double* A,
                             double* tvec) {
  int c = blockIdx.y;
  FitCand fc = cands[c];
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  // exponents geometric on [exp(lo), exp(hi)]; a single exponent sits at the middle of the range
  double lo = log(1.0 / B) + fc.a, hi = fc.b;
  auto pos = [K](int k) { return K > 1 ? (double)k / (double)(K - 1) : 0.5; };
  if (e < K) {
    double t = exp(lo + (hi - lo) * pos((int)e));
    tvec[(long)c * K + e] = t;
  }
  if (e < (long)m * K) {
    int j = (int)(e % m), k = (int)(e / m);
    double t = exp(lo + (hi - lo) * pos(k));
    double y = exp(log(B) * (double)j / (double)(m > 1 ? m - 1 : 1));
    A[(long)c * m * K + e] = exp(-t * y) / fit_target(kind, f, rho0, y);
  }
}
hipError_t fit_design(int kind, const SymFn& f, double rho0, double B, int K, int m, const FitCand* cands_dev,
                      int ncand, double* A, double* tvec, hipStream_t s) {
  long tot = (long)m * K;
  hipLaunchKernelGGL(k_fit_design, dim3((tot + 255) / 256, ncand), dim3(256), 0, s, kind, f, rho0, B, K, m, cands_dev,
                     A, tvec);
  return hipGetLastError();
}

// kFitSplit workgroups share the points of a candidate; each writes its maximum to part and a
// second kernel takes the maximum of those per candidate.
constexpr int kFitSplit = 16;
__global__ __launch_bounds__(256) void k_fit_error(int kind, SymFn f, double rho0, double B, int K, const double* t,
                                                   const double* w, int m, double* part) {
  __shared__ double red[256];
  const int c = blockIdx.x / kFitSplit, sub = blockIdx.x % kFitSplit;
  const double* tc = t + (long)c * K;
  const double* wc = w + (long)c * K;
  double mx = 0.0;
  for (int j = sub * 256 + threadIdx.x; j < m; j += 256 * kFitSplit) {
    double y = exp(log(B) * (double)j / (double)(m - 1));
    double v = 0.0;
    for (int k = 0; k < K; ++k) v += wc[k] * exp(-tc[k] * y);
    double r = fabs(v / fit_target(kind, f, rho0, y) - 1.0);
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
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_fit_error_max(int ncand, const double* part, double* err) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncand) return;
  double mx = part[(long)c * kFitSplit];
  for (int i = 1; i < kFitSplit; ++i) {
    const double a = part[(long)c * kFitSplit + i];
    mx = (mx >= a || isnan(mx)) ? mx : a;
  }
  err[c] = mx;
}
hipError_t fit_error(int kind, const SymFn& f, double rho0, double B, int K, const double* t, const double* w,
                     int ncand, int m, double* err, double* part, hipStream_t s) {
  if (ncand <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fit_error, dim3(ncand * kFitSplit), dim3(256), 0, s, kind, f, rho0, B, K, t, w, m, part);
  hipLaunchKernelGGL(k_fit_error_max, dim3((ncand + 255) / 256), dim3(256), 0, s, ncand, (const double*)part, err);
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
// Multi-indices outside the grid give NaN (no read outside the eigenvalue arrays).
__device__ inline bool idx_ok(const int* ix, int d, int n0, int n1, int n2) {
  return ix[0] >= 0 && ix[0] < n0 && ix[1] >= 0 && ix[1] < n1 && (d < 3 || (ix[2] >= 0 && ix[2] < n2));
}

__global__ void k_symbol_eval(int d, const int* idx, int count, int n0, int n1, int n2, const double* l0,
                              const double* l1, const double* l2, int opkind, int K, const double* tau,
                              const double* w, double c0, double* out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const int* ix = idx + (long)p * d;
  if (!idx_ok(ix, d, n0, n1, n2)) { out[p] = __longlong_as_double(0x7ff8000000000000LL); return; }
  double rho = l0[ix[0]] + l1[ix[1]];
  if (d == 3) rho += l2[ix[2]];
  double v = 0.0;
  for (int k = 0; k < K; ++k) v += w[k] * exp(-tau[k] * rho);
  out[p] = opkind == 0 ? c0 + rho * v : v;
}
hipError_t symbol_eval(int d, const int* idx, int count, const int* n, const double* lam0, const double* lam1,
                       const double* lam2, int opkind, int K, const double* tau, const double* w, double c0,
                       double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_symbol_eval, dim3((count + 255) / 256), dim3(256), 0, s, d, idx, count, n[0], n[1],
                     d == 3 ? n[2] : 1, lam0, lam1, lam2, opkind, K, tau, w, c0, out);
  return hipGetLastError();
}

template <typename T>
__global__ void k_cp_eval(int d, const int* idx, int count, int n0, int n1, int n2, const T* F0, const T* F1,
                          const T* F2, int R, const double* w, double* out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const int* ix = idx + (long)p * d;
  if (!idx_ok(ix, d, n0, n1, n2)) { out[p] = __longlong_as_double(0x7ff8000000000000LL); return; }
  double v = 0.0;
  for (int k = 0; k < R; ++k) {
    double t = w[k] * (double)F0[ix[0] + (long)n0 * k] * (double)F1[ix[1] + (long)n1 * k];
    if (d == 3) t *= (double)F2[ix[2] + (long)n2 * k];
    v += t;
  }
  out[p] = v;
}
template <typename T>
hipError_t cp_eval(int d, const int* idx, int count, const int* n, const T* const* F, int R, const double* w,
                   double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cp_eval<T>, dim3((count + 255) / 256), dim3(256), 0, s, d, idx, count, n[0], n[1],
                     d == 3 ? n[2] : 1, F[0], F[1], d == 3 ? F[2] : F[1], R, w, out);
  return hipGetLastError();
}
template hipError_t cp_eval<float>(int, const int*, int, const int*, const float* const*, int, const double*,
                                   double*, hipStream_t);
template hipError_t cp_eval<double>(int, const int*, int, const int*, const double* const*, int, const double*,
                                    double*, hipStream_t);

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
