// Complete-data path on matrix cores.
//
// When the input and output samples are each the full drug x target grid in
// the natural pair order (Section 4 Example), R(d,t) = I and the Kronecker
// product acts on vec(Vmat) as (M (x) N) vec(Vmat) = vec(M Vmat N^T) (row-major
// vec).  That is two dense GEMMs, W = M Vmat and Umat = W N^T, run here with
// MFMA tiles:
//   F64    v_mfma_f64_16x16x4f64
//   F32    v_mfma_f32_16x16x4f32
//   BF16X3 v_mfma_f32_16x16x32_bf16 on split operands x = hi + lo (bf16, RNE),
//          product ~ hi*hi' + hi*lo' + lo*hi' accumulated in FP32.  The
//          operands are split once in a bandwidth-bound pass; the first GEMM
//          writes W already split for the second.
//   BF16X6 the same with a three-way split x = hi + mid + lo and the six
//          products down to the FP32 rounding level.
//
// FP64/FP32 tiling: 256 threads (2 x 2 waves), block tile 128 x 128, each wave
// owns a 64 x 64 sub-tile (4 x 4 MFMA blocks of 16 x 16), global tiles
// prefetched into registers while the current LDS tile feeds the MFMAs.  The
// bf16x3 product has its own kernel (256 x 128 tiles, operands copied straight
// into a three-stage LDS ring); bf16x6 keeps the 128 x 128 split kernel.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace gvt {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// C[M x N] = A[M x K] * op(B),  op(B)[k][n] = BT ? B[n*ldb + k] : B[k*ldb + n]
template <class T, bool BT>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const T *__restrict__ A, int64_t lda,
                                                        const T *__restrict__ B, int64_t ldb,
                                                        T *__restrict__ C, int64_t ldc, int64_t M,
                                                        int64_t N, int64_t K,
    int64_t kchunk, int64_t cz) {
  // split-K: block z sums k in [z kchunk, min(K, (z + 1) kchunk)) into C + z cz
  {
    const int64_t kz0 = (int64_t)blockIdx.z * kchunk;
    A += kz0;
    B += BT ? kz0 : kz0 * ldb;
    K = K - kz0 < kchunk ? K - kz0 : kchunk;
    C += (int64_t)blockIdx.z * cz;
  }
  constexpr int BM = 128, BN = 128, BK = 16, PAD = 4;
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;

  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);

  // A tile (BM x BK, k contiguous in global): thread -> row tid/2, 8 k's at (tid&1)*8
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  // B tile: NT like A (rows = n); NN: k-row tid/16, 8 n's at (tid%16)*8
  const int br = BT ? (tid >> 1) : (tid >> 4);
  const int bc = BT ? ((tid & 1) * 8) : ((tid & 15) * 8);
  T ra[8], rb[8];

  auto load_tiles = [&](int64_t k0) {
    const int64_t gm = m0 + ar;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t gk = k0 + ak + u;
      ra[u] = (gm < M && gk < K) ? A[gm * lda + gk] : T(0);
    }
    if (BT) {
      const int64_t gn = n0 + br;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t gk = k0 + bc + u;
        rb[u] = (gn < N && gk < K) ? B[gn * ldb + gk] : T(0);
      }
    } else {
      const int64_t gk = k0 + br;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t gn = n0 + bc + u;
        rb[u] = (gk < K && gn < N) ? B[gk * ldb + gn] : T(0);
      }
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int u = 0; u < 8; ++u) As[ak + u][ar] = ra[u];
    if (BT) {
#pragma unroll
      for (int u = 0; u < 8; ++u) Bs[bc + u][br] = rb[u];
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) Bs[br][bc + u] = rb[u];
    }
  };

  load_tiles(0);
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    store_tiles();
    __syncthreads();
    if (k0 + BK < K) load_tiles(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T af[4], bf[4];
      const int kr = kk + (lane >> 4), cl = lane & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[kr][wm * 64 + i * 16 + cl];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[kr][wn * 64 + j * 16 + cl];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::op(af[i], bf[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + Mfma<T>::row(lane, v);
        if (row < M && col < N) C[row * ldc + col] = acc[i][j][v];
      }
    }
}

// MFMA GEMM with 16-byte loads (rows 16-byte aligned, K and N multiples of the
// vector length): C[M x N] = A[M x K] * op(B), op(B)[k][n] = BT ? B[n*ldb + k]
// : B[k*ldb + n].  A (and B^T) tiles are stored row-major along k with a row
// stride of BK + 16 bytes, which keeps both the 16-byte stores and the MFMA
// operand reads (16 rows at one k, four k's per wave) free of bank conflicts;
// a row-major B tile keeps n contiguous.  k steps of 32 (FP32) or 16 (FP64)
// elements, the next step prefetched into registers.
template <class T, bool BT>
__global__ __launch_bounds__(256) void gemm_vec_kernel(const T *__restrict__ A, int64_t lda,
                                                       const T *__restrict__ B, int64_t ldb,
                                                       T *__restrict__ C, int64_t ldc, int64_t M,
                                                       int64_t N, int64_t K,
    int64_t kchunk, int64_t cz) {
  // split-K: block z sums k in [z kchunk, min(K, (z + 1) kchunk)) into C + z cz
  {
    const int64_t kz0 = (int64_t)blockIdx.z * kchunk;
    A += kz0;
    B += BT ? kz0 : kz0 * ldb;
    K = K - kz0 < kchunk ? K - kz0 : kchunk;
    C += (int64_t)blockIdx.z * cz;
  }
  constexpr int VEC = 16 / sizeof(T);            // elements per 16-byte vector
  constexpr int BM = 128, BN = 128, BK = sizeof(T) == 4 ? 32 : 16;
  constexpr int AS = BK + VEC;                   // row stride: k step + 16 bytes
  constexpr int KPT = BK / 2, NV = KPT / VEC;    // elements / vectors per thread and operand
  constexpr int TPR = 256 / BK;                  // threads per k-row of a row-major B tile
  typedef T vt __attribute__((ext_vector_type(VEC)));
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ __attribute__((aligned(16))) T As[BM][AS];
  __shared__ __attribute__((aligned(16))) T Bs[BT ? BN : BK][BT ? AS : BN + VEC];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);
  // A (and B^T): thread -> row tid/2, KPT k's at (tid&1)*KPT
  const int ar = tid >> 1, ak = (tid & 1) * KPT;
  // row-major B: thread -> k-row tid/TPR, KPT n's at (tid%TPR)*KPT
  const int bk = tid / TPR, bn = (tid % TPR) * KPT;
  const bool arow = m0 + ar < M;
  const bool brow = BT ? (n0 + ar < N) : true;
  const unsigned am = arow ? 0xffffffffu : 0u, bm = brow ? 0xffffffffu : 0u;
  // row starts (row 0 stands in for rows past the edge); every fallback address is a
  // row start, valid because the vector path needs K >= VEC
  const T *ag = A + (arow ? (m0 + ar) * lda : 0);
  const T *bg = BT ? B + (brow ? (n0 + ar) * ldb : 0) : B;
  vt pa[NV], pb[NV];
  auto masked = [](vt v, unsigned mk) {
    return __builtin_bit_cast(vt, __builtin_bit_cast(uint4, v) & uint4{mk, mk, mk, mk});
  };
  auto load = [&](int64_t k0) {
    // rows past the edge and vectors past K are zeroed by a mask (not a select of
    // addresses); K is a multiple of VEC, so a vector is wholly inside or outside
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const bool kin = k0 + ak + VEC * u < K;
      pa[u] = masked(*reinterpret_cast<const vt *>(ag + (kin ? k0 + ak + VEC * u : 0)), kin ? am : 0u);
    }
    if (BT) {
#pragma unroll
      for (int u = 0; u < NV; ++u) {
        const bool kin = k0 + ak + VEC * u < K;
        pb[u] = masked(*reinterpret_cast<const vt *>(bg + (kin ? k0 + ak + VEC * u : 0)), kin ? bm : 0u);
      }
    } else {
      const int64_t gk = k0 + bk;
#pragma unroll
      for (int u = 0; u < NV; ++u) {
        const int64_t gn = n0 + bn + VEC * u;
        const bool ok = gk < K && gn < N;  // N is a multiple of VEC
        pb[u] = masked(*reinterpret_cast<const vt *>(B + (ok ? gk * ldb + gn : 0)), ok ? 0xffffffffu : 0u);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NV; ++u) *reinterpret_cast<vt *>(&As[ar][ak + VEC * u]) = pa[u];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      if (BT) *reinterpret_cast<vt *>(&Bs[ar][ak + VEC * u]) = pb[u];
      else *reinterpret_cast<vt *>(&Bs[bk][bn + VEC * u]) = pb[u];
    }
  };
  const int64_t kend = (K + BK - 1) / BK * BK;
  load(0);
  for (int64_t k0 = 0; k0 < kend; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4), cl = lane & 15;
      T af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[wm * 64 + i * 16 + cl][kr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = BT ? Bs[wn * 64 + j * 16 + cl][kr] : Bs[kr][wn * 64 + j * 16 + cl];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::op(af[i], bf[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + Mfma<T>::row(lane, v);
        if (row < M && col < N) C[row * ldc + col] = acc[i][j][v];
      }
    }
}

// ---- split-bf16 products ------------------------------------------------------
__device__ __forceinline__ unsigned short bf16_rne_bits(float x) {
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}
// x = s[0] + s[1] (+ s[2]) with each part the round-to-nearest-even bf16 of the
// remaining residual (the residuals are exact in FP32).
template <int NS>
__device__ __forceinline__ void split_bf16(float x, unsigned short (&s)[NS]) {
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    s[k] = bf16_rne_bits(x);
    x = x - bf16_bits_to_float(s[k]);
  }
}

// ---- operand splitting (one bandwidth-bound pass per operand) ---------------
// Where piece k of element (r, c) of a split operand with cols_pad columns
// (a multiple of 32) is stored.  Three pieces: one plane per piece,
// k*ps + r*cols_pad + c.  Two pieces: the planes interleaved per 32-column
// block, r*2*cols_pad + (c/32)*64 + 32k + c%32, so that the hi and lo halves
// of a 32-wide k step of a row are one contiguous 128-byte line.
template <int NS>
__device__ __forceinline__ int64_t piece_at(int k, int64_t r, int64_t c, int64_t cols_pad, int64_t ps) {
  if (NS == 2) return r * 2 * cols_pad + (c >> 5) * 64 + 32 * k + (c & 31);
  return k * ps + r * cols_pad + c;
}

// Piece k of X[r][c] for c < cols, 0 for cols <= c < cols_pad, at
// piece_at(k, r, c).  Four columns per thread.
template <int NS>
__global__ void split_rows_kernel(const float *__restrict__ X, int64_t ldx, int64_t rows,
                                  int64_t cols, int64_t cols_pad, unsigned short *__restrict__ P,
                                  int64_t ps) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t qpr = cols_pad / 4;
  if (q >= rows * qpr) return;
  const int64_t r = q / qpr, c0 = (q - r * qpr) * 4;
  unsigned short sp[4][NS];
#pragma unroll
  for (int u = 0; u < 4; ++u) split_bf16<NS>(c0 + u < cols ? X[r * ldx + c0 + u] : 0.f, sp[u]);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    typedef unsigned short us4 __attribute__((ext_vector_type(4)));
    us4 v = {sp[0][k], sp[1][k], sp[2][k], sp[3][k]};
    *reinterpret_cast<us4 *>(P + piece_at<NS>(k, r, c0, cols_pad, ps)) = v;
  }
}

// Piece k of X[r][c] (X: rows x cols) at piece_at(k, c, r) with rows_pad
// columns, 0 for rows <= r < rows_pad: the transposed split, through 32 x 32
// LDS tiles.
template <int NS>
__global__ __launch_bounds__(256) void split_transpose_kernel(const float *__restrict__ X, int64_t ldx,
                                                              int64_t rows, int64_t cols,
                                                              int64_t rows_pad,
                                                              unsigned short *__restrict__ P,
                                                              int64_t ps) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + j, c = c0 + tx;
    tile[j][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.f;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t c = c0 + j, r = r0 + tx;  // output row c, column r
    if (c < cols && r < rows_pad) {
      unsigned short sp[NS];
      split_bf16<NS>(tile[tx][j], sp);
#pragma unroll
      for (int k = 0; k < NS; ++k) P[piece_at<NS>(k, c, r, rows_pad, ps)] = sp[k];
    }
  }
}

// Split-operand GEMM on bf16 MFMA with FP32 accumulation, on operands split
// beforehand into three planes (piece_at<3>): C[M x N] = sum of the kept
// piece products of A (M x Kp) and B (N x Kp), both row-major along k with Kp
// a multiple of 32 (zero-padded).  NS = 3 keeps every product whose order is
// at most the FP32 rounding level: hh + hm + mh + hl + lh + mm (bf16x6).
// SPLIT_OUT writes C as NS split pieces (row stride ldcs, piece stride cps,
// columns up to ncols_pad, the padding being exact zeros) for a following
// GEMM; otherwise C is FP32.  Block tile 128 x 128, each wave 64 x 64; each
// thread prefetches the next k step of every piece with 16-byte loads while
// the MFMAs consume the LDS tile.
template <int NS, bool SPLIT_OUT, int BK>
__global__ __launch_bounds__(256) void gemm_bf16p_kernel(
    const unsigned short *__restrict__ A, int64_t lda, int64_t aps,
    const unsigned short *__restrict__ B, int64_t ldb, int64_t bps, float *__restrict__ C,
    int64_t ldc, unsigned short *__restrict__ Cs, int64_t ldcs, int64_t cps, int64_t ncols_pad,
    int64_t M, int64_t N, int64_t Kp) {
  constexpr int BM = 128, BN = 128, PK = BK + 8, WPR = BK / 16;  // 16-byte words per thread-row
  static_assert(BK % 32 == 0, "k step: whole MFMA k blocks");
  __shared__ __attribute__((aligned(16))) unsigned short As[NS][BM][PK];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[NS][BN][PK];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // global -> LDS: thread -> tile row tid/2, 16 k's (two 16-byte words) at
  // (tid&1)*16.  Rows past M (N) read row 0 and are stored as zeros.
  const int lr = tid >> 1, lk = (tid & 1) * (BK / 2);
  const bool arow = m0 + lr < M, brow = n0 + lr < N;
  const unsigned short *ag = A + (arow ? (m0 + lr) * lda : 0) + lk;
  const unsigned short *bg = B + (brow ? (n0 + lr) * ldb : 0) + lk;
  // rows past the edge are zeroed by masking (a select between two vectors
  // would be lowered to a select between their addresses)
  const unsigned am = arow ? 0xffffffffu : 0u, bm = brow ? 0xffffffffu : 0u;
  const uint4 amask = {am, am, am, am}, bmask = {bm, bm, bm, bm};
  uint4 pa[WPR * NS], pb[WPR * NS];
#define GVT_BF16P_LOAD(k0)                                                                   \
  _Pragma("unroll") for (int k = 0; k < NS; ++k) {                                           \
    const uint4 *sa = reinterpret_cast<const uint4 *>(ag + k * aps + (k0));                  \
    const uint4 *sb = reinterpret_cast<const uint4 *>(bg + k * bps + (k0));                  \
    _Pragma("unroll") for (int w = 0; w < WPR; ++w) {                                        \
      pa[WPR * k + w] = sa[w] & amask;                                                       \
      pb[WPR * k + w] = sb[w] & bmask;                                                       \
    }                                                                                        \
  }
  auto frag = [&](const unsigned short(&X)[BM][PK], int row, int kofs) {
    return __builtin_bit_cast(bf8, *reinterpret_cast<const us8 *>(&X[row][kofs]));
  };
  GVT_BF16P_LOAD(0)
  for (int64_t k0 = 0; k0 < Kp; k0 += BK) {
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int w = 0; w < WPR; ++w) {
        *reinterpret_cast<uint4 *>(&As[k][lr][lk + 8 * w]) = pa[WPR * k + w];
        *reinterpret_cast<uint4 *>(&Bs[k][lr][lk + 8 * w]) = pb[WPR * k + w];
      }
    __syncthreads();
    if (k0 + BK < Kp) {
      GVT_BF16P_LOAD(k0 + BK)
    }
#pragma unroll
    for (int kb = 0; kb < BK; kb += 32) {
    const int kofs = kb + 8 * (lane >> 4), rl = lane & 15;
    bf8 af[NS][4], bfr[NS][4];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        af[k][i] = frag(As[k], wm * 64 + i * 16 + rl, kofs);
        bfr[k][i] = frag(Bs[k], wn * 64 + i * 16 + rl, kofs);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // The correction products of this k-step are summed from zero, then
        // added to the running hi*hi sum with one FP32 add: accumulating them
        // straight into the large running sum loses their low bits.
        f4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[0][j], f4{0.f, 0.f, 0.f, 0.f},
                                                       0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[1][j], c, 0, 0, 0);
        if (NS == 3) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[1][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bfr[0][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[2][j], c, 0, 0, 0);
        }
        f4 h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[0][j], acc[i][j], 0, 0, 0);
        acc[i][j] = h + c;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        if (SPLIT_OUT) {
          if (row < M && col < ncols_pad) {
            unsigned short sp[NS];
            split_bf16<NS>(acc[i][j][v], sp);
#pragma unroll
            for (int k = 0; k < NS; ++k) Cs[k * cps + row * ldcs + col] = sp[k];
          }
        } else if (row < M && col < N) {
          C[row * ldc + col] = acc[i][j][v];
        }
      }
    }
}

// ---- bf16x3 product: large tiles, operands copied straight into LDS --------
// C = Ahi Bhi^T + Ahi Blo^T + Alo Bhi^T on two-piece operands (piece_at<2>,
// Kp a multiple of 32, so a row's k step is one 128-byte line: hi then lo).
// 256 threads (2 x 2 waves), block tile 256 x 128, each wave 128 x 64
// (8 x 4 MFMA blocks of 16 x 16).  The hi*hi products and the two correction
// products go to separate accumulators, updated by MFMAs only (so they stay in
// the accumulation registers) and added once at the end: the corrections are
// summed at their own scale instead of rounding into the large running sum
// three times per k step.
//
// Operand tiles go from global memory straight to LDS (global_load_lds_dwordx4:
// lane l of a wave writes its 16 bytes at the wave's LDS base + 16 l) through
// three LDS stages: the copies of k step kk + 2 are issued among the MFMAs
// of step kk.  One copy instruction moves 8 rows x 128 bytes; lane l takes row
// l / 8 and the 16-byte chunk that the XOR permutation (row bits 0-3) puts at
// position l % 8, which spreads the 16 rows of a fragment read over distinct
// banks.  Each wave waits for its own copies (vmcnt) before the barrier that
// ends a step; the barrier is a bare s_barrier, since a __syncthreads fence
// would also wait for the copies still in flight.  A and B share one LDS
// array: with two, the compiler makes every fragment read wait for all copies.
//
// Workgroups go to the 8 XCDs round-robin by id; ids are remapped so that each
// XCD runs a contiguous run of tiles, taken in groups of 4 tile rows, which
// share operand panels in that XCD's L2.

// s_waitcnt with only the vector-memory count limited (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima), and
// with only the LDS/scalar count at zero
#define GVT_WAIT_VMCNT(n) __builtin_amdgcn_s_waitcnt(((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))
#define GVT_WAIT_LGKMCNT0() __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4))

__device__ __forceinline__ int bf16x3_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

template <bool SPLIT_OUT>
__global__ __launch_bounds__(256, 1) void gemm_bf16x3_kernel(
    const unsigned short *__restrict__ A, const unsigned short *__restrict__ B, float *__restrict__ C,
    int64_t ldc, unsigned short *__restrict__ Cs, int64_t ncols_pad, int64_t M, int64_t N, int64_t Kp,
    int tiles_m, int tiles_n) {
  constexpr int WTM = 8, WTN = 4, BM = 256, BN = 128, NST = 3;
  constexpr int CPA = BM / 32, CPB = BN / 32;  // copy instructions per wave and stage (8 rows each)
  constexpr int NCOPY = CPA + CPB;
  __shared__ u32x4 Ls[NST][BM + BN][8];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int64_t ld = 2 * Kp;  // row stride of both operands

  int t = blockIdx.x;
  const int total = tiles_m * tiles_n;
  if ((total & 7) == 0) t = (t & 7) * (total >> 3) + (t >> 3);
  constexpr int GM = 4;
  const int grp = t / (GM * tiles_n), first = grp * GM, gs = min(tiles_m - first, GM);
  const int tin = t - grp * GM * tiles_n;
  const int64_t m0 = (int64_t)(first + tin % gs) * BM, n0 = (int64_t)(tin / gs) * BN;

  // copy q of this wave fills LDS rows wid*(BM/4) + 8q + lane/8 (A) or
  // BM + wid*(BN/4) + 8q + lane/8 (B); rows past M (N) read row 0 instead
  // (they only reach rows and columns of the tile that are not stored, and
  // padding columns of a split output are written as zeros)
  const int crow = lane >> 3;
  const unsigned short *ap[CPA], *bp[CPB];
#pragma unroll
  for (int q = 0; q < CPA; ++q) {
    const int64_t r = m0 + wid * (BM / 4) + 8 * q + crow;
    const int ch = (lane & 7) ^ bf16x3_swz(8 * (q & 1) + crow);
    ap[q] = A + (r < M ? r * ld : 0) + 8 * ch;
  }
#pragma unroll
  for (int q = 0; q < CPB; ++q) {
    const int64_t r = n0 + wid * (BN / 4) + 8 * q + crow;
    const int ch = (lane & 7) ^ bf16x3_swz(8 * (q & 1) + crow);
    bp[q] = B + (r < N ? r * ld : 0) + 8 * ch;
  }
#define GVT_BF16X3_COPY_A(st, q, kk)                                                              \
  __builtin_amdgcn_global_load_lds((const void *)(ap[q] + 64 * (kk)),                             \
      (__attribute__((address_space(3))) void *)&Ls[st][wid * (BM / 4) + 8 * (q)][0], 16, 0, 0)
#define GVT_BF16X3_COPY_B(st, q, kk)                                                              \
  __builtin_amdgcn_global_load_lds((const void *)(bp[q] + 64 * (kk)),                             \
      (__attribute__((address_space(3))) void *)&Ls[st][BM + wid * (BN / 4) + 8 * (q)][0], 16, 0, 0)
#define GVT_BF16X3_COPY(st, kk)                                                                   \
  _Pragma("unroll") for (int q = 0; q < CPA; ++q) GVT_BF16X3_COPY_A(st, q, kk);                   \
  _Pragma("unroll") for (int q = 0; q < CPB; ++q) GVT_BF16X3_COPY_B(st, q, kk);
  static_assert(CPA == WTM && CPB <= WTM, "one A copy (and at most one B copy) per MFMA group");

  f4 acc[WTM][WTN], cor[WTM][WTN];
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      cor[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // fragment reads: lane -> row lane % 16 of a 16-row block, chunk lane / 16
  // of the piece (chunks 0-3 hi, 4-7 lo)
  const int fr = lane & 15;
  const int fh = (lane >> 4) ^ bf16x3_swz(fr), fl = (4 + (lane >> 4)) ^ bf16x3_swz(fr);
  const int ar0 = wm * 16 * WTM + fr, br0 = BM + wn * 16 * WTN + fr;
  const int64_t nk = Kp / 32;
  if (nk > 0) {
    GVT_BF16X3_COPY(0, 0)
  }
  if (nk > 1) {
    GVT_BF16X3_COPY(1, 1)
    GVT_WAIT_VMCNT(NCOPY);
  } else {
    GVT_WAIT_VMCNT(0);
  }
  __builtin_amdgcn_s_barrier();
  int st = 0;
  for (int64_t kk = 0; kk < nk; ++kk) {
    const bool ahead = kk + 2 < nk;
    const int s2 = st == 0 ? 2 : st - 1;  // (kk + 2) mod 3
    // all of B, then A one 16-row block ahead of its MFMAs (the scheduling
    // barriers keep each block's reads in front of the previous block's
    // MFMAs, so the waits overlap with MFMA execution); the copies of step
    // kk + 2 are spread over the MFMA groups, one A copy (and one B copy in
    // the first CPB groups) each, which keeps the memory pipeline fed evenly
    bf8 bh[WTN], bl[WTN];
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
      bh[j] = __builtin_bit_cast(bf8, Ls[st][br0 + 16 * j][fh]);
      bl[j] = __builtin_bit_cast(bf8, Ls[st][br0 + 16 * j][fl]);
    }
    bf8 ah = __builtin_bit_cast(bf8, Ls[st][ar0][fh]);
    bf8 al = __builtin_bit_cast(bf8, Ls[st][ar0][fl]);
#pragma unroll
    for (int i = 0; i < WTM; ++i) {
      bf8 ahn = ah, aln = al;
      if (i + 1 < WTM) {
        ahn = __builtin_bit_cast(bf8, Ls[st][ar0 + 16 * (i + 1)][fh]);
        aln = __builtin_bit_cast(bf8, Ls[st][ar0 + 16 * (i + 1)][fl]);
      }
      if (ahead) {
        GVT_BF16X3_COPY_A(s2, i, kk + 2);
        if (i < CPB) GVT_BF16X3_COPY_B(s2, i, kk + 2);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < WTN; ++j)
        cor[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], cor[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < WTN; ++j)
        cor[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], cor[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < WTN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      ah = ahn;
      al = aln;
    }
    // this wave's copies of step kk + 1 have landed (those of kk + 2 may
    // still be in flight) and its reads of step kk are done; then the barrier
    if (ahead) {
      GVT_WAIT_VMCNT(NCOPY);
    } else {
      GVT_WAIT_VMCNT(0);
    }
    GVT_WAIT_LGKMCNT0();
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    st = st == 2 ? 0 : st + 1;
  }
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j) {
      const int64_t col = n0 + wn * 16 * WTN + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 16 * WTM + i * 16 + 4 * (lane >> 4) + v;
        const float x = col >= N ? 0.f : acc[i][j][v] + cor[i][j][v];
        if (SPLIT_OUT) {
          if (row < M && col < ncols_pad) {
            unsigned short sp[2];
            split_bf16<2>(x, sp);
            Cs[piece_at<2>(0, row, col, ncols_pad, 0)] = sp[0];
            Cs[piece_at<2>(1, row, col, ncols_pad, 0)] = sp[1];
          }
        } else if (row < M && col < N) {
          C[row * ldc + col] = x;
        }
      }
    }
}
#undef GVT_BF16X3_COPY
#undef GVT_BF16X3_COPY_A
#undef GVT_BF16X3_COPY_B
#undef GVT_WAIT_VMCNT
#undef GVT_WAIT_LGKMCNT0

// C = sum_z P[z] (fixed order), P[z] row-major M x N at z * M * N
template <class T>
__global__ void splitk_sum_kernel(const T *__restrict__ P, int splits, int64_t M, int64_t N, T *__restrict__ C,
                                  int64_t ldc) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M * N) return;
  T acc = P[q];
  for (int z = 1; z < splits; ++z) acc += P[(int64_t)z * M * N + q];
  C[(q / N) * ldc + q % N] = acc;
}

// Number of k splits that brings a launch of M x N output tiles to about two
// workgroups per CU (each split keeps at least 128 k's), and its workspace.
static int gemm_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ceil_div(M, 128) * ceil_div(N, 128);
  if (tiles >= 256) return 1;
  const int64_t want = ceil_div(512, tiles), most = K / 128;
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, std::min<int64_t>(most, 16)));
}
static size_t gemm_splits_bytes(int64_t M, int64_t N, int64_t K, size_t es) {
  const int sp = gemm_splits(M, N, K);
  return sp > 1 ? (size_t)sp * M * N * es : 0;
}

// C[M x N] = A op(B); with too few output tiles for the chip the k range is
// split over a third grid dimension into `part` (gemm_splits_bytes) and summed
// in a fixed order.
template <class T, bool BT>
static void gemm(const T *A, int64_t lda, const T *B, int64_t ldb, T *C, int64_t ldc, int64_t M,
                 int64_t N, int64_t K, T *part, hipStream_t s) {
  constexpr int64_t V = 16 / sizeof(T);
  constexpr int64_t BKV = sizeof(T) == 4 ? 32 : 16;  // k step of the vector kernel
  const int sp = part ? gemm_splits(M, N, K) : 1;
  const int64_t kchunk = sp > 1 ? ceil_div(ceil_div(K, sp), BKV) * BKV : K;
  const int nz = sp > 1 ? (int)ceil_div(K, kchunk) : 1;
  dim3 grid((unsigned)ceil_div(N, 128), (unsigned)ceil_div(M, 128), (unsigned)nz);
  T *Cout = nz > 1 ? part : C;
  const int64_t ldo = nz > 1 ? N : ldc, cz = nz > 1 ? M * N : 0;
  // 16-byte loads need aligned rows and whole vectors along k (and along n for B)
  auto al16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
  if (al16(A) && al16(B) && lda % V == 0 && ldb % V == 0 && K % V == 0 && (BT || N % V == 0))
    gemm_vec_kernel<T, BT><<<grid, 256, 0, s>>>(A, lda, B, ldb, Cout, ldo, M, N, K, kchunk, cz);
  else
    gemm_mfma_kernel<T, BT><<<grid, 256, 0, s>>>(A, lda, B, ldb, Cout, ldo, M, N, K, kchunk, cz);
  if (nz > 1) splitk_sum_kernel<T><<<(unsigned)ceil_div(M * N, 256), 256, 0, s>>>(part, nz, M, N, C, ldc);
}

// Piece layout of the split-bf16 product: M and N split by rows, Vmat
// transposed (k padded to whole k steps of the GEMM), W written as split
// pieces by the first GEMM.  Offsets and the total are in bf16 elements; the
// pieces of one operand are al(size) elements apart, every piece 256-byte
// aligned.
struct SplitLayout {
  int64_t k1, k2, pm, pv, pw, pn, om, ov, ow, on, total;
  static int64_t al(int64_t e) { return (e * 2 + 255) / 256 * 128; }
  SplitLayout(int NS, int64_t mr, int64_t mc, int64_t nr, int64_t nc) {
    const int KQ = 32;  // k padding: whole k steps of the GEMMs
    k1 = ceil_div(mc, KQ) * KQ;
    k2 = ceil_div(nc, KQ) * KQ;
    pm = mr * k1; pv = nc * k1; pw = mr * k2; pn = nr * k2;
    om = 0; ov = om + NS * al(pm); ow = ov + NS * al(pv); on = ow + NS * al(pw);
    total = on + NS * al(pn);
  }
  size_t bytes() const { return (size_t)total * 2 + 256; }
};

// One bf16x3 product: C (M x N) from two-piece operands with Kp k's.
template <bool SPLIT_OUT>
static void launch_bf16x3(const unsigned short *A, const unsigned short *B, float *C, int64_t ldc,
                          unsigned short *Cs, int64_t ncols_pad, int64_t M, int64_t N, int64_t Kp,
                          hipStream_t s) {
  const int64_t tm = ceil_div(M, 256), tn = ceil_div(N, 128);
  if (tm == 0 || tn == 0) return;
  GVT_REQUIRE(tm * tn < (int64_t)1 << 31, GVT_ERR_ARG, "dense product too large for one launch");
  gemm_bf16x3_kernel<SPLIT_OUT><<<(unsigned)(tm * tn), 256, 0, s>>>(A, B, C, ldc, Cs, ncols_pad, M, N, Kp,
                                                                   (int)tm, (int)tn);
}

// Umat = M Vmat N^T with split-bf16 products: split M and N by rows and Vmat
// transposed, W = M Vmat written as split pieces by the first GEMM, then
// Umat = W N^T.  ws: caller workspace of at least SplitLayout::bytes() (null:
// a stream-ordered allocation).
template <int NS>
static void dense_split_bf16(const float *M, int64_t mr, int64_t mc, int64_t ldm, const float *N,
                             int64_t nr, int64_t nc, int64_t ldn, const float *V, int64_t ldv,
                             float *U, int64_t ldu, void *ws, hipStream_t s) {
  const SplitLayout L(NS, mr, mc, nr, nc);
  const int64_t k1 = L.k1, k2 = L.k2;
  auto al = SplitLayout::al;
  void *buf = ws;
  if (!buf) GVT_HIP_CHECK(hipMallocAsync(&buf, L.bytes(), s));
  unsigned short *base = (unsigned short *)buf;
  unsigned short *Ms = base + L.om, *Vt = base + L.ov, *Ws = base + L.ow, *Ns = base + L.on;
  split_rows_kernel<NS><<<(unsigned)ceil_div(mr * (k1 / 4), 256), 256, 0, s>>>(M, ldm, mr, mc, k1, Ms,
                                                                             al(L.pm));
  split_rows_kernel<NS><<<(unsigned)ceil_div(nr * (k2 / 4), 256), 256, 0, s>>>(N, ldn, nr, nc, k2, Ns,
                                                                             al(L.pn));
  split_transpose_kernel<NS><<<dim3((unsigned)ceil_div(k1, 32), (unsigned)ceil_div(nc, 32)), 256, 0, s>>>(
      V, ldv, mc, nc, k1, Vt, al(L.pv));
  if constexpr (NS == 2) {
    launch_bf16x3<true>(Ms, Vt, nullptr, 0, Ws, k2, mr, nc, k1, s);
    launch_bf16x3<false>(Ws, Ns, U, ldu, nullptr, 0, mr, nr, k2, s);
  } else {
    dim3 g1((unsigned)ceil_div(nc, 128), (unsigned)ceil_div(mr, 128));
    gemm_bf16p_kernel<NS, true, 32><<<g1, 256, 0, s>>>(Ms, k1, al(L.pm), Vt, k1, al(L.pv), nullptr, 0, Ws,
                                                        k2, al(L.pw), k2, mr, nc, k1);
    dim3 g2((unsigned)ceil_div(nr, 128), (unsigned)ceil_div(mr, 128));
    gemm_bf16p_kernel<NS, false, 32><<<g2, 256, 0, s>>>(Ws, k2, al(L.pw), Ns, k2, al(L.pn), U, ldu,
                                                         nullptr, 0, 0, 0, mr, nr, k2);
  }
  check_launch(s);
  if (!ws) GVT_HIP_CHECK(hipFreeAsync(buf, s));
}

size_t dense_workspace_bytes(int prec, int64_t mr, int64_t mc, int64_t nr, int64_t nc) {
  if (mr == 0 || nr == 0) return 0;
  if (prec == GVT_BF16X3) return SplitLayout(2, mr, mc, nr, nc).bytes();
  if (prec == GVT_BF16X6) return SplitLayout(3, mr, mc, nr, nc).bytes();
  const size_t es = prec == GVT_F64 ? sizeof(double) : sizeof(float);
  const size_t w = ((size_t)mr * nc * es + 255) / 256 * 256;
  const size_t sp = std::max(gemm_splits_bytes(mr, nc, mc, es), gemm_splits_bytes(mr, nr, nc, es));
  return w + sp + 256;
}

// Umat (mr x nr) = M (mr x mc) Vmat (mc x nc) N^T (N: nr x nc)
void dense_matvec(int prec, const void *Mp, int64_t mr, int64_t mc, int64_t ldm, const void *Np,
                  int64_t nr, int64_t nc, int64_t ldn, const void *Vp, int64_t ldv, void *Up,
                  int64_t ldu, void *ws, hipStream_t s) {
  if (mr == 0 || nr == 0) return;
  if (prec == GVT_BF16X3 || prec == GVT_BF16X6) {
    if (prec == GVT_BF16X3)
      dense_split_bf16<2>((const float *)Mp, mr, mc, ldm, (const float *)Np, nr, nc, ldn,
                          (const float *)Vp, ldv, (float *)Up, ldu, ws, s);
    else
      dense_split_bf16<3>((const float *)Mp, mr, mc, ldm, (const float *)Np, nr, nc, ldn,
                          (const float *)Vp, ldv, (float *)Up, ldu, ws, s);
    return;
  }
  void *W = ws;
  if (!W) GVT_HIP_CHECK(hipMallocAsync(&W, dense_workspace_bytes(prec, mr, mc, nr, nc), s));
  const size_t es = prec == GVT_F64 ? sizeof(double) : sizeof(float);
  void *part = static_cast<char *>(W) + ((size_t)mr * nc * es + 255) / 256 * 256;  // split-K partials
  if (prec == GVT_F64) {
    gemm<double, false>((const double *)Mp, ldm, (const double *)Vp, ldv, (double *)W, nc, mr, nc, mc,
                        (double *)part, s);
    gemm<double, true>((const double *)W, nc, (const double *)Np, ldn, (double *)Up, ldu, mr, nr, nc,
                       (double *)part, s);
  } else if (prec == GVT_F32) {
    gemm<float, false>((const float *)Mp, ldm, (const float *)Vp, ldv, (float *)W, nc, mr, nc, mc,
                       (float *)part, s);
    gemm<float, true>((const float *)W, nc, (const float *)Np, ldn, (float *)Up, ldu, mr, nr, nc,
                      (float *)part, s);
  }
  check_launch(s);
  if (!ws) GVT_HIP_CHECK(hipFreeAsync(W, s));
}

// ---- the product without allocation ----------------------------------------
// One workspace per device for gvt_dense_matvec_noalloc, in the code object's
// own device memory (each device that loads the library holds its copy until
// the process ends).  Host code never passes the array's name to a kernel: in
// host code it is only a stand-in for the symbol, so its device address is
// looked up once per device with that device current and kept.
static __device__ __align__(256) unsigned char dense_scratch[kDenseScratchBytes];

void *dense_scratch_ptr() {
  static std::mutex mu;
  static std::map<int, void *> ptr_of;
  int dev = 0;
  GVT_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptr_of.find(dev);
  if (it != ptr_of.end()) return it->second;
  void *p = nullptr;
  GVT_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(dense_scratch)));
  GVT_REQUIRE(p != nullptr, GVT_ERR_HIP, "no device address for the dense workspace");
  ptr_of[dev] = p;
  return p;
}

}  // namespace gvt
