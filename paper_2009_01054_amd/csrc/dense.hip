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
//          product ~ hi*hi' + hi*lo' + lo*hi' accumulated in FP32; the FP32
//          intermediate W is split again for the second GEMM.
//   BF16X6 the same with a three-way split x = hi + mid + lo and the six
//          products down to the FP32 rounding level.
//
// Tiling: 256 threads (2 x 2 waves), block tile 128 x 128, each wave owns a
// 64 x 64 sub-tile (4 x 4 MFMA blocks of 16 x 16).  Global tiles are
// prefetched into registers while the current LDS tile feeds the MFMAs.
#include "common.h"
#include "kernels.h"

namespace gvt {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// Output layout of the 16x16 MFMA blocks (checked with a one-hot lane probe on
// gfx950): lane l holds column l % 16; item v holds row 4*(l/16) + v for the
// FP32 and bf16 instructions but row (l/16) + 4*v for v_mfma_f64_16x16x4f64.
template <class T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// C[M x N] = A[M x K] * op(B),  op(B)[k][n] = BT ? B[n*ldb + k] : B[k*ldb + n]
template <class T, bool BT>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const T *__restrict__ A, int64_t lda,
                                                        const T *__restrict__ B, int64_t ldb,
                                                        T *__restrict__ C, int64_t ldc, int64_t M,
                                                        int64_t N, int64_t K) {
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

// Split-operand GEMM on bf16 MFMA with FP32 accumulation.  NS = 2 keeps the
// products hi*hi + hi*lo + lo*hi (bf16x3); NS = 3 keeps every product whose
// order is at most the FP32 rounding level: hh + hm + mh + hl + lh + mm
// (bf16x6).  Small terms are accumulated first.
template <int NS, bool BT>
__global__ __launch_bounds__(256) void gemm_bf16s_kernel(const float *__restrict__ A, int64_t lda,
                                                         const float *__restrict__ B, int64_t ldb,
                                                         float *__restrict__ C, int64_t ldc,
                                                         int64_t M, int64_t N, int64_t K) {
  constexpr int BM = 128, BN = 128, BK = 32, PK = BK + 8;
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

  // A tile BM x BK: thread -> row tid/2, 16 k's at (tid&1)*16
  const int ar = tid >> 1, ak = (tid & 1) * 16;
  // B: NT like A; NN: k-row tid/8 (0..31), 16 n's at (tid%8)*16
  const int br = BT ? (tid >> 1) : (tid >> 3);
  const int bc = BT ? ((tid & 1) * 16) : ((tid & 7) * 16);
  float ra[16], rb[16];
  auto load_tiles = [&](int64_t k0) {
    const int64_t gm = m0 + ar;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t gk = k0 + ak + u;
      ra[u] = (gm < M && gk < K) ? A[gm * lda + gk] : 0.f;
    }
    if (BT) {
      const int64_t gn = n0 + br;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t gk = k0 + bc + u;
        rb[u] = (gn < N && gk < K) ? B[gn * ldb + gk] : 0.f;
      }
    } else {
      const int64_t gk = k0 + br;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t gn = n0 + bc + u;
        rb[u] = (gk < K && gn < N) ? B[gk * ldb + gn] : 0.f;
      }
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      unsigned short sp[NS];
      split_bf16<NS>(ra[u], sp);
#pragma unroll
      for (int k = 0; k < NS; ++k) As[k][ar][ak + u] = sp[k];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      unsigned short sp[NS];
      split_bf16<NS>(rb[u], sp);
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        if (BT) Bs[k][br][bc + u] = sp[k];
        else Bs[k][bc + u][br] = sp[k];
      }
    }
  };
  auto frag = [&](const unsigned short(&X)[BM][PK], int row, int kofs) {
    return __builtin_bit_cast(bf8, *reinterpret_cast<const us8 *>(&X[row][kofs]));
  };
  load_tiles(0);
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    store_tiles();
    __syncthreads();
    if (k0 + BK < K) load_tiles(k0 + BK);
    const int kofs = 8 * (lane >> 4), rl = lane & 15;
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
        if (row < M && col < N) C[row * ldc + col] = acc[i][j][v];
      }
    }
}

template <class T, bool BT>
static void gemm(const T *A, int64_t lda, const T *B, int64_t ldb, T *C, int64_t ldc, int64_t M,
                 int64_t N, int64_t K, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(N, 128), (unsigned)ceil_div(M, 128));
  gemm_mfma_kernel<T, BT><<<grid, 256, 0, s>>>(A, lda, B, ldb, C, ldc, M, N, K);
}

template <int NS, bool BT>
static void gemm_bf16s(const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(N, 128), (unsigned)ceil_div(M, 128));
  gemm_bf16s_kernel<NS, BT><<<grid, 256, 0, s>>>(A, lda, B, ldb, C, ldc, M, N, K);
}

// Umat (mr x nr) = M (mr x mc) Vmat (mc x nc) N^T (N: nr x nc)
void dense_matvec(int prec, const void *Mp, int64_t mr, int64_t mc, int64_t ldm, const void *Np,
                  int64_t nr, int64_t nc, int64_t ldn, const void *Vp, int64_t ldv, void *Up,
                  int64_t ldu, hipStream_t s) {
  if (mr == 0 || nr == 0) return;
  const size_t es = prec == GVT_F64 ? sizeof(double) : sizeof(float);
  void *W = nullptr;
  GVT_HIP_CHECK(hipMallocAsync(&W, (size_t)mr * nc * es + 256, s));
  if (prec == GVT_F64) {
    gemm<double, false>((const double *)Mp, ldm, (const double *)Vp, ldv, (double *)W, nc, mr, nc, mc, s);
    gemm<double, true>((const double *)W, nc, (const double *)Np, ldn, (double *)Up, ldu, mr, nr, nc, s);
  } else if (prec == GVT_F32) {
    gemm<float, false>((const float *)Mp, ldm, (const float *)Vp, ldv, (float *)W, nc, mr, nc, mc, s);
    gemm<float, true>((const float *)W, nc, (const float *)Np, ldn, (float *)Up, ldu, mr, nr, nc, s);
  } else if (prec == GVT_BF16X3) {
    gemm_bf16s<2, false>((const float *)Mp, ldm, (const float *)Vp, ldv, (float *)W, nc, mr, nc, mc, s);
    gemm_bf16s<2, true>((const float *)W, nc, (const float *)Np, ldn, (float *)Up, ldu, mr, nr, nc, s);
  } else {
    gemm_bf16s<3, false>((const float *)Mp, ldm, (const float *)Vp, ldv, (float *)W, nc, mr, nc, mc, s);
    gemm_bf16s<3, true>((const float *)W, nc, (const float *)Np, ldn, (float *)Up, ldu, mr, nr, nc, s);
  }
  check_launch(s);
  GVT_HIP_CHECK(hipFreeAsync(W, s));
}

}  // namespace gvt
