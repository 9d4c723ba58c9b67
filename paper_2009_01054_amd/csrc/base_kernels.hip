// Base kernel matrices from object features (Section 5): the drug and target
// kernels D and T that every pairwise kernel of the library is built from.
//
//   linear    k(x, y) = <x, y>
//   gaussian  k(x, y) = exp(-gamma ||x - y||^2)   (squared Euclidean norm)
//   tanimoto  k(v, w) = |v and w| / |v or w| on binary vectors (packed bits)
//
// Linear and Gaussian kernels are a Gram product X Y^T on matrix cores with
// the kernel applied in the store epilogue: for the Gaussian,
// ||x - y||^2 = ||x||^2 + ||y||^2 - 2 <x, y> from row norms computed first,
// clamped at 0, and 0 on the diagonal of a kernel of one sample with itself.
// The feature dimension is short (tens to a few hundred), so the kernel
// matrix write dominates: one pass over K, nothing re-read.  With Y = X the
// launch computes the tiles on and above the diagonal only and writes each
// off-diagonal value to both (i, j) and (j, i), so the result is exactly
// symmetric (the library's symmetric-base flag reads columns as rows).
//
// The Tanimoto kernel counts bits with popcount over 64-bit words: each block
// stages 64 rows of each sample in LDS, 16 words at a time, and every thread
// keeps 4 x 4 intersection counts; the row counts come from a first pass.
// Counts are exact integers and the ratio is formed in double, so results do
// not depend on the order of anything.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace gvt {

// sq[i] = ||X_i||^2 (sum in ascending feature order)
template <class T>
__global__ void row_sqnorm_kernel(const T *__restrict__ X, int64_t ldx, int64_t n, int64_t dim,
                                  T *__restrict__ sq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = T(0);
  for (int64_t k = 0; k < dim; ++k) {
    const T x = X[i * ldx + k];
    s += x * x;
  }
  sq[i] = s;
}

template <class T> __device__ __forceinline__ T kexp(T x);
template <> __device__ __forceinline__ double kexp<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float kexp<float>(float x) { return expf(x); }

// K[i, j] = k(X_i, Y_j) for one 128 x 128 tile; 256 threads as 2 x 2 waves of
// 64 x 64 (4 x 4 MFMA blocks of 16 x 16), k steps of 16 features.
// GAUSS: 0 linear, 1 Gaussian.  sym: Y == X, tiles below the diagonal return
// at once and each value above it is written twice.
template <class T, int GAUSS>
__global__ __launch_bounds__(256) void gram_kernel(const T *__restrict__ X, int64_t ldx,
                                                   const T *__restrict__ Y, int64_t ldy,
                                                   const T *__restrict__ xsq, const T *__restrict__ ysq,
                                                   int64_t nx, int64_t ny, int64_t dim, T gamma,
                                                   T *__restrict__ K, int64_t ldk, int sym) {
  constexpr int BM = 128, BN = 128, BK = 16, PAD = 4;
  typedef typename Mfma<T>::acc_t acc_t;
  if (sym && blockIdx.x < blockIdx.y) return;
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
  // thread -> tile row tid/2, 8 features at (tid&1)*8, for both operands
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  T ra[8], rb[8];
  auto load = [&](int64_t k0) {
    const int64_t gm = m0 + ar, gn = n0 + ar;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t gk = k0 + ak + u;
      ra[u] = (gm < nx && gk < dim) ? X[gm * ldx + gk] : T(0);
      rb[u] = (gn < ny && gk < dim) ? Y[gn * ldy + gk] : T(0);
    }
  };
  load(0);
  for (int64_t k0 = 0; k0 < dim; k0 += BK) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      As[ak + u][ar] = ra[u];
      Bs[ak + u][ar] = rb[u];
    }
    __syncthreads();
    if (k0 + BK < dim) load(k0 + BK);
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
  const bool diag_tile = sym && blockIdx.x == blockIdx.y;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + Mfma<T>::row(lane, v);
        if (row >= nx || col >= ny) continue;
        if (diag_tile && row > col) continue;  // written as the mirror of (col, row)
        T val = acc[i][j][v];
        if (GAUSS) {
          T d2 = (sym && row == col) ? T(0) : xsq[row] + ysq[col] - T(2) * val;
          d2 = d2 > T(0) ? d2 : T(0);
          val = kexp<T>(-gamma * d2);
        }
        K[row * ldk + col] = val;
        if (sym && row != col) K[col * ldk + row] = val;
      }
    }
}

// ---- Tanimoto on packed bits ------------------------------------------------------
// cnt[i] = number of set bits among the first nbits bits of row i
__global__ void row_popcount_kernel(const uint64_t *__restrict__ X, int64_t ldx, int64_t n,
                                    int64_t words, uint64_t lastmask, int32_t *__restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = 0;
  for (int64_t w = 0; w < words; ++w) {
    uint64_t x = X[i * ldx + w];
    if (w == words - 1) x &= lastmask;
    c += __popcll(x);
  }
  cnt[i] = c;
}

constexpr int kTaniTile = 64, kTaniWords = 16;

template <class T>
__global__ __launch_bounds__(256) void tanimoto_kernel(const uint64_t *__restrict__ X, int64_t ldx,
                                                       const uint64_t *__restrict__ Y, int64_t ldy,
                                                       const int32_t *__restrict__ xc,
                                                       const int32_t *__restrict__ yc, int64_t nx,
                                                       int64_t ny, int64_t words, uint64_t lastmask,
                                                       T *__restrict__ K, int64_t ldk) {
  __shared__ uint64_t xs[kTaniTile][kTaniWords + 1];
  __shared__ uint64_t ys[kTaniTile][kTaniWords + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t m0 = (int64_t)blockIdx.y * kTaniTile, n0 = (int64_t)blockIdx.x * kTaniTile;
  int32_t both[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w) both[u][w] = 0;
  for (int64_t w0 = 0; w0 < words; w0 += kTaniWords) {
    for (int e = tid; e < kTaniTile * kTaniWords; e += 256) {
      const int r = e / kTaniWords, k = e % kTaniWords;
      const int64_t gw = w0 + k;
      const uint64_t mk = gw == words - 1 ? lastmask : ~(uint64_t)0;
      xs[r][k] = (m0 + r < nx && gw < words) ? (X[(m0 + r) * ldx + gw] & mk) : 0;
      ys[r][k] = (n0 + r < ny && gw < words) ? (Y[(n0 + r) * ldy + gw] & mk) : 0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kTaniWords; ++k) {
      uint64_t a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = xs[ty * 4 + u][k];
#pragma unroll
      for (int w = 0; w < 4; ++w) b[w] = ys[tx + 16 * w][k];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) both[u][w] += __popcll(a[u] & b[w]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t row = m0 + ty * 4 + u;
    if (row >= nx) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int64_t col = n0 + tx + 16 * w;
      if (col >= ny) continue;
      const int32_t c = both[u][w], either = xc[row] + yc[col] - c;
      const double r = either == 0 ? 1.0 : (double)c / (double)either;
      K[row * ldk + col] = (T)r;
    }
  }
}

// ---- host side -----------------------------------------------------------------------
template <class T>
static void gram_t(int gauss, const T *X, int64_t nx, int64_t ldx, const T *Y, int64_t ny, int64_t ldy,
                   int64_t dim, double gamma, T *K, int64_t ldk, hipStream_t s) {
  const int sym = Y == nullptr;
  if (sym) {
    Y = X;
    ldy = ldx;
  }
  T *xsq = nullptr, *ysq = nullptr;
  if (gauss) {
    void *buf = nullptr;
    GVT_HIP_CHECK(hipMallocAsync(&buf, (size_t)(nx + ny) * sizeof(T) + 256, s));
    xsq = (T *)buf;
    row_sqnorm_kernel<T><<<(unsigned)ceil_div(nx, 256), 256, 0, s>>>(X, ldx, nx, dim, xsq);
    ysq = xsq;
    if (!sym) {
      ysq = xsq + nx;
      row_sqnorm_kernel<T><<<(unsigned)ceil_div(ny, 256), 256, 0, s>>>(Y, ldy, ny, dim, ysq);
    }
  }
  const dim3 grid((unsigned)ceil_div(ny, 128), (unsigned)ceil_div(nx, 128));
  if (gauss)
    gram_kernel<T, 1><<<grid, 256, 0, s>>>(X, ldx, Y, ldy, xsq, ysq, nx, ny, dim, (T)gamma, K, ldk, sym);
  else
    gram_kernel<T, 0><<<grid, 256, 0, s>>>(X, ldx, Y, ldy, xsq, ysq, nx, ny, dim, (T)gamma, K, ldk, sym);
  check_launch(s);
  if (gauss) GVT_HIP_CHECK(hipFreeAsync(xsq, s));
}

void base_kernel(int kind, int prec, const void *X, int64_t nx, int64_t ldx, const void *Y, int64_t ny,
                 int64_t ldy, int64_t dim, double gamma, void *K, int64_t ldk, hipStream_t s) {
  if (nx == 0 || ny == 0) return;
  const int gauss = kind == GVT_BASE_GAUSSIAN;
  if (prec == GVT_F64)
    gram_t<double>(gauss, (const double *)X, nx, ldx, (const double *)Y, ny, ldy, dim, gamma, (double *)K,
                   ldk, s);
  else
    gram_t<float>(gauss, (const float *)X, nx, ldx, (const float *)Y, ny, ldy, dim, gamma, (float *)K, ldk,
                  s);
}

void tanimoto_kernel_matrix(int prec, const uint64_t *X, int64_t nx, int64_t ldx, const uint64_t *Y,
                            int64_t ny, int64_t ldy, int64_t nbits, void *K, int64_t ldk, hipStream_t s) {
  if (nx == 0 || ny == 0) return;
  const bool sym = Y == nullptr;
  if (sym) {
    Y = X;
    ldy = ldx;
  }
  const int64_t words = (nbits + 63) / 64;
  const uint64_t lastmask = nbits % 64 == 0 ? ~(uint64_t)0 : (((uint64_t)1 << (nbits % 64)) - 1);
  void *buf = nullptr;
  GVT_HIP_CHECK(hipMallocAsync(&buf, (size_t)(nx + ny) * sizeof(int32_t) + 256, s));
  int32_t *xc = (int32_t *)buf, *yc = xc + nx;
  row_popcount_kernel<<<(unsigned)ceil_div(nx, 256), 256, 0, s>>>(X, ldx, nx, words, lastmask, xc);
  row_popcount_kernel<<<(unsigned)ceil_div(ny, 256), 256, 0, s>>>(Y, ldy, ny, words, lastmask, yc);
  const dim3 grid((unsigned)ceil_div(ny, kTaniTile), (unsigned)ceil_div(nx, kTaniTile));
  if (prec == GVT_F64)
    tanimoto_kernel<double><<<grid, 256, 0, s>>>(X, ldx, Y, ldy, xc, yc, nx, ny, words, lastmask, (double *)K, ldk);
  else
    tanimoto_kernel<float><<<grid, 256, 0, s>>>(X, ldx, Y, ldy, xc, yc, nx, ny, words, lastmask, (float *)K, ldk);
  check_launch(s);
  GVT_HIP_CHECK(hipFreeAsync(buf, s));
}

}  // namespace gvt
