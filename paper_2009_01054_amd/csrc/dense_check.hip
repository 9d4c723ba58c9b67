// Error estimate of a complete-data product against FP64 arithmetic.
//
// The split-bf16 products keep about 16 (bf16x3) or 24 (bf16x6) significant
// bits of each operand, so their error relative to |Umat| depends on how much
// the sums cancel, which the inputs decide.  The checked product therefore
// measures it: for NSAMP rows of Umat, spread evenly over the rows, it
// recomputes Umat[r, :] = (M[r, :] Vmat) N^T in FP64 from the same stored
// operands and returns ||U_S - U_S,ref||_F / ||U_S,ref||_F over those rows.
//
// Kernels (all sums in a fixed order, so the estimate is reproducible):
//   sample_mv_kernel   P_part[c][i, j] = sum_{k in k-chunk c} M[r_i, k] Vmat[k, j]
//                      one thread per column j, the chunk of the NSAMP rows of
//                      M staged in LDS as FP64, NSAMP accumulators per thread
//   sample_fold_kernel P[i, j] = sum_c P_part[c][i, j]   (ascending c)
//   sample_err_kernel  two columns t of Umat per wave, the lanes split k over
//                      panels of P staged in LDS: Uref[i, t] = sum_k P[i, k] N[t, k],
//                      then per-block sums of (U[r_i, t] - Uref[i, t])^2 and Uref[i, t]^2
//   sample_norm_kernel folds the block sums into two doubles
#include "common.h"
#include "kernels.h"

namespace gvt {

constexpr int kSampleRows = 16;  // rows of Umat sampled (fewer when Umat has fewer)
constexpr int kSampleKc = 64;    // k-chunk of M rows staged in LDS
constexpr int kSampleThreads = 256;

__device__ __forceinline__ int64_t sample_row(int i, int ns, int64_t mr) {
  return (int64_t)i * mr / ns;
}

template <class T>
__global__ __launch_bounds__(kSampleThreads) void sample_mv_kernel(
    const T *__restrict__ M, int64_t ldm, int64_t mr, int ns, const T *__restrict__ V, int64_t ldv,
    int64_t mc, int64_t nc, int64_t kper, double *__restrict__ part) {
  __shared__ double ms[kSampleRows][kSampleKc];
  const int64_t j = (int64_t)blockIdx.x * kSampleThreads + threadIdx.x;
  const int64_t kbeg = (int64_t)blockIdx.y * kper, kend = min(mc, kbeg + kper);
  double acc[kSampleRows];
#pragma unroll
  for (int i = 0; i < kSampleRows; ++i) acc[i] = 0.0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kSampleKc) {
    for (int e = threadIdx.x; e < kSampleRows * kSampleKc; e += kSampleThreads) {
      const int i = e / kSampleKc, kk = e % kSampleKc;
      ms[i][kk] = (i < ns && k0 + kk < kend) ? (double)M[sample_row(i, ns, mr) * ldm + k0 + kk] : 0.0;
    }
    __syncthreads();
    if (j < nc) {
      const int kn = (int)min((int64_t)kSampleKc, kend - k0);
      for (int kk = 0; kk < kn; ++kk) {
        const double v = (double)V[(k0 + kk) * ldv + j];
#pragma unroll
        for (int i = 0; i < kSampleRows; ++i) acc[i] += ms[i][kk] * v;
      }
    }
    __syncthreads();
  }
  if (j < nc)
    for (int i = 0; i < ns; ++i) part[((int64_t)blockIdx.y * ns + i) * nc + j] = acc[i];
}

__global__ void sample_fold_kernel(const double *__restrict__ part, int nsplit, int ns, int64_t nc,
                                   double *__restrict__ P) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)ns * nc) return;
  double s = 0.0;
  for (int c = 0; c < nsplit; ++c) s += part[(int64_t)c * ns * nc + q];
  P[q] = s;
}

// Sum over the 64 lanes of a wave; every lane ends with the same value.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Two output columns per wave, eight per block: each step stages a 32 x 64
// panel of P in LDS once for the block; a lane takes one k of the panel.
constexpr int kErrCols = 2 * (kSampleThreads / 64);

template <class T>
__global__ __launch_bounds__(kSampleThreads) void sample_err_kernel(
    const double *__restrict__ P, int ns, int64_t nc, const T *__restrict__ N, int64_t ldn,
    int64_t nr, const T *__restrict__ U, int64_t ldu, int64_t mr, double *__restrict__ blocksums) {
  __shared__ double pp[kSampleRows][64];
  __shared__ double sh[2][kSampleThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kErrCols + 2 * w;  // this wave's columns t0, t0 + 1
  double acc[2][kSampleRows];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < kSampleRows; ++i) acc[c][i] = 0.0;
  for (int64_t k0 = 0; k0 < nc; k0 += 64) {
    for (int e = threadIdx.x; e < kSampleRows * 64; e += kSampleThreads) {
      const int i = e >> 6, kk = e & 63;
      pp[i][kk] = (i < ns && k0 + kk < nc) ? P[(int64_t)i * nc + k0 + kk] : 0.0;
    }
    __syncthreads();
    const int64_t k = k0 + lane;
    const double n0 = (t0 < nr && k < nc) ? (double)N[t0 * ldn + k] : 0.0;
    const double n1 = (t0 + 1 < nr && k < nc) ? (double)N[(t0 + 1) * ldn + k] : 0.0;
#pragma unroll
    for (int i = 0; i < kSampleRows; ++i) {
      const double pv = pp[i][lane];
      acc[0][i] += pv * n0;
      acc[1][i] += pv * n1;
    }
    __syncthreads();
  }
  double e2 = 0.0, r2 = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int64_t t = t0 + c;
#pragma unroll
    for (int i = 0; i < kSampleRows; ++i) {
      const double ref = wave_sum(acc[c][i]);  // every lane of the wave takes part
      if (i < ns && t < nr) {
        const double d = (double)U[sample_row(i, ns, mr) * ldu + t] - ref;
        e2 += d * d;
        r2 += ref * ref;
      }
    }
  }
  if (lane == 0) {
    sh[0][w] = e2;
    sh[1][w] = r2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < kSampleThreads / 64; ++i) {
      a += sh[0][i];
      b += sh[1][i];
    }
    blocksums[2 * blockIdx.x] = a;
    blocksums[2 * blockIdx.x + 1] = b;
  }
}

__global__ void sample_norm_kernel(const double *__restrict__ blocksums, int64_t nb,
                                   double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int64_t i = 0; i < nb; ++i) {
    a += blocksums[2 * i];
    b += blocksums[2 * i + 1];
  }
  out[0] = a;
  out[1] = b;
}

template <class T>
static double sample_relerr_t(const T *M, int64_t mr, int64_t mc, int64_t ldm, const T *N, int64_t nr,
                              int64_t nc, int64_t ldn, const T *V, int64_t ldv, const T *U, int64_t ldu,
                              hipStream_t s) {
  const int ns = (int)std::min<int64_t>(mr, kSampleRows);
  const int64_t jb = ceil_div(nc, kSampleThreads);
  // split k so that the first kernel has about 512 blocks
  const int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>(ceil_div(512, jb), ceil_div(mc, kSampleKc)));
  const int64_t kper = ceil_div(ceil_div(mc, nsplit), kSampleKc) * kSampleKc;
  const int64_t nsp = std::max<int64_t>(1, ceil_div(mc, kper));
  const int64_t eb = ceil_div(nr, kErrCols);
  const size_t bytes = (size_t)(nsp * ns * nc + ns * nc + 2 * eb + 2) * sizeof(double);
  DevMem buf;
  double *base = (double *)buf.ensure(bytes);
  double *part = base, *P = part + nsp * ns * nc, *bs = P + ns * nc, *out = bs + 2 * eb;
  if (mc > 0) {
    sample_mv_kernel<T><<<dim3((unsigned)jb, (unsigned)nsp), kSampleThreads, 0, s>>>(
        M, ldm, mr, ns, V, ldv, mc, nc, kper, part);
    sample_fold_kernel<<<(unsigned)ceil_div((int64_t)ns * nc, 256), 256, 0, s>>>(part, (int)nsp, ns, nc, P);
  } else {
    GVT_HIP_CHECK(hipMemsetAsync(P, 0, (size_t)ns * nc * sizeof(double), s));
  }
  sample_err_kernel<T><<<(unsigned)eb, kSampleThreads, 0, s>>>(P, ns, nc, N, ldn, nr, U, ldu, mr, bs);
  sample_norm_kernel<<<1, 64, 0, s>>>(bs, eb, out);
  check_launch(s);
  double h[2];
  GVT_HIP_CHECK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return NAN;
  return h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
}

double dense_sample_relerr(int prec, const void *M, int64_t mr, int64_t mc, int64_t ldm, const void *N,
                           int64_t nr, int64_t nc, int64_t ldn, const void *V, int64_t ldv,
                           const void *U, int64_t ldu, hipStream_t s) {
  if (mr == 0 || nr == 0) return 0.0;
  if (prec == GVT_F64)
    return sample_relerr_t<double>((const double *)M, mr, mc, ldm, (const double *)N, nr, nc, ldn,
                                   (const double *)V, ldv, (const double *)U, ldu, s);
  return sample_relerr_t<float>((const float *)M, mr, mc, ldm, (const float *)N, nr, nc, ldn,
                                (const float *)V, ldv, (const float *)U, ldu, s);
}

}  // namespace gvt
