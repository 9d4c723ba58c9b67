// Gather-path kernels of the generalized vec trick (Theorem 1) for gfx950.
//
// One Kronecker term u_i = sum_j F1[x_i, k_j] F2[y_i, o_j] v_j is applied in
// two stages:
//   stage 1 (segmented scatter-reduce):  S[y, k] = sum_{j: k_j = k} F2[y, o_j] v_j
//   stage 2 (gather-dot):                u_i    = sum_k F1[x_i, k] S[y_i, k]
// Input pairs are pre-sorted by the key k into contiguous segments, so every
// sum is a sequential loop or a fixed lane tree: results are deterministic
// (no atomics).  Several right-hand sides (R) ride along in the innermost
// dimension so that each gathered base-matrix element feeds R FMAs.
#include "common.h"
#include "kernels.h"

namespace gvt {

static constexpr int WAVE = 64;

__device__ __forceinline__ int wave_id_uniform() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// ---------------------------------------------------------------------------
// vs[p*R + r] = V[perm[p] + r*ldv]  (input vector gathered into key order)
template <class T>
__global__ void pack_v_kernel(const T *__restrict__ V, int64_t ldv, const int32_t *__restrict__ perm,
                              int64_t n, int R, T *__restrict__ vs) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int64_t j = perm[p];
  for (int r = 0; r < R; ++r) vs[p * R + r] = V[j + r * ldv];
}

// s[k*R + r] = sum_{p in seg(k)} vs[p*R + r]   (segment sums, sequential per key)
template <class T>
__global__ void segsum_kernel(const int64_t *__restrict__ seg, const T *__restrict__ vs,
                              int64_t nkeys, int R, T *__restrict__ s) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  int64_t p0 = seg[k], p1 = seg[k + 1];
  for (int r = 0; r < R; ++r) {
    T acc = T(0);
    for (int64_t p = p0; p < p1; ++p) acc += vs[p * R + r];
    s[k * R + r] = acc;
  }
}

// ---------------------------------------------------------------------------
// Stage 1.  Fc holds F2 column-accessible: F2[y, o] = Fc[o*ldc + y].
// Block = 4 waves; lane <-> one S row (64 rows per block); each wave owns
// KB/4 consecutive keys.  Segment data (other index, packed v) are wave-
// uniform and come through the scalar cache; the F2 column segment load is
// coalesced across lanes.  The [64 x KB*R] result tile is staged in LDS and
// written row-contiguously.
template <class T, int R, int KB>
__global__ __launch_bounds__(256) void stage1_kernel(
    const T *__restrict__ Fc, int64_t ldc, const int32_t *__restrict__ rows, int64_t nrows,
    const int64_t *__restrict__ seg, const int32_t *__restrict__ other,
    const T *__restrict__ vs, int64_t nkeys, T *__restrict__ S) {
  __shared__ T tile[64][KB * R + 1];
  const int lane = threadIdx.x & 63;
  const int w = wave_id_uniform();
  const int64_t k0 = (int64_t)blockIdx.x * KB;
  const int64_t rho0 = (int64_t)blockIdx.y * 64;
  const int64_t rho = rho0 + lane;
  const bool live = rho < nrows;
  const int64_t y = live ? rows[rho] : 0;
  constexpr int KPW = KB / 4;
#pragma unroll 1
  for (int t = 0; t < KPW; ++t) {
    const int kk = w * KPW + t;
    const int64_t k = k0 + kk;
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);
    if (k < nkeys) {
      const int64_t p0 = seg[k], p1 = seg[k + 1];
#pragma unroll 4
      for (int64_t p = p0; p < p1; ++p) {
        const int64_t o = other[p];
        const T f = live ? Fc[o * ldc + y] : T(0);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += f * vs[p * R + r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) tile[lane][kk * R + r] = acc[r];
  }
  __syncthreads();
  const int64_t kcount = (nkeys - k0) < KB ? (nkeys - k0) : KB;
  const int width = (int)kcount * R;
  for (int idx = threadIdx.x; idx < 64 * KB * R; idx += 256) {
    const int rr = idx / (KB * R);
    const int cc = idx - rr * (KB * R);
    const int64_t orow = rho0 + rr;
    if (orow < nrows && cc < width) S[(orow * nkeys + k0) * R + cc] = tile[rr][cc];
  }
}

// Degenerate stage 1 (key == other index): S[rho, k] = F2[rows[rho], k] * s[k].
template <class T>
__global__ void colscale_kernel(const T *__restrict__ F, int64_t ldf, const int32_t *__restrict__ rows,
                                int64_t nrows, const T *__restrict__ s, int64_t nkeys, int R,
                                T *__restrict__ S) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = nrows * nkeys;
  if (idx >= total) return;
  int64_t rho = idx / nkeys, k = idx - rho * nkeys;
  T f = F[(int64_t)rows[rho] * ldf + k];
  for (int r = 0; r < R; ++r) S[idx * R + r] = f * s[k * R + r];
}

// ---------------------------------------------------------------------------
// Stage 2.  Outputs are visited in plan order (grouped by x, the F1 row);
// 8 lanes cooperate on one output, striding over k; the partial sums meet in
// a fixed 3-step butterfly.  out[i*ldi + r*ldr] = coef * sum_k F1[x,k] S[yrow,k,r]
template <class T, int R>
__global__ __launch_bounds__(256) void stage2_kernel(
    const T *__restrict__ F1, int64_t ld1, const int32_t *__restrict__ xs,
    const int32_t *__restrict__ yrows, const int32_t *__restrict__ perm, int64_t nq,
    const T *__restrict__ S, int64_t nkeys, T coef, T *__restrict__ out, int64_t ldi,
    int64_t ldr) {
  const int sub = threadIdx.x & 7;
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const bool live = q < nq;
  T acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = T(0);
  if (live) {
    const T *frow = F1 + (int64_t)xs[q] * ld1;
    const T *srow = S + (int64_t)yrows[q] * nkeys * R;
#pragma unroll 4
    for (int64_t k = sub; k < nkeys; k += 8) {
      const T f = frow[k];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += f * srow[k * R + r];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    acc[r] += __shfl_xor(acc[r], 1);
    acc[r] += __shfl_xor(acc[r], 2);
    acc[r] += __shfl_xor(acc[r], 4);
  }
  if (live && sub == 0) {
    const int64_t i = perm[q];
#pragma unroll
    for (int r = 0; r < R; ++r) out[i * ldi + r * ldr] = coef * acc[r];
  }
}

// ---------------------------------------------------------------------------
// One-factor terms: g[x*R + r] = sum_k F(x,k)^{1|2} s[k*R + r]; one wave per row.
template <class T, bool SQ>
__global__ __launch_bounds__(256) void gemv_kernel(const T *__restrict__ F, int64_t ldf,
                                                   int64_t nrows, int64_t ncols,
                                                   const T *__restrict__ s, int R,
                                                   T *__restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int64_t x = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= nrows) return;
  const T *frow = F + x * ldf;
  for (int r = 0; r < R; ++r) {
    T acc = T(0);
    for (int64_t k = lane; k < ncols; k += WAVE) {
      T f = frow[k];
      if (SQ) f = f * f;
      acc += f * s[k * R + r];
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) g[x * R + r] = acc;
  }
}

// t[i*R + r] = g[sel[i]*R + r]
template <class T>
__global__ void gather_rows_kernel(const T *__restrict__ g, const int32_t *__restrict__ sel,
                                   int64_t n, int R, T *__restrict__ t) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t x = sel[i];
  for (int r = 0; r < R; ++r) t[i * R + r] = g[x * R + r];
}

// Cartesian sparse-match term: t[i] = sum_{p in seg(kv_i)} F[x_i, other_p] vs[p]
// (kv_i >= nkeys: the object never occurs on the input side -> 0).
template <class T>
__global__ void match_kernel(const T *__restrict__ F, int64_t ldf, const int32_t *__restrict__ xsel,
                             const int32_t *__restrict__ ksel, int64_t n, const int64_t *__restrict__ seg,
                             const int32_t *__restrict__ other, const T *__restrict__ vs,
                             int64_t nkeys, int R, T *__restrict__ t) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t kv = ksel[i];
  const T *frow = F + (int64_t)xsel[i] * ldf;
  int64_t p0 = 0, p1 = 0;
  if (kv < nkeys) { p0 = seg[kv]; p1 = seg[kv + 1]; }
  for (int r = 0; r < R; ++r) {
    T acc = T(0);
    for (int64_t p = p0; p < p1; ++p) acc += frow[other[p]] * vs[p * R + r];
    t[i * R + r] = acc;
  }
}

// Ft[o*ldt + y] = F[y*ldf + o]  (32x32 LDS tiles)
template <class T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *__restrict__ F, int64_t ldf,
                                                        int64_t rows, int64_t cols,
                                                        T *__restrict__ Ft, int64_t ldt) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int j = ty; j < 32; j += 8) {
    int64_t r = r0 + j, c = c0 + tx;
    if (r < rows && c < cols) tile[j][tx] = F[r * ldf + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    int64_t c = c0 + j, r = r0 + tx;
    if (r < rows && c < cols) Ft[c * ldt + r] = tile[tx][j];
  }
}

// U_o[i + r*ldu] = sum_k coef[o][k] * t_k[i*R + r]
template <class T>
__global__ void combine_kernel(CombineArgs<T> a, int64_t n, int R, T *__restrict__ U, int64_t ldu,
                               int64_t block_stride) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int o = 0; o < a.nout; ++o) {
    T *Uo = U + o * block_stride;
    for (int r = 0; r < R; ++r) {
      T acc = T(0);
      for (int k = 0; k < a.nterms; ++k) {
        const T c = a.coef[o][k];
        if (c != T(0)) acc += c * a.t[k][i * R + r];
      }
      Uo[i + r * ldu] = acc;
    }
  }
}

template <class T>
__global__ void fill_kernel(T *__restrict__ U, int64_t rows, int64_t cols, int64_t ld, T val) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  int64_t c = idx / rows, r = idx - c * rows;
  U[r + c * ld] = val;
}

// ===========================================================================
// Launchers
// ===========================================================================
static inline dim3 grid1(int64_t n, int bs) { return dim3((unsigned)ceil_div(n, bs)); }

template <class T>
void launch_pack_v(const T *V, int64_t ldv, const int32_t *perm, int64_t n, int R, T *vs,
                   hipStream_t s) {
  if (n <= 0) return;
  pack_v_kernel<T><<<grid1(n, 256), 256, 0, s>>>(V, ldv, perm, n, R, vs);
}

template <class T>
void launch_segsum(const int64_t *seg, const T *vs, int64_t nkeys, int R, T *out, hipStream_t s) {
  if (nkeys <= 0) return;
  segsum_kernel<T><<<grid1(nkeys, 256), 256, 0, s>>>(seg, vs, nkeys, R, out);
}

template <class T, int R>
static void stage1_r(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows, const int64_t *seg,
                     const int32_t *other, const T *vs, int64_t nkeys, T *S, hipStream_t s) {
  constexpr int KB = (R >= 8) ? 8 : 16;
  dim3 grid((unsigned)ceil_div(nkeys, KB), (unsigned)ceil_div(nrows, 64));
  stage1_kernel<T, R, KB><<<grid, 256, 0, s>>>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S);
}

template <class T>
void launch_stage1(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows, const int64_t *seg,
                   const int32_t *other, const T *vs, int64_t nkeys, int R, T *S, hipStream_t s) {
  if (nrows <= 0 || nkeys <= 0) return;
  switch (R) {
    case 1: stage1_r<T, 1>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, s); break;
    case 2: stage1_r<T, 2>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, s); break;
    case 4: stage1_r<T, 4>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, s); break;
    case 8: stage1_r<T, 8>(Fc, ldc, rows, nrows, seg, other, vs, nkeys, S, s); break;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in stage 1"};
  }
}

template <class T>
void launch_colscale(const T *F, int64_t ldf, const int32_t *rows, int64_t nrows, const T *sv,
                     int64_t nkeys, int R, T *S, hipStream_t s) {
  if (nrows * nkeys <= 0) return;
  colscale_kernel<T><<<grid1(nrows * nkeys, 256), 256, 0, s>>>(F, ldf, rows, nrows, sv, nkeys, R, S);
}

template <class T>
void launch_stage2(const T *F1, int64_t ld1, const int32_t *xs, const int32_t *yrows,
                   const int32_t *perm, int64_t nq, const T *S, int64_t nkeys, int R, T coef, T *out,
                   int64_t ldi, int64_t ldr, hipStream_t s) {
  if (nq <= 0) return;
  dim3 grid = grid1(nq * 8, 256);
  switch (R) {
    case 1: stage2_kernel<T, 1><<<grid, 256, 0, s>>>(F1, ld1, xs, yrows, perm, nq, S, nkeys, coef, out, ldi, ldr); break;
    case 2: stage2_kernel<T, 2><<<grid, 256, 0, s>>>(F1, ld1, xs, yrows, perm, nq, S, nkeys, coef, out, ldi, ldr); break;
    case 4: stage2_kernel<T, 4><<<grid, 256, 0, s>>>(F1, ld1, xs, yrows, perm, nq, S, nkeys, coef, out, ldi, ldr); break;
    case 8: stage2_kernel<T, 8><<<grid, 256, 0, s>>>(F1, ld1, xs, yrows, perm, nq, S, nkeys, coef, out, ldi, ldr); break;
    default: throw Error{GVT_ERR_ARG, "internal: unsupported RHS block in stage 2"};
  }
}

template <class T>
void launch_gemv(const T *F, int64_t ldf, int64_t nrows, int64_t ncols, bool sq, const T *sv, int R,
                 T *g, hipStream_t s) {
  if (nrows <= 0) return;
  dim3 grid((unsigned)ceil_div(nrows, 4));
  if (sq) gemv_kernel<T, true><<<grid, 256, 0, s>>>(F, ldf, nrows, ncols, sv, R, g);
  else gemv_kernel<T, false><<<grid, 256, 0, s>>>(F, ldf, nrows, ncols, sv, R, g);
}

template <class T>
void launch_gather_rows(const T *g, const int32_t *sel, int64_t n, int R, T *t, hipStream_t s) {
  if (n <= 0) return;
  gather_rows_kernel<T><<<grid1(n, 256), 256, 0, s>>>(g, sel, n, R, t);
}

template <class T>
void launch_match(const T *F, int64_t ldf, const int32_t *xsel, const int32_t *ksel, int64_t n,
                  const int64_t *seg, const int32_t *other, const T *vs, int64_t nkeys, int R, T *t,
                  hipStream_t s) {
  if (n <= 0) return;
  match_kernel<T><<<grid1(n, 256), 256, 0, s>>>(F, ldf, xsel, ksel, n, seg, other, vs, nkeys, R, t);
}

template <class T>
void launch_transpose(const T *F, int64_t ldf, int64_t rows, int64_t cols, T *Ft, int64_t ldt,
                      hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32));
  transpose_kernel<T><<<grid, 256, 0, s>>>(F, ldf, rows, cols, Ft, ldt);
}

template <class T>
void launch_combine(const CombineArgs<T> &a, int64_t n, int R, T *U, int64_t ldu,
                    int64_t block_stride, hipStream_t s) {
  if (n <= 0) return;
  combine_kernel<T><<<grid1(n, 256), 256, 0, s>>>(a, n, R, U, ldu, block_stride);
}

template <class T>
void launch_fill(T *U, int64_t rows, int64_t cols, int64_t ld, T val, hipStream_t s) {
  if (rows * cols <= 0) return;
  fill_kernel<T><<<grid1(rows * cols, 256), 256, 0, s>>>(U, rows, cols, ld, val);
}

#define GVT_INSTANTIATE(T)                                                                      \
  template void launch_pack_v<T>(const T *, int64_t, const int32_t *, int64_t, int, T *,          \
                                 hipStream_t);                                                   \
  template void launch_segsum<T>(const int64_t *, const T *, int64_t, int, T *, hipStream_t);    \
  template void launch_stage1<T>(const T *, int64_t, const int32_t *, int64_t, const int64_t *,  \
                                 const int32_t *, const T *, int64_t, int, T *, hipStream_t);    \
  template void launch_colscale<T>(const T *, int64_t, const int32_t *, int64_t, const T *,      \
                                   int64_t, int, T *, hipStream_t);                              \
  template void launch_stage2<T>(const T *, int64_t, const int32_t *, const int32_t *,           \
                                 const int32_t *, int64_t, const T *, int64_t, int, T, T *,      \
                                 int64_t, int64_t, hipStream_t);                                 \
  template void launch_gemv<T>(const T *, int64_t, int64_t, int64_t, bool, const T *, int, T *,  \
                               hipStream_t);                                                     \
  template void launch_gather_rows<T>(const T *, const int32_t *, int64_t, int, T *,             \
                                      hipStream_t);                                              \
  template void launch_match<T>(const T *, int64_t, const int32_t *, const int32_t *, int64_t,   \
                                const int64_t *, const int32_t *, const T *, int64_t, int, T *,  \
                                hipStream_t);                                                    \
  template void launch_transpose<T>(const T *, int64_t, int64_t, int64_t, T *, int64_t,          \
                                    hipStream_t);                                                \
  template void launch_combine<T>(const CombineArgs<T> &, int64_t, int, T *, int64_t, int64_t,   \
                                  hipStream_t);                                                  \
  template void launch_fill<T>(T *, int64_t, int64_t, int64_t, T, hipStream_t);

GVT_INSTANTIATE(double)
GVT_INSTANTIATE(float)

}  // namespace gvt
