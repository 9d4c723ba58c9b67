// Kernel ridge regression by conjugate gradients (Section 3, eq. (1)):
//   (R K R^T + lambda_l I) a_l = y,   l < nlam.
// All lambda systems share one operator; their search directions are
// multiplied together as one multi-RHS product.  Vectors, inner products and
// step lengths are FP64; the product may run in FP32, in which case a system
// whose recurrence residual meets the tolerance is re-checked with an FP64
// product and restarted from its true residual if it has not really
// converged.  Reductions use a fixed grid and a fixed tree, so runs are
// bitwise reproducible.  The per-iteration scalar work stays on the device;
// the host only looks at the state every `check_every` iterations, and those
// iteration blocks are replayed from a captured HIP graph.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstdlib>
#include <cstring>

#include "plan.h"
#include "tuning.h"

namespace gvt {

static constexpr int RB = 256;   // reduction block size
static constexpr int RNB = 240;  // reduction grid (fixed for determinism)
static constexpr int CG_PF = 4;  // elements per thread loaded ahead of a fold
static_assert(RNB <= RB, "partials are folded by one block");

enum CgState { CG_DONE = 0, CG_ACTIVE = 1, CG_PENDING = 2, CG_BREAKDOWN = 3, CG_MAXITER = 4 };

struct CgScalars {
  double rho, pw, alpha, beta, ynorm;
  double rho_prev;  // the rho the last update step used
  int state, iters;
  int gate;         // last update step: 0 system not active, 1 stepped, 2 breakdown (p.w <= 0)
  int extra;        // iterations granted beyond max_iter (the FP64 finish of an FP32-product solve)
};

// Sum over the block in a fixed order: a butterfly inside each wave (every
// lane ends with the same value, since a + b == b + a exactly), then the four
// wave sums in order.  One barrier instead of one per tree level.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  static_assert(RB == 256, "four waves per block");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// partial[b*nlam + l] = sum over this block's strided range of x_l . y_l
__global__ __launch_bounds__(RB) void dot_partial_kernel(const double *__restrict__ X, int64_t ldx,
                                                         const double *__restrict__ Y, int64_t ldy,
                                                         int64_t n, int nlam,
                                                         double *__restrict__ partial) {
  __shared__ double sh[RB];
  for (int l = 0; l < nlam; ++l) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)RNB * RB)
      acc += X[i + l * ldx] * Y[i + l * ldy];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x * nlam + l] = s;
  }
}

// Fixed-order fold of the RNB block partials of system l by one 256-thread block.
__device__ __forceinline__ double fold_partials(const double *partial, int nlam, int l, double *sh) {
  const double v = threadIdx.x < RNB ? partial[threadIdx.x * nlam + l] : 0.0;
  return block_sum(v, sh);
}

// Per iteration the vector work is three kernels: p.w, then the update of a
// and r with alpha, then the new search direction with beta.  The step
// lengths come from block partials folded in a fixed order; instead of a
// kernel of its own, every block of the next kernel folds them itself (the
// same reads in the same order, so every block gets the same value) and
// block 0 records the scalars.  No kernel reads a scalar field that it also
// writes: the update writes alpha, p.w, rho_prev and gate, the direction
// kernel reads gate and rho_prev and writes rho, beta, iters and state.

// w = K p (+ FP32 product cast) + lambda p ; partial dot p.w.  The update
// kernel recomputes w the same way rather than reading it back.
template <class TW>
__device__ __forceinline__ double cg_w(const TW *wraw, const double *p, double lm, int64_t i) {
  return (double)wraw[i] + lm * p[i];
}

template <class TW>
__global__ __launch_bounds__(RB) void cg_pw_kernel(const TW *__restrict__ wraw,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ lam, int64_t n,
                                                   int nlam, const CgScalars *__restrict__ sc,
                                                   double *__restrict__ partial) {
  __shared__ double sh[RB];
  for (int l = 0; l < nlam; ++l) {
    double acc = 0.0;
    if (sc[l].state == CG_ACTIVE) {
      const double lm = lam[l];
      // a few elements per thread: unrolled so that their loads are in flight together
#pragma unroll 4
      for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)RNB * RB)
        acc += p[i + l * n] * cg_w(wraw, p, lm, i + l * n);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x * nlam + l] = s;
  }
}

// alpha = rho / p.w; a += alpha p; r -= alpha w; partial r.r
template <class TW>
__global__ __launch_bounds__(RB) void cg_update_kernel(double *__restrict__ a, int64_t lda,
                                                       double *__restrict__ r,
                                                       const double *__restrict__ p,
                                                       const TW *__restrict__ wraw,
                                                       const double *__restrict__ lam, int64_t n,
                                                       int nlam, CgScalars *sc,
                                                       const double *__restrict__ part_pw,
                                                       double *__restrict__ part_rr) {
  __shared__ double sh[RB];
  const bool rec = blockIdx.x == 0 && threadIdx.x == 0;
  for (int l = 0; l < nlam; ++l) {
    double acc = 0.0;
    if (sc[l].state == CG_ACTIVE) {  // uniform: state is not written by this kernel
      // this thread's first CG_PF elements are loaded before the fold, so the two
      // round trips to memory overlap; the sums keep their element order
      const int64_t i0 = (int64_t)blockIdx.x * RB + threadIdx.x, st = (int64_t)RNB * RB;
      double pa[CG_PF], pp[CG_PF], pr[CG_PF], pwr[CG_PF];
#pragma unroll
      for (int k = 0; k < CG_PF; ++k) {
        const int64_t i = i0 + k * st;
        if (i < n) {
          pa[k] = a[i + l * lda];
          pp[k] = p[i + l * n];
          pr[k] = r[i + l * n];
          pwr[k] = (double)wraw[i + l * n];
        }
      }
      const double pw = fold_partials(part_pw, nlam, l, sh);
      const double rho = sc[l].rho;
      const bool ok = pw > 0.0 && isfinite(pw);
      const double al = rho / pw;
      if (ok) {
        const double lm = lam[l];
#pragma unroll
        for (int k = 0; k < CG_PF; ++k) {
          const int64_t i = i0 + k * st;
          if (i < n) {
            a[i + l * lda] = pa[k] + al * pp[k];
            const double ri = pr[k] - al * (pwr[k] + lm * pp[k]);
            r[i + l * n] = ri;
            acc += ri * ri;
          }
        }
        for (int64_t i = i0 + CG_PF * st; i < n; i += st) {
          a[i + l * lda] += al * p[i + l * n];
          const double ri = r[i + l * n] - al * cg_w(wraw, p, lm, i + l * n);
          r[i + l * n] = ri;
          acc += ri * ri;
        }
      }
      if (rec) {
        sc[l].pw = pw;
        sc[l].alpha = al;
        sc[l].rho_prev = rho;
        sc[l].gate = ok ? 1 : 2;
      }
    } else if (rec) {
      sc[l].gate = 0;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x * nlam + l] = s;
  }
}

// beta = rho_new / rho; p = r + beta p (and its FP32 copy p32, if given) for
// systems that stepped; block 0 advances iters, rho and the state, and sets
// *run to whether any system is still active (the next product's gate).  A
// system that has just stopped gets its p updated too; nothing reads it
// afterwards (a restart sets p again).  With pack targets (vs[k] non-null)
// the new p also goes straight into the key order the next product reads
// (element (i, l) to vs[k][inv[k][i] * nlam + l]), which saves that product
// its pack.
template <class TV> struct PackTo {
  TV *vs[2];
  const int32_t *inv[2];
};

template <class TV>
__global__ __launch_bounds__(RB) void cg_p_kernel(double *__restrict__ p, float *__restrict__ p32,
                                                  const double *__restrict__ r, int64_t n, int nlam,
                                                  CgScalars *sc, const double *__restrict__ part_rr,
                                                  double tol, int max_iter, int lowprec,
                                                  int *__restrict__ run, PackTo<TV> pk) {
  __shared__ double sh[RB];
  const bool rec = blockIdx.x == 0 && threadIdx.x == 0;
  for (int l = 0; l < nlam; ++l) {
    const int gate = sc[l].gate;  // uniform: written only by the update kernel
    if (gate == 0) continue;
    if (gate == 2) {
      if (rec) sc[l].state = CG_BREAKDOWN;
      continue;
    }
    TV *__restrict__ vs0 = pk.vs[0];
    TV *__restrict__ vs1 = pk.vs[1];
    const int32_t *__restrict__ inv0 = pk.inv[0];
    const int32_t *__restrict__ inv1 = pk.inv[1];
    // as in the update: the first CG_PF elements' loads overlap the fold
    const int64_t i0 = (int64_t)blockIdx.x * RB + threadIdx.x, st = (int64_t)RNB * RB;
    double qr[CG_PF], qp[CG_PF];
    int32_t q0[CG_PF], q1[CG_PF];
#pragma unroll
    for (int k = 0; k < CG_PF; ++k) {
      const int64_t i = i0 + k * st;
      if (i < n) {
        qr[k] = r[i + l * n];
        qp[k] = p[i + l * n];
        q0[k] = vs0 ? inv0[i] : 0;
        q1[k] = vs1 ? inv1[i] : 0;
      }
    }
    const double rho_new = fold_partials(part_rr, nlam, l, sh);
    const double beta = rho_new / sc[l].rho_prev;
    if (isfinite(rho_new)) {
#pragma unroll
      for (int k = 0; k < CG_PF; ++k) {
        const int64_t i = i0 + k * st;
        if (i < n) {
          const double pi = qr[k] + beta * qp[k];
          p[i + l * n] = pi;
          if (p32) p32[i + l * n] = (float)pi;
          if (vs0) vs0[(int64_t)q0[k] * nlam + l] = (TV)pi;
          if (vs1) vs1[(int64_t)q1[k] * nlam + l] = (TV)pi;
        }
      }
      for (int64_t i = i0 + CG_PF * st; i < n; i += st) {
        const double pi = r[i + l * n] + beta * p[i + l * n];
        p[i + l * n] = pi;
        if (p32) p32[i + l * n] = (float)pi;
        if (vs0) vs0[(int64_t)inv0[i] * nlam + l] = (TV)pi;
        if (vs1) vs1[(int64_t)inv1[i] * nlam + l] = (TV)pi;
      }
    }
    if (rec) {
      sc[l].iters += 1;
      if (!isfinite(rho_new)) {
        sc[l].state = CG_BREAKDOWN;
      } else {
        sc[l].beta = beta;
        sc[l].rho = rho_new;
        if (sqrt(rho_new) / sc[l].ynorm < tol)
          sc[l].state = lowprec ? CG_PENDING : CG_DONE;
        else if (sc[l].iters >= max_iter + sc[l].extra)
          sc[l].state = CG_MAXITER;
      }
    }
  }
  if (rec) {
    int any = 0;
    for (int l = 0; l < nlam; ++l) any |= sc[l].state == CG_ACTIVE;
    *run = any;
  }
}

// Initial per-system state from ||y||^2 (ynorm2) and the starting r.r (rho0,
// or ||y||^2 for every system when rho0 is null); *run = any system active.
__global__ void cg_init_kernel(CgScalars *sc, const double *__restrict__ ynorm2,
                               const double *__restrict__ rho0, int nlam, double tol,
                               int *__restrict__ run) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double yn = sqrt(*ynorm2);
  int any = 0;
  for (int l = 0; l < nlam; ++l) {
    CgScalars c;
    c.pw = c.alpha = c.beta = c.rho_prev = 0.0;
    c.iters = c.gate = c.extra = 0;
    // all-zero labels: residuals are measured against 1 (a = 0 solves the system)
    c.ynorm = yn == 0.0 ? 1.0 : yn;
    c.rho = rho0 ? rho0[l] : *ynorm2;
    c.state = !isfinite(yn) ? CG_BREAKDOWN : (sqrt(c.rho) / c.ynorm < tol ? CG_DONE : CG_ACTIVE);
    any |= c.state == CG_ACTIVE;
    sc[l] = c;
  }
  *run = any;
}

// r = y - (wraw + lambda a)  (true residual after an FP64 product w = K a); partial r.r
__global__ __launch_bounds__(RB) void residual_kernel(const double *__restrict__ y,
                                                      const double *__restrict__ wraw,
                                                      const double *__restrict__ a, int64_t lda,
                                                      const double *__restrict__ lam, int64_t n,
                                                      int nlam, double *__restrict__ r,
                                                      double *__restrict__ partial) {
  __shared__ double sh[RB];
  for (int l = 0; l < nlam; ++l) {
    double acc = 0.0;
    const double lm = lam[l];
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)RNB * RB) {
      const double ri = y[i] - (wraw[i + l * n] + lm * a[i + l * lda]);
      r[i + l * n] = ri;
      acc += ri * ri;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x * nlam + l] = s;
  }
}

// fold partials into out[l] (one block per system)
__global__ __launch_bounds__(RB) void fold_kernel(const double *__restrict__ partial, int nlam,
                                                  double *__restrict__ out) {
  __shared__ double sh[RB];
  const int l = blockIdx.x;
  const double v = fold_partials(partial, nlam, l, sh);
  if (threadIdx.x == 0) out[l] = v;
}

__global__ void copy_cols_kernel(const double *__restrict__ src, int64_t lds, double *__restrict__ dst,
                                 int64_t ldd, int64_t n, int nlam, int only_state,
                                 const CgScalars *__restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int l = 0; l < nlam; ++l)
    if (only_state < 0 || (sc && sc[l].state == only_state)) dst[i + l * ldd] = src[i + l * lds];
}

// p = w + beta (p - r); r = w (one system: the residual replaced by the true one
// w, the search continuing along the last direction)
__global__ void axpy_dir_kernel(const double *__restrict__ w, double *__restrict__ r, double *__restrict__ p,
                                double beta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = w[i] + beta * (p[i] - r[i]);
  r[i] = w[i];
}

__global__ void bcast_col_kernel(const double *__restrict__ y, double *__restrict__ dst, int64_t ldd,
                                 int64_t n, int nlam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int l = 0; l < nlam; ++l) dst[i + l * ldd] = y[i];
}

__global__ void to_f32_kernel(const double *__restrict__ x, float *__restrict__ y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = (float)x[i];
}

// FP32 copy of a base matrix with row stride ldy >= cols; the padding columns
// are written as zeros.
__global__ void mat_to_f32_kernel(const double *__restrict__ x, int64_t ldx, float *__restrict__ y,
                                  int64_t ldy, int64_t rows, int64_t cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ldy) return;
  const int64_t r = idx / ldy, c = idx - r * ldy;
  y[idx] = c < cols ? (float)x[r * ldx + c] : 0.0f;
}

// Row stride of the FP32 copies: whole 64-byte lines, so that every row starts
// on a 16-byte boundary and the stage-2 kernels stage F1 in vector pieces.
inline int64_t f32_copy_ld(int64_t cols) { return (cols + 15) / 16 * 16; }

// ---------------------------------------------------------------------------
namespace {

struct CgRun {
  gvt_plan *plan = nullptr;
  ~CgRun() {
    if (plan) {
      if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
      delete plan;
    }
  }
};

}  // namespace

static dim3 g1(int64_t n) { return dim3((unsigned)ceil_div(n, 256)); }

int krr_cg_impl(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                const double *lambdas, int nlam, double *A, int64_t lda, const double *A0,
                int64_t lda0, int max_iter, double tol, int mprec, int check_every,
                int64_t *iters_out, double *relres_out, hipStream_t s) {
  GVT_REQUIRE(n >= 1 && nlam >= 1 && nlam <= 64, GVT_ERR_ARG, "need n >= 1 and 1 <= nlam <= 64");
  GVT_REQUIRE(D && c && e && y && lambdas && A && iters_out && relres_out, GVT_ERR_ARG, "null argument");
  GVT_REQUIRE(lda >= n && (!A0 || lda0 >= n), GVT_ERR_ARG, "lda < n");
  GVT_REQUIRE(max_iter >= 1 && tol > 0 && check_every >= 1, GVT_ERR_ARG, "bad max_iter/tol/check_every");
  GVT_REQUIRE(mprec == GVT_F64 || mprec == GVT_F32, GVT_ERR_UNSUPPORTED,
              "CG products run in GVT_F64 or GVT_F32");
  for (int l = 0; l < nlam; ++l)
    GVT_REQUIRE(lambdas[l] > 0 && std::isfinite(lambdas[l]), GVT_ERR_ARG, "lambda must be > 0");
  const bool hom = kind == GVT_SYMMETRIC || kind == GVT_ANTISYMMETRIC || kind == GVT_RANKING ||
                   kind == GVT_MLPK;
  if (hom) { T = D; t = d; ldt = ldd; }
  GVT_REQUIRE(T, GVT_ERR_ARG, "null T");
  GVT_REQUIRE(ldd >= d && ldt >= t, GVT_ERR_ARG, "ld < cols");

  CgRun run;
  run.plan = new gvt_plan();
  gvt_plan *P = run.plan;
  plan_build(P, &kind, 1, d, d, t, t, c, e, n, c, e, n, GVT_FLAG_SYMMETRIC_BASES, s, nlam);
  GVT_REQUIRE(!P->dense, GVT_ERR_UNSUPPORTED, "complete-data training grid: use the dense product");

  // workspace
  DevMem m_r, m_p, m_w, m_wraw, m_p32, m_w32, m_D32, m_T32, m_part, m_sc, m_lam, m_tmp;
  const size_t nv = (size_t)n * nlam;
  double *r = (double *)m_r.ensure(nv * 8);
  double *p = (double *)m_p.ensure(nv * 8);
  double *w = (double *)m_w.ensure(nv * 8);
  double *wraw = (double *)m_wraw.ensure(nv * 8);
  double *part = (double *)m_part.ensure((size_t)RNB * nlam * 8 * 2);
  double *part2 = part + (size_t)RNB * nlam;  // r.r partials (part holds p.w)
  CgScalars *sc = (CgScalars *)m_sc.ensure(sizeof(CgScalars) * nlam);
  double *lam = (double *)m_lam.ensure(nlam * 8);
  // tmp: up to 65 fold results (||y||^2, then one per system); the products' run flag after them
  double *tmp = (double *)m_tmp.ensure(128 * 8 + 256);
  int *gate = reinterpret_cast<int *>(tmp + 128);  // run flag of the iteration products
  float *p32 = nullptr, *w32 = nullptr, *D32 = nullptr, *T32 = nullptr;
  const int64_t ldd32 = f32_copy_ld(d), ldt32 = hom ? ldd32 : f32_copy_ld(t);
  GVT_HIP_CHECK(hipMemcpyAsync(lam, lambdas, nlam * 8, hipMemcpyHostToDevice, s));
  if (mprec == GVT_F32) {
    p32 = (float *)m_p32.ensure(nv * 4);
    w32 = (float *)m_w32.ensure(nv * 4);
    D32 = (float *)m_D32.ensure((size_t)d * ldd32 * 4);
    mat_to_f32_kernel<<<g1(d * ldd32), 256, 0, s>>>(D, ldd, D32, ldd32, d, d);
    if (!hom) {
      T32 = (float *)m_T32.ensure((size_t)t * ldt32 * 4);
      mat_to_f32_kernel<<<g1(t * ldt32), 256, 0, s>>>(T, ldt, T32, ldt32, t, t);
    } else {
      T32 = D32;
    }
  }
  auto matvec64 = [&](const double *X, double *Y) {
    plan_execute(P, GVT_F64, D, ldd, T, ldt, X, nlam, n, Y, n, s);
  };

  // ||y||^2 into tmp[0]
  dot_partial_kernel<<<RNB, RB, 0, s>>>(y, 0, y, 0, n, 1, part);
  fold_kernel<<<1, RB, 0, s>>>(part, 1, tmp);

  // init: a = A0 or 0; r = y - (K + lambda) a; p = r; rho = r.r.  The states
  // are set on the device; the host first reads them after the first block
  // of iterations (until then it takes every system to be active).
  std::vector<CgScalars> hs(nlam);
  if (A0) {
    copy_cols_kernel<<<g1(n), 256, 0, s>>>(A0, lda0, A, lda, n, nlam, -1, nullptr);
  } else {
    for (int l = 0; l < nlam; ++l) GVT_HIP_CHECK(hipMemsetAsync(A + l * lda, 0, n * 8, s));
  }
  if (A0) {
    // true residual of the initial guess needs a contiguous copy of A
    double *acopy = p;
    copy_cols_kernel<<<g1(n), 256, 0, s>>>(A, lda, acopy, n, n, nlam, -1, nullptr);
    matvec64(acopy, wraw);
    residual_kernel<<<RNB, RB, 0, s>>>(y, wraw, A, lda, lam, n, nlam, r, part);
    fold_kernel<<<nlam, RB, 0, s>>>(part, nlam, tmp + 1);
  } else {
    // r = y for every system: its r.r is ||y||^2, summed above in the same order
    bcast_col_kernel<<<g1(n), 256, 0, s>>>(y, r, n, n, nlam);
  }
  copy_cols_kernel<<<g1(n), 256, 0, s>>>(r, n, p, n, n, nlam, -1, nullptr);
  cg_init_kernel<<<1, 64, 0, s>>>(sc, tmp, A0 ? tmp + 1 : nullptr, nlam, tol, gate);
  for (int l = 0; l < nlam; ++l) {
    std::memset(&hs[l], 0, sizeof(CgScalars));
    hs[l].state = CG_ACTIVE;
  }

  // lowprec: FP32 products.  When a system's FP32 recurrence reaches tol but
  // its true residual does not, the rest of the solve runs FP64 products
  // (R13(i): a system that converges with FP64 products must converge here).
  int lowprec = mprec == GVT_F32 ? 1 : 0;
  // p32 (FP32 products) is kept in step with p by the direction kernel; after
  // the host sets p (start, restart) it is refreshed here
  auto refresh_p32 = [&]() {
    if (lowprec) to_f32_kernel<<<g1((int64_t)nv), 256, 0, s>>>(p, p32, (int64_t)nv);
  };
  refresh_p32();
  // When the nlam systems form one RHS block of the plan, the direction kernel
  // writes p in the key order of the iteration products as well, and those
  // products skip their pack; after the host sets p it is packed here.
  int iprec = GVT_F64;
  bool fuse_pack = false;
  PackTo<double> pk64{{nullptr, nullptr}, {nullptr, nullptr}};
  PackTo<float> pk32{{nullptr, nullptr}, {nullptr, nullptr}};
  auto setup_pack = [&]() {
    iprec = lowprec ? GVT_F32 : GVT_F64;
    fuse_pack = rhs_block(nlam, rhs_cap(P, iprec)) == nlam;
    pk64 = PackTo<double>{{nullptr, nullptr}, {nullptr, nullptr}};
    pk32 = PackTo<float>{{nullptr, nullptr}, {nullptr, nullptr}};
    if (!fuse_pack) return;
    void *vs[2] = {nullptr, nullptr};
    const int32_t *inv[2] = {nullptr, nullptr};
    const int nk = plan_pack_targets(P, iprec, nlam, vs, inv);
    for (int k = 0; k < nk; ++k) {
      if (lowprec) {
        pk32.vs[k] = static_cast<float *>(vs[k]);
        pk32.inv[k] = inv[k];
      } else {
        pk64.vs[k] = static_cast<double *>(vs[k]);
        pk64.inv[k] = inv[k];
      }
    }
  };
  setup_pack();
  auto repack = [&]() {
    if (fuse_pack) plan_pack(P, iprec, lowprec ? (const void *)p32 : (const void *)p, n, nlam, s);
  };
  // Products inside iterations are gated by `gate`: once every system has
  // stopped, the rest of a captured block of iterations skips its products.
  // Products outside iterations (certification, final residual) always run.
  bool packed = false;  // whether the key-ordered copy of p is current
  auto iteration = [&]() {
    P->gate = gate;
    P->prepacked = fuse_pack && packed;
    if (lowprec) {
      plan_execute(P, GVT_F32, D32, ldd32, T32, ldt32, p32, nlam, n, w32, n, s);
      cg_pw_kernel<float><<<RNB, RB, 0, s>>>(w32, p, lam, n, nlam, sc, part);
      cg_update_kernel<float><<<RNB, RB, 0, s>>>(A, lda, r, p, w32, lam, n, nlam, sc, part, part2);
    } else {
      matvec64(p, wraw);
      cg_pw_kernel<double><<<RNB, RB, 0, s>>>(wraw, p, lam, n, nlam, sc, part);
      cg_update_kernel<double><<<RNB, RB, 0, s>>>(A, lda, r, p, wraw, lam, n, nlam, sc, part, part2);
    }
    P->prepacked = false;
    if (lowprec)
      cg_p_kernel<float><<<RNB, RB, 0, s>>>(p, p32, r, n, nlam, sc, part2, tol, max_iter, lowprec, gate, pk32);
    else
      cg_p_kernel<double><<<RNB, RB, 0, s>>>(p, p32, r, n, nlam, sc, part2, tol, max_iter, lowprec, gate, pk64);
    packed = true;
    P->gate = nullptr;
  };

  // warm-up layout of plan workspaces (allocation must not happen inside a capture)
  // by running one iteration eagerly, then capture blocks of check_every iterations.
  // graphs need a capturable (non-null) stream
  const bool use_graph = s != nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;  // capture stream (default priority)
  struct CapStream {
    hipStream_t &c;
    ~CapStream() {
      if (c) (void)hipStreamDestroy(c);
    }
  } cap_guard{cap};
  int status = GVT_OK;
  int total_iter = 0;
  bool first = true;
  while (true) {
    bool any_active = false;
    for (int l = 0; l < nlam; ++l) any_active |= hs[l].state == CG_ACTIVE;
    if (!any_active) {
      // certify systems whose low-precision recurrence claims convergence, and
      // (FP32 products) systems at the iteration cap, which get the FP64 finish
      bool pending = false;
      for (int l = 0; l < nlam; ++l)
        pending |= hs[l].state == CG_PENDING ||
                   (lowprec && hs[l].state == CG_MAXITER && hs[l].extra == 0);
      if (!pending) break;
      bool finish = false;
      copy_cols_kernel<<<g1(n), 256, 0, s>>>(A, lda, w, n, n, nlam, -1, nullptr);
      matvec64(w, wraw);
      residual_kernel<<<RNB, RB, 0, s>>>(y, wraw, A, lda, lam, n, nlam, w, part);
      fold_kernel<<<nlam, RB, 0, s>>>(part, nlam, tmp);
      std::vector<double> rt(nlam);
      GVT_HIP_CHECK(hipMemcpyAsync(rt.data(), tmp, nlam * 8, hipMemcpyDeviceToHost, s));
      GVT_HIP_CHECK(hipStreamSynchronize(s));
      const bool was_low = lowprec != 0;
      std::vector<uint8_t> keep_dir(nlam, 0);
      for (int l = 0; l < nlam; ++l) {
        const bool capped = was_low && hs[l].state == CG_MAXITER && hs[l].extra == 0;
        if (hs[l].state != CG_PENDING && !capped) continue;
        if (std::sqrt(rt[l]) / hs[l].ynorm < tol) {
          hs[l].state = CG_DONE;
        } else if (capped) {
          // FP64 finish: at most max_iter / 10 more iterations with FP64
          // products, the residual replaced by the true one and the search
          // continuing along the last direction
          hs[l].state = CG_ACTIVE;
          hs[l].extra = std::max(1, max_iter / 10);
          const double be = rt[l] / hs[l].rho;
          hs[l].beta = std::isfinite(be) ? be : 0.0;
          hs[l].rho = rt[l];
          keep_dir[l] = 1;
          finish = true;
        } else if (hs[l].iters >= max_iter + hs[l].extra) {
          hs[l].state = CG_MAXITER;
        } else {
          hs[l].state = CG_ACTIVE;  // restart from the true residual
          hs[l].rho = rt[l];
          finish = true;
        }
      }
      if (finish && lowprec) {
        // FP32 products could not carry a system to tol: FP64 products from
        // here, with the iteration block captured again
        lowprec = 0;
        setup_pack();
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        first = true;
      }
      // restarted systems: r = w (true residual), p = r; finishing systems:
      // p = w + beta (p - r), r = w
      GVT_HIP_CHECK(hipMemcpyAsync(sc, hs.data(), sizeof(CgScalars) * nlam, hipMemcpyHostToDevice, s));
      for (int l = 0; l < nlam; ++l) {
        if (hs[l].state != CG_ACTIVE) continue;
        double *pl = p + (int64_t)l * n, *rl = r + (int64_t)l * n;
        const double *wl = w + (int64_t)l * n;
        if (keep_dir[l]) {
          axpy_dir_kernel<<<g1(n), 256, 0, s>>>(wl, rl, pl, hs[l].beta, n);
        } else {
          GVT_HIP_CHECK(hipMemcpyAsync(rl, wl, n * 8, hipMemcpyDeviceToDevice, s));
          GVT_HIP_CHECK(hipMemcpyAsync(pl, wl, n * 8, hipMemcpyDeviceToDevice, s));
        }
      }
      refresh_p32();
      repack();
      GVT_HIP_CHECK(hipMemsetD32Async(gate, 1, 1, s));
      continue;
    }
    if (first) {
      // one eager iteration lays out every workspace (no allocation may happen
      // inside a capture); then capture a block of check_every iterations
      iteration();
      ++total_iter;
      first = false;
      if (use_graph) {
        // the first block also runs eagerly on s, and while the device works
        // through it the same block is captured on a stream of the solve's own
        // (a graph holds kernels and arguments, not a stream) and instantiated;
        // the iterations run as before, the host checks after this block
        for (int k = 0; k < check_every; ++k) iteration();
        total_iter += check_every;
        if (!cap) GVT_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        const hipStream_t run_s = s;
        s = cap;  // the iteration's launches follow s
        GVT_HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
          for (int k = 0; k < check_every; ++k) iteration();
        } catch (...) {
          s = run_s;
          P->last_stream = run_s;
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cap, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        s = run_s;
        P->last_stream = run_s;
        GVT_HIP_CHECK(hipStreamEndCapture(cap, &graph));
        GVT_HIP_CHECK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      }
    } else if (use_graph) {
      GVT_HIP_CHECK(hipGraphLaunch(gexec, s));
      total_iter += check_every;
    } else {
      for (int k = 0; k < check_every; ++k) iteration();
      total_iter += check_every;
    }
    GVT_HIP_CHECK(hipMemcpyAsync(hs.data(), sc, sizeof(CgScalars) * nlam, hipMemcpyDeviceToHost, s));
    GVT_HIP_CHECK(hipStreamSynchronize(s));
    for (int l = 0; l < nlam; ++l)
      if (hs[l].state == CG_BREAKDOWN) status = GVT_ERR_BREAKDOWN;
    if (status != GVT_OK) break;
    if (total_iter > 4 * max_iter + 8) break;  // safety net; states already cap iterations
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);

  // final true residuals with an FP64 product
  copy_cols_kernel<<<g1(n), 256, 0, s>>>(A, lda, w, n, n, nlam, -1, nullptr);
  matvec64(w, wraw);
  residual_kernel<<<RNB, RB, 0, s>>>(y, wraw, A, lda, lam, n, nlam, r, part);
  fold_kernel<<<nlam, RB, 0, s>>>(part, nlam, tmp);
  std::vector<double> rt(nlam);
  GVT_HIP_CHECK(hipMemcpyAsync(rt.data(), tmp, nlam * 8, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipMemcpyAsync(hs.data(), sc, sizeof(CgScalars) * nlam, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  check_launch(s);
  GVT_REQUIRE(std::isfinite(hs[0].ynorm), GVT_ERR_BREAKDOWN, "non-finite labels");
  bool all_done = true;
  for (int l = 0; l < nlam; ++l) {
    iters_out[l] = hs[l].iters;
    relres_out[l] = std::sqrt(rt[l]) / hs[l].ynorm;
    if (hs[l].state == CG_BREAKDOWN) status = GVT_ERR_BREAKDOWN;
    if (hs[l].state != CG_DONE) all_done = false;
  }
  if (status == GVT_OK && !all_done) status = GVT_NOT_CONVERGED;
  return status;
}

// ===========================================================================
// Many independent ridge problems, each with its own base kernels, pairs and
// labels, solved together for one grid of lambdas.  One set of CG vectors
// holds every problem's nlam systems back to back (problem p, system l at
// voff_p + l * n_p); the vector kernels walk fixed chunks that each belong to
// one system, and per-system sums fold the chunk partials in a fixed order,
// so results are reproducible.  The products of all problems run as grouped
// launches (one launch per stage covers every problem's blocks, largest
// problems first), problems whose systems have all stopped are skipped by a
// device-side mask, and blocks of iterations are replayed from a HIP graph.
// ===========================================================================
static constexpr int BCH = 4096;  // elements per chunk

struct BChunk {
  int64_t start;  // element offset in the concatenated vectors
  int64_t yoff;   // offset of the chunk's first pair in the concatenated labels
  int32_t sys;    // system index = problem * nlam + lambda index
  int32_t len;
};

// fold the chunk partials [c0, c1) of one system in a fixed order
__device__ __forceinline__ double fold_range(const double *part, int64_t c0, int64_t c1, double *sh) {
  double v = 0.0;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += RB) v += part[c];
  return block_sum(v, sh);
}

// w = wraw + lambda p; partial p.w
template <class TW>
__global__ __launch_bounds__(RB) void bcg_pw_kernel(const BChunk *__restrict__ ch,
                                                    const TW *__restrict__ wraw, double *__restrict__ w,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ lam, int nlam,
                                                    const CgScalars *__restrict__ sc,
                                                    double *__restrict__ part) {
  __shared__ double sh[RB];
  const BChunk c = ch[blockIdx.x];
  double acc = 0.0;
  if (sc[c.sys].state == CG_ACTIVE) {  // uniform per block
    const double lm = lam[c.sys % nlam];
    for (int i = threadIdx.x; i < c.len; i += RB) {
      const int64_t g = c.start + i;
      const double pi = p[g];
      const double wi = (double)wraw[g] + lm * pi;
      w[g] = wi;
      acc += pi * wi;
    }
  }
  const double v = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// p.w with each problem's product in FP32 (w32) or, once switched (hi), FP64 (w64)
__global__ __launch_bounds__(RB) void bcg_pw_mixed_kernel(const BChunk *__restrict__ ch,
                                                          const float *__restrict__ w32,
                                                          const double *__restrict__ w64,
                                                          const uint8_t *__restrict__ hi, double *__restrict__ w,
                                                          const double *__restrict__ p,
                                                          const double *__restrict__ lam, int nlam,
                                                          const CgScalars *__restrict__ sc,
                                                          double *__restrict__ part) {
  __shared__ double sh[RB];
  const BChunk c = ch[blockIdx.x];
  double acc = 0.0;
  if (sc[c.sys].state == CG_ACTIVE) {  // uniform per block
    const double lm = lam[c.sys % nlam];
    const bool h = hi[c.sys / nlam] != 0;
    for (int i = threadIdx.x; i < c.len; i += RB) {
      const int64_t g = c.start + i;
      const double pi = p[g];
      const double wi = (h ? w64[g] : (double)w32[g]) + lm * pi;
      w[g] = wi;
      acc += pi * wi;
    }
  }
  const double v = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(RB) void bcg_alpha_kernel(CgScalars *sc, const double *__restrict__ part,
                                                       const int64_t *__restrict__ cfirst) {
  __shared__ double sh[RB];
  const int sy = blockIdx.x;
  if (sc[sy].state != CG_ACTIVE) return;  // uniform per block
  const double pw = fold_range(part, cfirst[sy], cfirst[sy + 1], sh);
  if (threadIdx.x != 0) return;
  sc[sy].pw = pw;
  if (!(pw > 0.0) || !isfinite(pw)) {
    sc[sy].state = CG_BREAKDOWN;
    return;
  }
  sc[sy].alpha = sc[sy].rho / pw;
}

// a += alpha p; r -= alpha w; partial r.r
__global__ __launch_bounds__(RB) void bcg_update_kernel(const BChunk *__restrict__ ch,
                                                        double *__restrict__ a, double *__restrict__ r,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ w,
                                                        const CgScalars *__restrict__ sc,
                                                        double *__restrict__ part) {
  __shared__ double sh[RB];
  const BChunk c = ch[blockIdx.x];
  double acc = 0.0;
  if (sc[c.sys].state == CG_ACTIVE) {
    const double al = sc[c.sys].alpha;
    for (int i = threadIdx.x; i < c.len; i += RB) {
      const int64_t g = c.start + i;
      a[g] += al * p[g];
      const double ri = r[g] - al * w[g];
      r[g] = ri;
      acc += ri * ri;
    }
  }
  const double v = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(RB) void bcg_beta_kernel(CgScalars *sc, const double *__restrict__ part,
                                                      const int64_t *__restrict__ cfirst, double tol,
                                                      int max_iter, int lowprec) {
  __shared__ double sh[RB];
  const int sy = blockIdx.x;
  if (sc[sy].state != CG_ACTIVE) return;  // uniform per block
  const double rho_new = fold_range(part, cfirst[sy], cfirst[sy + 1], sh);
  if (threadIdx.x != 0) return;
  sc[sy].iters += 1;
  if (!isfinite(rho_new)) {
    sc[sy].state = CG_BREAKDOWN;
    return;
  }
  sc[sy].beta = rho_new / sc[sy].rho;
  sc[sy].rho = rho_new;
  if (sqrt(rho_new) / sc[sy].ynorm < tol) {
    sc[sy].state = lowprec ? CG_PENDING : CG_DONE;
  } else if (sc[sy].iters >= max_iter + sc[sy].extra) {
    sc[sy].state = CG_MAXITER;
  }
}

// p = r + beta p (active systems)
__global__ __launch_bounds__(RB) void bcg_p_kernel(const BChunk *__restrict__ ch, double *__restrict__ p,
                                                   const double *__restrict__ r,
                                                   const CgScalars *__restrict__ sc) {
  const BChunk c = ch[blockIdx.x];
  if (sc[c.sys].state != CG_ACTIVE) return;
  const double be = sc[c.sys].beta;
  for (int i = threadIdx.x; i < c.len; i += RB) {
    const int64_t g = c.start + i;
    p[g] = r[g] + be * p[g];
  }
}

// Systems set active again after a certification: r = w (the true residual),
// and p = w (restart) or, with keep[sys], p = w + beta p (the FP64 finish,
// continuing along the last direction)
__global__ __launch_bounds__(RB) void bcg_reactivate_kernel(const BChunk *__restrict__ ch,
                                                            const double *__restrict__ w, double *__restrict__ r,
                                                            double *__restrict__ p,
                                                            const CgScalars *__restrict__ sc,
                                                            const uint8_t *__restrict__ keep) {
  const BChunk c = ch[blockIdx.x];
  if (sc[c.sys].state != CG_ACTIVE) return;
  const double be = keep[c.sys] ? sc[c.sys].beta : 0.0;
  for (int i = threadIdx.x; i < c.len; i += RB) {
    const int64_t g = c.start + i;
    const double wi = w[g];
    p[g] = be != 0.0 ? wi + be * p[g] : wi;
    r[g] = wi;
  }
}

// Masks of the iteration products per RHS block: the grouped products run
// the systems of a problem in blocks of RHS (the block layout of each product
// precision, block b = systems [start[b], start[b + 1])), and a block whose
// systems have all stopped costs no product work.
struct BlockMasks {
  const int32_t *start64, *start32;  // block starts (nb + 1 entries) of the FP64 / FP32 layouts
  int nb64, nb32;
  uint8_t *bm64, *bm32;  // [b * nprob + p]; null: not kept
};

// active[p] = some system of problem p is still iterating; with hi (FP32
// mode) also the active problems by product precision: act32 = active and not
// hi, act64 = active and hi.  Per RHS block (bm): bm64 = the block has an
// active system and the problem is on FP64 products (every problem in FP64
// mode, hi null); bm32 = the block has an active system and the problem is
// still on FP32 products.
__global__ void bcg_mask_kernel(const CgScalars *__restrict__ sc, int nprob, int nlam,
                                uint8_t *__restrict__ active, const uint8_t *__restrict__ hi,
                                uint8_t *__restrict__ act32, uint8_t *__restrict__ act64, BlockMasks bm) {
  const int pb = blockIdx.x * blockDim.x + threadIdx.x;
  if (pb >= nprob) return;
  uint8_t any = 0;
  for (int l = 0; l < nlam; ++l) any |= sc[pb * nlam + l].state == CG_ACTIVE ? 1 : 0;
  active[pb] = any;
  if (hi) {
    act32[pb] = any && !hi[pb];
    act64[pb] = any && hi[pb];
  }
  auto block_any = [&](int l0, int l1) {
    uint8_t a = 0;
    for (int l = l0; l < l1; ++l) a |= sc[pb * nlam + l].state == CG_ACTIVE ? 1 : 0;
    return a;
  };
  if (bm.bm64) {
    const uint8_t on = hi ? hi[pb] : 1;
    for (int b = 0; b < bm.nb64; ++b)
      bm.bm64[(int64_t)b * nprob + pb] = on && block_any(bm.start64[b], bm.start64[b + 1]);
  }
  if (bm.bm32) {
    const uint8_t on = hi ? !hi[pb] : 0;
    for (int b = 0; b < bm.nb32; ++b)
      bm.bm32[(int64_t)b * nprob + pb] = on && block_any(bm.start32[b], bm.start32[b + 1]);
  }
}

// r = y (every system of a problem starts from its labels); partial r.r
__global__ __launch_bounds__(RB) void bcg_bcast_kernel(const BChunk *__restrict__ ch,
                                                       const double *__restrict__ y,
                                                       double *__restrict__ r,
                                                       double *__restrict__ part) {
  __shared__ double sh[RB];
  const BChunk c = ch[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < c.len; i += RB) {
    const double yi = y[c.yoff + i];
    r[c.start + i] = yi;
    acc += yi * yi;
  }
  const double v = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// out = y - (wraw + lambda a); partial out.out
__global__ __launch_bounds__(RB) void bcg_residual_kernel(const BChunk *__restrict__ ch,
                                                          const double *__restrict__ y,
                                                          const double *__restrict__ wraw,
                                                          const double *__restrict__ a,
                                                          const double *__restrict__ lam, int nlam,
                                                          double *__restrict__ out,
                                                          double *__restrict__ part) {
  __shared__ double sh[RB];
  const BChunk c = ch[blockIdx.x];
  const double lm = lam[c.sys % nlam];
  double acc = 0.0;
  for (int i = threadIdx.x; i < c.len; i += RB) {
    const int64_t g = c.start + i;
    const double ri = y[c.yoff + i] - (wraw[g] + lm * a[g]);
    out[g] = ri;
    acc += ri * ri;
  }
  const double v = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(RB) void bcg_fold_kernel(const double *__restrict__ part,
                                                      const int64_t *__restrict__ cfirst,
                                                      double *__restrict__ out) {
  __shared__ double sh[RB];
  const int sy = blockIdx.x;
  const double v = fold_range(part, cfirst[sy], cfirst[sy + 1], sh);
  if (threadIdx.x == 0) out[sy] = v;
}

// dst = src for the systems in `only_state` (every system when only_state < 0)
__global__ __launch_bounds__(RB) void bcg_copy_kernel(const BChunk *__restrict__ ch,
                                                      const double *__restrict__ src,
                                                      double *__restrict__ dst, int only_state,
                                                      const CgScalars *__restrict__ sc) {
  const BChunk c = ch[blockIdx.x];
  if (only_state >= 0 && sc[c.sys].state != only_state) return;
  for (int i = threadIdx.x; i < c.len; i += RB) dst[c.start + i] = src[c.start + i];
}

namespace {

struct PlanSet {
  std::vector<gvt_plan *> plans;
  hipStream_t s = nullptr;
  ~PlanSet() {
    if (!plans.empty()) (void)hipStreamSynchronize(s);
    for (gvt_plan *P : plans) delete P;
  }
};

}  // namespace

int krr_cg_batched_impl(int kind, const gvt_krr_problem *pr, int nprob, const double *lambdas,
                        int nlam, int max_iter, double tol, int mprec, int check_every,
                        int64_t *iters_out, double *relres_out, hipStream_t s) {
  GVT_REQUIRE(pr && lambdas && iters_out && relres_out, GVT_ERR_ARG, "null argument");
  GVT_REQUIRE(nprob >= 1 && nlam >= 1 && nlam <= 64, GVT_ERR_ARG, "need nprob >= 1 and 1 <= nlam <= 64");
  GVT_REQUIRE(max_iter >= 1 && tol > 0 && check_every >= 1, GVT_ERR_ARG, "bad max_iter/tol/check_every");
  GVT_REQUIRE(mprec == GVT_F64 || mprec == GVT_F32, GVT_ERR_UNSUPPORTED,
              "CG products run in GVT_F64 or GVT_F32");
  for (int l = 0; l < nlam; ++l)
    GVT_REQUIRE(lambdas[l] > 0 && std::isfinite(lambdas[l]), GVT_ERR_ARG, "lambda must be > 0");
  const bool hom = kind == GVT_SYMMETRIC || kind == GVT_ANTISYMMETRIC || kind == GVT_RANKING ||
                   kind == GVT_MLPK;

  // ---- per-problem plans and offsets
  struct Prob {
    const double *D, *T;
    int64_t d, t, ldd, ldt, n, noff, voff;
    float *D32, *T32;
    int64_t ldd32, ldt32;  // row strides of the FP32 copies
  };
  std::vector<Prob> pb(nprob);
  PlanSet ps;
  ps.s = s;
  int64_t ntot = 0;
  for (int i = 0; i < nprob; ++i) {
    const gvt_krr_problem &q = pr[i];
    Prob &b = pb[i];
    GVT_REQUIRE(q.D && q.c && q.e && q.y && q.A, GVT_ERR_ARG,
                "problem " + std::to_string(i) + ": null argument");
    GVT_REQUIRE(q.n >= 1 && q.lda >= q.n && (!q.A0 || q.lda0 >= q.n), GVT_ERR_ARG,
                "problem " + std::to_string(i) + ": need n >= 1 and lda, lda0 >= n");
    b.D = q.D;
    b.d = q.d;
    b.ldd = q.ldd;
    if (hom) {
      b.T = b.D; b.t = b.d; b.ldt = b.ldd;
    } else {
      GVT_REQUIRE(q.T, GVT_ERR_ARG, "problem " + std::to_string(i) + ": null T");
      b.T = q.T; b.t = q.t; b.ldt = q.ldt;
    }
    GVT_REQUIRE(b.ldd >= b.d && b.ldt >= b.t, GVT_ERR_ARG,
                "problem " + std::to_string(i) + ": ld < cols");
    b.n = q.n;
    b.noff = ntot;
    b.voff = ntot * nlam;
    ntot += q.n;
    gvt_plan *P = new gvt_plan();
    ps.plans.push_back(P);
    try {
      plan_build(P, &kind, 1, b.d, b.d, b.t, b.t, q.c, q.e, q.n, q.c, q.e, q.n,
                 GVT_FLAG_SYMMETRIC_BASES, s, nlam);
    } catch (Error &e) {
      e.msg = "problem " + std::to_string(i) + ": " + e.msg;
      throw;
    }
    GVT_REQUIRE(!P->dense, GVT_ERR_UNSUPPORTED,
                "problem " + std::to_string(i) + ": complete-data training grid");
  }
  const int64_t nv = ntot * nlam;
  const int nsys = nprob * nlam;

  // ---- chunks of the concatenated vectors
  std::vector<BChunk> hch;
  std::vector<int64_t> hcf(nsys + 1);
  for (int i = 0; i < nprob; ++i)
    for (int l = 0; l < nlam; ++l) {
      hcf[i * nlam + l] = (int64_t)hch.size();
      for (int64_t k = 0; k < pb[i].n; k += BCH)
        hch.push_back({pb[i].voff + l * pb[i].n + k, pb[i].noff + k, i * nlam + l,
                       (int32_t)std::min<int64_t>(BCH, pb[i].n - k)});
    }
  hcf[nsys] = (int64_t)hch.size();
  const int64_t nch = (int64_t)hch.size();
  GVT_REQUIRE(nch < (int64_t)1 << 31, GVT_ERR_ARG, "too many chunks");

  // ---- grouped products when every plan is one plain Kronecker term
  bool grouped = true;
  for (gvt_plan *P : ps.plans)
    grouped = grouped && P->direct && P->sbufs.size() == 1 && !P->sbufs[0].degenerate;
  // RHS blocks of the grouped products, per product precision (every plan of
  // the set has the same caps); buffers are sized for the larger first block
  const int maxR64 = ps.plans[0]->max_rhs[0], maxR32 = ps.plans[0]->max_rhs[1];
  const int Rmax = std::max(rhs_block(nlam, maxR64), rhs_block(nlam, maxR32));

  // ---- device memory
  DevMem m_a, m_r, m_p, m_w, m_wraw, m_p32, m_w32, m_y, m_part, m_sc, m_lam, m_tmp, m_act, m_cmask,
      m_ch, m_cf, m_mat32, m_vs, m_S, m_desc, m_items;
  double *A = (double *)m_a.ensure(nv * 8);
  double *r = (double *)m_r.ensure(nv * 8);
  double *p = (double *)m_p.ensure(nv * 8);
  double *w = (double *)m_w.ensure(nv * 8);
  double *wraw = (double *)m_wraw.ensure(nv * 8);
  double *ycat = (double *)m_y.ensure(ntot * 8);
  double *part = (double *)m_part.ensure(nch * 8);
  CgScalars *sc = (CgScalars *)m_sc.ensure(sizeof(CgScalars) * nsys);
  double *lam = (double *)m_lam.ensure(nlam * 8);
  double *tmp = (double *)m_tmp.ensure(nsys * 8);
  // active: problem has a system iterating; hi: problem switched to FP64
  // products (FP32 mode); act32 / act64: active problems by product precision
  uint8_t *active = (uint8_t *)m_act.ensure((size_t)nprob * 4);
  uint8_t *hi = active + nprob, *act32 = hi + nprob, *act64 = act32 + nprob;
  // per-RHS-block masks of the iteration products and the block layouts
  std::vector<int32_t> hstart;
  auto add_layout = [&](int maxR) {
    const int nb0 = (int)hstart.size();
    for (int64_t r0 = 0; r0 < nlam; r0 += rhs_block(nlam - r0, maxR)) hstart.push_back((int32_t)r0);
    hstart.push_back((int32_t)nlam);
    return (int)hstart.size() - nb0 - 1;
  };
  const int nb64 = add_layout(maxR64), nb32 = add_layout(maxR32);
  DevMem m_bm;
  const size_t bmbytes = ((size_t)(nb64 + nb32) * nprob + 15) / 16 * 16;
  uint8_t *bmbase = (uint8_t *)m_bm.ensure(bmbytes + hstart.size() * 4);
  int32_t *dstart = (int32_t *)(bmbase + bmbytes);
  GVT_HIP_CHECK(hipMemcpyAsync(dstart, hstart.data(), hstart.size() * 4, hipMemcpyHostToDevice, s));
  const BlockMasks bmk{dstart, dstart + nb64 + 1, nb64, nb32, bmbase,
                       mprec == GVT_F32 ? bmbase + (size_t)nb64 * nprob : nullptr};
  uint8_t *cmask = (uint8_t *)m_cmask.ensure((size_t)nprob + nsys);
  uint8_t *modes = cmask + nprob;  // per system: 1 = continue along the last direction
  GVT_HIP_CHECK(hipMemsetAsync(hi, 0, nprob, s));
  BChunk *ch = (BChunk *)m_ch.ensure(sizeof(BChunk) * nch);
  int64_t *cf = (int64_t *)m_cf.ensure(8 * (nsys + 1));
  float *p32 = nullptr, *w32 = nullptr;
  GVT_HIP_CHECK(hipMemcpyAsync(lam, lambdas, nlam * 8, hipMemcpyHostToDevice, s));
  GVT_HIP_CHECK(hipMemcpyAsync(ch, hch.data(), sizeof(BChunk) * nch, hipMemcpyHostToDevice, s));
  GVT_HIP_CHECK(hipMemcpyAsync(cf, hcf.data(), 8 * (nsys + 1), hipMemcpyHostToDevice, s));
  if (mprec == GVT_F32) {
    p32 = (float *)m_p32.ensure(nv * 4);
    w32 = (float *)m_w32.ensure(nv * 4);
    size_t tot = 0;
    for (int i = 0; i < nprob; ++i) {
      Prob &b = pb[i];
      b.ldd32 = f32_copy_ld(b.d);
      b.ldt32 = hom ? b.ldd32 : f32_copy_ld(b.t);
      tot += (size_t)(b.d * b.ldd32 + (hom ? 0 : b.t * b.ldt32));
    }
    float *base = (float *)m_mat32.ensure(tot * 4);
    size_t off = 0;
    for (int i = 0; i < nprob; ++i) {
      Prob &b = pb[i];
      b.D32 = base + off;
      off += (size_t)(b.d * b.ldd32);
      mat_to_f32_kernel<<<g1(b.d * b.ldd32), 256, 0, s>>>(b.D, b.ldd, b.D32, b.ldd32, b.d, b.d);
      if (hom) {
        b.T32 = b.D32;
      } else {
        b.T32 = base + off;
        off += (size_t)(b.t * b.ldt32);
        mat_to_f32_kernel<<<g1(b.t * b.ldt32), 256, 0, s>>>(b.T, b.ldt, b.T32, b.ldt32, b.t, b.t);
      }
    }
  }

  // descriptor sets: [0] FP64 iteration (p -> wraw), [1] FP32 iteration
  // (p32 -> w32), [2] FP64 residual product (w -> wraw)
  GroupDesc<double> *dd_it = nullptr, *dd_res = nullptr;
  GroupDesc<float> *df_it = nullptr;
  GroupItem *it_pack = nullptr, *it_s1 = nullptr, *it_s1f = nullptr, *it_s1s = nullptr,
            *it_s1fs = nullptr, *it_s2[kTileClasses] = {nullptr, nullptr};
  int64_t n_pack = 0, n_s1 = 0, n_s1f = 0, n_s1s = 0, n_s1fs = 0, n_s2[kTileClasses] = {0, 0};
  size_t lds_s1s = 0, lds_s1fs = 0;  // dynamic LDS of the slice walks (FP64, FP32)
  bool need_cls[kTileClasses] = {false, false};
  for (int maxR : {maxR64, maxR32})
    for (int64_t r0 = 0; r0 < nlam; r0 += rhs_block(nlam - r0, maxR))
      need_cls[tile_class(rhs_block(nlam - r0, maxR))] = true;
  if (grouped) {
    for (gvt_plan *P : ps.plans)
      for (int cls = 0; cls < kTileClasses; ++cls)
        if (need_cls[cls]) plan_ensure_tiles(P, cls, s);
    std::vector<size_t> vs_off(nprob), S_off(nprob);
    size_t vs_tot = 0, S_tot = 0;
    for (int i = 0; i < nprob; ++i) {
      const gvt_plan *P = ps.plans[i];
      const SBufSpec &sb = P->sbufs[0];
      vs_off[i] = vs_tot;
      vs_tot += ((size_t)pb[i].n * Rmax * 8 + 255) & ~size_t(255);
      S_off[i] = S_tot;
      S_tot += ((size_t)sb.rows.size() * sbuf_row_ld<double>(nkeys_of(P, sb.key), Rmax) * 8 + 255) &
               ~size_t(255);
    }
    char *vs_base = (char *)m_vs.ensure(vs_tot);
    char *S_base = (char *)m_S.ensure(S_tot);
    std::vector<GroupDesc<double>> h64(nprob), hres(nprob);
    std::vector<GroupDesc<float>> h32(nprob);
    auto fill = [&](auto &dsc, int i, auto *F0, int64_t ld0, auto *F1m, int64_t ld1m, auto *V, auto *U) {
      const gvt_plan *P = ps.plans[i];
      const TermSpec &t = P->terms[P->outputs[0][0].first];
      const SBufSpec &sb = P->sbufs[t.sbuf];
      const InputSort &is = P->insort[sb.key == SC ? 0 : 1];
      typedef typename std::remove_pointer<decltype(V)>::type Tv;
      typedef typename std::remove_const<Tv>::type T;
      const T *F[2] = {F0, F1m};
      const int64_t ldF[2] = {ld0, ld1m};
      dsc.V = V;
      dsc.ldv = pb[i].n;
      dsc.perm_in = is.perm.as<int32_t>();
      dsc.n_in = pb[i].n;
      dsc.vs = (T *)(vs_base + vs_off[i]);
      dsc.Fc = F[sb.fsc];
      dsc.ldc = ldF[sb.fsc];
      dsc.rows = sb.d_rows.as<int32_t>();
      dsc.nrows = (int64_t)sb.rows.size();
      dsc.seg = is.seg.as<int64_t>();
      dsc.other = is.other.as<int32_t>();
      dsc.nkeys = is.nkeys;
      dsc.nother = is.nother;
      dsc.S = (T *)(S_base + S_off[i]);
      dsc.F1 = F[t.fdot];
      dsc.ld1 = ldF[t.fdot];
      dsc.nx = rows_of(P, t.fdot);
      for (int cls = 0; cls < kTileClasses; ++cls) {  // unbuilt classes stay unused
        const TileSet &tl = t.tiles[cls];
        dsc.tileoff[cls] = tl.tileoff.as<int64_t>();
        dsc.tiley[cls] = tl.tiley.as<int32_t>();
        dsc.tilemax[cls] = tl.tilemax.as<int32_t>();
        dsc.grow[cls] = tl.grow.as<uint8_t>();
        dsc.yrows[cls] = tl.yrows.as<int32_t>();
        dsc.perm_out[cls] = tl.perm.as<int32_t>();
        dsc.nyb[cls] = tl.nyb;
      }
      dsc.U = U;
      dsc.ldu = pb[i].n;
      return group_stage1_setup(dsc, sb.row0);  // after n_in, nkeys, nrows and nother
    };
    std::vector<int64_t> s1blocks(nprob), s1blocks32(nprob, 0);  // stage-1 blocks per precision
    for (int i = 0; i < nprob; ++i) {
      const Prob &b = pb[i];
      s1blocks[i] = fill(h64[i], i, b.D, b.ldd, b.T, b.ldt, (const double *)(p + b.voff), wraw + b.voff);
      fill(hres[i], i, b.D, b.ldd, b.T, b.ldt, (const double *)(w + b.voff), wraw + b.voff);
      if (mprec == GVT_F32)
        s1blocks32[i] = fill(h32[i], i, (const float *)b.D32, b.ldd32, (const float *)b.T32, b.ldt32,
                             (const float *)(p32 + b.voff), w32 + b.voff);
    }
    // work lists: problems by decreasing Theorem 1 cost, each problem's blocks in order
    std::vector<int> order(nprob);
    for (int i = 0; i < nprob; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return ps.plans[x]->cost_fma > ps.plans[y]->cost_fma;
    });
    std::vector<GroupItem> hp, h1, h1f, h1s, h1fs, h2[kTileClasses];
    for (int i : order) {
      const GroupDesc<double> &g = h64[i];
      const int64_t np = group_pack_blocks(g.n_in);
      const int64_t n1 = s1blocks[i], n1f = s1blocks32[i];
      GVT_REQUIRE(np < (1 << 30) && n1 < (1 << 30) && n1f < (1 << 30), GVT_ERR_ARG, "problem too large");
      for (int64_t k = 0; k < np; ++k) hp.push_back({i, (int32_t)k});
      // stage 1: the slice walk's problems in lists of their own
      std::vector<GroupItem> &l1 = g.slice ? h1s : h1;
      for (int64_t k = 0; k < n1; ++k) l1.push_back({i, (int32_t)k});
      std::vector<GroupItem> &l1f = h32[i].slice ? h1fs : h1f;
      for (int64_t k = 0; k < n1f; ++k) l1f.push_back({i, (int32_t)k});
      lds_s1s = std::max(lds_s1s, group_stage1_slice_lds(g));
      if (mprec == GVT_F32) lds_s1fs = std::max(lds_s1fs, group_stage1_slice_lds(h32[i]));
      const TermSpec &t = ps.plans[i]->terms[ps.plans[i]->outputs[0][0].first];
      for (int cls = 0; cls < kTileClasses; ++cls) {
        if (!need_cls[cls]) continue;
        const int64_t n2 = t.tiles[cls].ntiles;
        GVT_REQUIRE(n2 < (1 << 30), GVT_ERR_ARG, "problem too large");
        for (int64_t k = 0; k < n2; ++k) h2[cls].push_back({i, (int32_t)k});
      }
    }
    n_pack = (int64_t)hp.size();
    n_s1 = (int64_t)h1.size();
    n_s1f = (int64_t)h1f.size();
    n_s1s = (int64_t)h1s.size();
    n_s1fs = (int64_t)h1fs.size();
    n_s2[0] = (int64_t)h2[0].size();
    n_s2[1] = (int64_t)h2[1].size();
    const size_t dsz64 = sizeof(GroupDesc<double>) * nprob, dsz32 = sizeof(GroupDesc<float>) * nprob;
    char *db = (char *)m_desc.ensure(2 * dsz64 + dsz32 + 256);
    dd_it = (GroupDesc<double> *)db;
    dd_res = (GroupDesc<double> *)(db + dsz64);
    df_it = (GroupDesc<float> *)(db + 2 * dsz64);
    GVT_HIP_CHECK(hipMemcpyAsync(dd_it, h64.data(), dsz64, hipMemcpyHostToDevice, s));
    GVT_HIP_CHECK(hipMemcpyAsync(dd_res, hres.data(), dsz64, hipMemcpyHostToDevice, s));
    if (mprec == GVT_F32)
      GVT_HIP_CHECK(hipMemcpyAsync(df_it, h32.data(), dsz32, hipMemcpyHostToDevice, s));
    GroupItem *ib = (GroupItem *)m_items.ensure(
        sizeof(GroupItem) * (n_pack + n_s1 + n_s1f + n_s1s + n_s1fs + n_s2[0] + n_s2[1] + 1));
    it_pack = ib;
    it_s1 = it_pack + n_pack;
    it_s1f = it_s1 + n_s1;
    it_s1s = it_s1f + n_s1f;
    it_s1fs = it_s1s + n_s1s;
    it_s2[0] = it_s1fs + n_s1fs;
    it_s2[1] = it_s2[0] + n_s2[0];
    GVT_HIP_CHECK(hipMemcpyAsync(it_pack, hp.data(), sizeof(GroupItem) * n_pack, hipMemcpyHostToDevice, s));
    GVT_HIP_CHECK(hipMemcpyAsync(it_s1, h1.data(), sizeof(GroupItem) * n_s1, hipMemcpyHostToDevice, s));
    if (n_s1f)
      GVT_HIP_CHECK(hipMemcpyAsync(it_s1f, h1f.data(), sizeof(GroupItem) * n_s1f, hipMemcpyHostToDevice, s));
    if (n_s1s)
      GVT_HIP_CHECK(hipMemcpyAsync(it_s1s, h1s.data(), sizeof(GroupItem) * n_s1s, hipMemcpyHostToDevice, s));
    if (n_s1fs)
      GVT_HIP_CHECK(hipMemcpyAsync(it_s1fs, h1fs.data(), sizeof(GroupItem) * n_s1fs, hipMemcpyHostToDevice, s));
    for (int cls = 0; cls < kTileClasses; ++cls)
      if (n_s2[cls])
        GVT_HIP_CHECK(hipMemcpyAsync(it_s2[cls], h2[cls].data(), sizeof(GroupItem) * n_s2[cls],
                                     hipMemcpyHostToDevice, s));
    // the host vectors above are released at scope end: wait for the copies
    GVT_HIP_CHECK(hipStreamSynchronize(s));
  }

  // ---- products of every problem: out = K in (RHS blocks of at most the
  // precision's cap)
  // (per_block: mask holds one per-problem mask per RHS block of the
  // precision's layout, block b at mask + b * nprob)
  auto grouped_product = [&](auto *desc, const uint8_t *mask, bool per_block) {
    constexpr bool f64 = std::is_same<std::remove_pointer_t<decltype(desc)>, GroupDesc<double>>::value;
    const int maxR = f64 ? maxR64 : maxR32;
    int64_t b = 0;
    for (int64_t r0 = 0; r0 < nlam; ++b) {
      const int R = rhs_block(nlam - r0, maxR);
      const uint8_t *mk = per_block ? mask + b * nprob : mask;
      launch_group_pack(desc, it_pack, n_pack, R, r0, mk, s);
      launch_group_stage1(desc, f64 ? it_s1 : it_s1f, f64 ? n_s1 : n_s1f, R, mk, s);
      launch_group_stage1_slice(desc, f64 ? it_s1s : it_s1fs, f64 ? n_s1s : n_s1fs, R, mk,
                                f64 ? lds_s1s : lds_s1fs, s);
      launch_group_stage2(desc, it_s2[tile_class(R)], n_s2[tile_class(R)], R, r0, mk, s);
      r0 += R;
    }
  };
  auto product64 = [&](const double *in, double *out, bool residual_set, const uint8_t *mask,
                       bool per_block = false) {
    if (grouped) {
      grouped_product(residual_set ? dd_res : dd_it, mask, per_block);
      return;
    }
    for (int i = 0; i < nprob; ++i)
      plan_execute(ps.plans[i], GVT_F64, pb[i].D, pb[i].ldd, pb[i].T, pb[i].ldt, in + pb[i].voff, nlam,
                   pb[i].n, out + pb[i].voff, pb[i].n, s);
  };
  // FP32-mode products: problems still on FP32 products (act32) and those
  // switched to FP64 after a failed certification (act64, into wraw)
  std::vector<uint8_t> hhi(nprob, 0);
  auto product32 = [&]() {
    if (grouped) {
      grouped_product(df_it, bmk.bm32, true);
      grouped_product(dd_it, bmk.bm64, true);
      return;
    }
    for (int i = 0; i < nprob; ++i) {
      if (hhi[i])
        plan_execute(ps.plans[i], GVT_F64, pb[i].D, pb[i].ldd, pb[i].T, pb[i].ldt, p + pb[i].voff, nlam,
                     pb[i].n, wraw + pb[i].voff, pb[i].n, s);
      else
        plan_execute(ps.plans[i], GVT_F32, pb[i].D32, pb[i].ldd32, pb[i].T32, pb[i].ldt32, p32 + pb[i].voff, nlam,
                     pb[i].n, w32 + pb[i].voff, pb[i].n, s);
    }
  };

  // ---- labels, norms, initial residuals
  bool any_a0 = false;
  for (int i = 0; i < nprob; ++i) {
    GVT_HIP_CHECK(hipMemcpyAsync(ycat + pb[i].noff, pr[i].y, pb[i].n * 8, hipMemcpyDeviceToDevice, s));
    if (pr[i].A0) {
      any_a0 = true;
      GVT_HIP_CHECK(hipMemcpy2DAsync(A + pb[i].voff, pb[i].n * 8, pr[i].A0, pr[i].lda0 * 8, pb[i].n * 8,
                                     nlam, hipMemcpyDeviceToDevice, s));
    } else {
      GVT_HIP_CHECK(hipMemsetAsync(A + pb[i].voff, 0, (size_t)pb[i].n * nlam * 8, s));
    }
  }
  bcg_bcast_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, ycat, r, part);
  bcg_fold_kernel<<<nsys, RB, 0, s>>>(part, cf, tmp);
  std::vector<double> ynorm(nsys), rho0(nsys);
  GVT_HIP_CHECK(hipMemcpyAsync(ynorm.data(), tmp, nsys * 8, hipMemcpyDeviceToHost, s));
  if (any_a0) {
    bcg_copy_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, A, w, -1, nullptr);
    product64(w, wraw, true, nullptr);
    bcg_residual_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, ycat, wraw, A, lam, nlam, r, part);
    bcg_fold_kernel<<<nsys, RB, 0, s>>>(part, cf, tmp);
  }
  GVT_HIP_CHECK(hipMemcpyAsync(rho0.data(), tmp, nsys * 8, hipMemcpyDeviceToHost, s));
  bcg_copy_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, r, p, -1, nullptr);
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  std::vector<CgScalars> hs(nsys);
  std::vector<uint8_t> hmask(nprob);
  for (int sy = 0; sy < nsys; ++sy) {
    ynorm[sy] = std::sqrt(ynorm[sy]);
    GVT_REQUIRE(std::isfinite(ynorm[sy]), GVT_ERR_BREAKDOWN, "non-finite labels");
    std::memset(&hs[sy], 0, sizeof(CgScalars));
    hs[sy].rho = rho0[sy];
    // all-zero labels: a = 0 is the exact solution
    hs[sy].ynorm = ynorm[sy] > 0 ? ynorm[sy] : 1.0;
    hs[sy].state = (std::sqrt(rho0[sy]) / hs[sy].ynorm < tol) ? CG_DONE : CG_ACTIVE;
  }
  auto upload_states = [&]() {
    for (int i = 0; i < nprob; ++i) {
      hmask[i] = 0;
      for (int l = 0; l < nlam; ++l) hmask[i] |= hs[i * nlam + l].state == CG_ACTIVE ? 1 : 0;
    }
    GVT_HIP_CHECK(hipMemcpyAsync(sc, hs.data(), sizeof(CgScalars) * nsys, hipMemcpyHostToDevice, s));
    GVT_HIP_CHECK(hipMemcpyAsync(active, hmask.data(), nprob, hipMemcpyHostToDevice, s));
    GVT_HIP_CHECK(hipMemcpyAsync(hi, hhi.data(), nprob, hipMemcpyHostToDevice, s));
    bcg_mask_kernel<<<(unsigned)ceil_div(nprob, 256), 256, 0, s>>>(sc, nprob, nlam, active,
                                                                   mprec == GVT_F32 ? hi : nullptr, act32, act64,
                                                                   bmk);
    GVT_HIP_CHECK(hipStreamSynchronize(s));  // the host arrays are reused
  };
  upload_states();

  const int lowprec = mprec == GVT_F32 ? 1 : 0;
  const unsigned gm = (unsigned)ceil_div(nprob, 256);
  // recurrence residual below which a problem leaves FP32 products (tuned)
  double f32_switch = kF32SwitchRelres;
  if (const char *ev = std::getenv("GVT_F32_SWITCH")) f32_switch = std::atof(ev);
  auto iteration = [&]() {
    if (lowprec) {
      to_f32_kernel<<<g1(nv), 256, 0, s>>>(p, p32, nv);
      product32();
      bcg_pw_mixed_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, w32, wraw, hi, w, p, lam, nlam, sc, part);
    } else {
      product64(p, wraw, false, bmk.bm64, true);
      bcg_pw_kernel<double><<<(unsigned)nch, RB, 0, s>>>(ch, wraw, w, p, lam, nlam, sc, part);
    }
    bcg_alpha_kernel<<<nsys, RB, 0, s>>>(sc, part, cf);
    bcg_update_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, A, r, p, w, sc, part);
    bcg_beta_kernel<<<nsys, RB, 0, s>>>(sc, part, cf, tol, max_iter, lowprec);
    bcg_p_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, p, r, sc);
    bcg_mask_kernel<<<gm, 256, 0, s>>>(sc, nprob, nlam, active, lowprec ? hi : nullptr, act32, act64, bmk);
  };

  const bool use_graph = s != nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int status = GVT_OK;
  int total_iter = 0;
  bool first = true;
  std::vector<double> rt(nsys);
  bool switched = false;
  try {
    while (true) {
      bool any_active = false;
      for (int sy = 0; sy < nsys; ++sy) any_active |= hs[sy].state == CG_ACTIVE;
      if (!any_active) {
        // certify systems whose FP32 recurrence claims convergence, and FP32
        // systems at the iteration cap, which get the FP64 finish
        auto certify = [&](const CgScalars &c) {
          return c.state == CG_PENDING || (lowprec && c.state == CG_MAXITER && c.extra == 0);
        };
        bool pending = false;
        for (int i = 0; i < nprob; ++i) {
          hmask[i] = 0;
          for (int l = 0; l < nlam; ++l) hmask[i] |= certify(hs[i * nlam + l]) ? 1 : 0;
          pending |= hmask[i] != 0;
        }
        if (!pending) break;
        std::vector<uint8_t> keep_dir(nsys, 0);
        GVT_HIP_CHECK(hipMemcpyAsync(cmask, hmask.data(), nprob, hipMemcpyHostToDevice, s));
        bcg_copy_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, A, w, -1, nullptr);
        product64(w, wraw, true, cmask);
        bcg_residual_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, ycat, wraw, A, lam, nlam, w, part);
        bcg_fold_kernel<<<nsys, RB, 0, s>>>(part, cf, tmp);
        GVT_HIP_CHECK(hipMemcpyAsync(rt.data(), tmp, nsys * 8, hipMemcpyDeviceToHost, s));
        GVT_HIP_CHECK(hipStreamSynchronize(s));
        for (int sy = 0; sy < nsys; ++sy) {
          if (!certify(hs[sy])) continue;
          const bool capped = hs[sy].state == CG_MAXITER;
          if (std::sqrt(rt[sy]) / hs[sy].ynorm < tol) {
            hs[sy].state = CG_DONE;
          } else if (capped) {
            // FP64 finish: at most max_iter / 10 more iterations with FP64
            // products, the residual replaced by the true one and the search
            // continuing along the last direction (p_k: the direction kernel
            // leaves capped systems alone), p = r + (rho_true / rho_k) p_k
            const double rho_k = hs[sy].rho / hs[sy].beta;
            const double be = rt[sy] / rho_k;
            hs[sy].state = CG_ACTIVE;
            hs[sy].extra = std::max(1, max_iter / 10);
            hs[sy].beta = std::isfinite(be) ? be : 0.0;
            hs[sy].rho = rt[sy];
            keep_dir[sy] = 1;
            if (!hhi[sy / nlam]) {
              hhi[sy / nlam] = 1;
              switched = true;
            }
          } else if (hs[sy].iters >= max_iter + hs[sy].extra) {
            hs[sy].state = CG_MAXITER;
          } else {
            // the FP32 products could not carry this system to tol: its
            // problem continues with FP64 products, restarted from the true
            // residual (R13(i): a system that converges with FP64 products
            // must converge in this form too)
            hs[sy].state = CG_ACTIVE;
            hs[sy].rho = rt[sy];
            if (!hhi[sy / nlam]) {
              hhi[sy / nlam] = 1;
              switched = true;
            }
          }
        }
        if (switched && !grouped) {
          // the plan path bakes each problem's product precision into the
          // captured graph: capture again
          if (gexec) (void)hipGraphExecDestroy(gexec);
          if (graph) (void)hipGraphDestroy(graph);
          gexec = nullptr;
          graph = nullptr;
          first = true;
        }
        switched = false;
        upload_states();
        GVT_HIP_CHECK(hipMemcpyAsync(modes, keep_dir.data(), nsys, hipMemcpyHostToDevice, s));
        bcg_reactivate_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, w, r, p, sc, modes);
        GVT_HIP_CHECK(hipStreamSynchronize(s));  // keep_dir is released at scope end
        continue;
      }
      if (first) {
        iteration();  // eager: every workspace is in place before a capture
        ++total_iter;
        first = false;
        if (use_graph) {
          GVT_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          try {
            for (int k = 0; k < check_every; ++k) iteration();
          } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          GVT_HIP_CHECK(hipStreamEndCapture(s, &graph));
          GVT_HIP_CHECK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        }
      } else if (use_graph) {
        GVT_HIP_CHECK(hipGraphLaunch(gexec, s));
        total_iter += check_every;
      } else {
        for (int k = 0; k < check_every; ++k) iteration();
        total_iter += check_every;
      }
      GVT_HIP_CHECK(hipMemcpyAsync(hs.data(), sc, sizeof(CgScalars) * nsys, hipMemcpyDeviceToHost, s));
      GVT_HIP_CHECK(hipStreamSynchronize(s));
      for (int sy = 0; sy < nsys; ++sy)
        if (hs[sy].state == CG_BREAKDOWN) status = GVT_ERR_BREAKDOWN;
      if (status != GVT_OK) break;
      if (lowprec) {
        // a problem whose active systems all have recurrence residuals below
        // the switch level continues with FP64 products (the FP32 products
        // carry the early iterations, where their rounding costs no progress)
        bool any = false;
        for (int i = 0; i < nprob; ++i) {
          if (hhi[i]) continue;
          bool act = false, below = true;
          for (int l = 0; l < nlam; ++l) {
            const CgScalars &c = hs[i * nlam + l];
            if (c.state != CG_ACTIVE) continue;
            act = true;
            below = below && std::sqrt(c.rho) / c.ynorm < f32_switch;
          }
          if (act && below) {
            hhi[i] = 1;
            any = true;
          }
        }
        if (any) {
          if (!grouped) {
            if (gexec) (void)hipGraphExecDestroy(gexec);
            if (graph) (void)hipGraphDestroy(graph);
            gexec = nullptr;
            graph = nullptr;
            first = true;
          }
          GVT_HIP_CHECK(hipMemcpyAsync(hi, hhi.data(), nprob, hipMemcpyHostToDevice, s));
          bcg_mask_kernel<<<(unsigned)ceil_div(nprob, 256), 256, 0, s>>>(sc, nprob, nlam, active, hi, act32,
                                                                         act64, bmk);
          GVT_HIP_CHECK(hipStreamSynchronize(s));
        }
      }
      if (total_iter > 4 * max_iter + 8) break;  // safety net; states already cap iterations
    }
  } catch (...) {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);

  // ---- final true residuals (FP64 products of every problem) and results
  bcg_copy_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, A, w, -1, nullptr);
  product64(w, wraw, true, nullptr);
  bcg_residual_kernel<<<(unsigned)nch, RB, 0, s>>>(ch, ycat, wraw, A, lam, nlam, r, part);
  bcg_fold_kernel<<<nsys, RB, 0, s>>>(part, cf, tmp);
  GVT_HIP_CHECK(hipMemcpyAsync(rt.data(), tmp, nsys * 8, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipMemcpyAsync(hs.data(), sc, sizeof(CgScalars) * nsys, hipMemcpyDeviceToHost, s));
  for (int i = 0; i < nprob; ++i)
    GVT_HIP_CHECK(hipMemcpy2DAsync(pr[i].A, pr[i].lda * 8, A + pb[i].voff, pb[i].n * 8, pb[i].n * 8,
                                   nlam, hipMemcpyDeviceToDevice, s));
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  check_launch(s);
  bool all_done = true;
  for (int sy = 0; sy < nsys; ++sy) {
    iters_out[sy] = hs[sy].iters;
    relres_out[sy] = std::sqrt(rt[sy]) / hs[sy].ynorm;
    if (hs[sy].state == CG_BREAKDOWN) status = GVT_ERR_BREAKDOWN;
    if (hs[sy].state != CG_DONE) all_done = false;
  }
  if (status == GVT_OK && !all_done) status = GVT_NOT_CONVERGED;
  return status;
}

}  // namespace gvt
