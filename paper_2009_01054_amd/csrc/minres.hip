// Kernel ridge regression by the minimal residual method with early stopping
// (Section 3 eq. (1) solved as the paper does: MINRES, with the number of
// iterations chosen by the AUC on a validation sample, Section 6).
//
// Multi-shift Lanczos.  MINRES on (K + lambda I) a = y from a = 0 works in the
// Krylov spaces K_k(K + lambda I, y) = K_k(K, y), and the Lanczos vectors of
// K + lambda I are those of K (the shift only adds lambda to each diagonal
// entry alpha_k of the tridiagonal matrix).  So all lambdas of the grid share
// one Lanczos basis: an iteration is ONE single-right-hand-side product K v_k,
// whatever the number of lambdas, and each lambda keeps only its own Givens
// rotations, direction vectors d_k and iterate a_k.
//
// Early stopping.  The validation predictions p = R_val K R^T a_k obey the
// same linear recurrences as a_k (a_k = a_{k-1} + tau_k d_k, d_k a combination
// of v_k, d_{k-1}, d_{k-2}), so the product K_val v_k of the Lanczos vector
// with the validation rows updates every lambda's predictions: one more
// single-RHS product per iteration.  The AUC against binary validation labels
// counts the (positive, negative) pairs the predictions order correctly (ties
// one half): the negatives' predictions are sorted and every positive counts
// by binary search, in integers, so the AUC is exact and reproducible.
// A system keeps its best AUC (strictly larger than every earlier one,
// starting from a_0 = 0), copies a into the caller's output when the AUC
// improves, and stops after `patience` iterations without improvement.
//
// Kernels per iteration (FP64 vectors; the products FP64 or FP32):
//   w = K v, wv = K_val v                          plan products
//   mr_alpha   q = w - beta_k v_{k-1};  partials of v.q
//   mr_beta    alpha_k = v.q;  q -= alpha_k v;  partials of q.q
//   mr_update  beta_{k+1} = ||q||; per system the Givens step with
//              alpha_k + lambda; d_k, a_k; v_{k+1} = q / beta_{k+1}
//   mr_val     the validation images of d_k and the predictions
//   mr_auc     sorted negatives; per positive, pair counts by binary search
//   mr_state   AUC, best, patience, residual test, iteration count
//   mr_best    a -> caller's output for systems whose AUC improved
// Scalars are double-buffered by iteration parity: a kernel that computes new
// scalars reads the previous iteration's set and writes the other, so no
// kernel reads a field that another block of the same launch writes.
#include <algorithm>
#include <cmath>
#include <cstring>

#include <hipcub/hipcub.hpp>

#include "plan.h"

namespace gvt {

static constexpr int MB = 256;   // reduction block size
static constexpr int MNB = 240;  // reduction grid (fixed for determinism)
static_assert(MNB <= MB, "partials are folded by one block");

enum MrState { MR_DONE = 0, MR_ACTIVE = 1, MR_STOPPED = 2, MR_MAXITER = 3, MR_BREAKDOWN = 4 };

struct MrShared {  // Lanczos scalars shared by every system
  double beta;     // beta_k (norm of the unnormalised v_k)
};

struct MrSys {
  double c1, s1, c2, s2;  // rotations k-1 and k-2
  double phibar;          // signed residual norm estimate
  double tau, delta, eps, gamma;  // the step's coefficients (read by mr_val)
  double best_auc, auc;
  int state, iters, best_iter, improved;
};

__device__ __forceinline__ double mr_block_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double mr_fold(const double *partial, double *sh) {
  return mr_block_sum(threadIdx.x < MNB ? partial[threadIdx.x] : 0.0, sh);
}

// partials of ||y||^2
__global__ __launch_bounds__(MB) void mr_norm_kernel(const double *__restrict__ y, int64_t n,
                                                     double *__restrict__ part) {
  __shared__ double sh[MB / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < n; i += (int64_t)MNB * MB) acc += y[i] * y[i];
  const double s = mr_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// v = y / ||y||, vprev = 0; per system a = 0, d1 = d2 = 0; scalars
__global__ __launch_bounds__(MB) void mr_init_kernel(const double *__restrict__ y, int64_t n, int nlam,
                                                     const double *__restrict__ part, double *__restrict__ v,
                                                     double *__restrict__ vprev, float *__restrict__ v32,
                                                     double *__restrict__ x, double *__restrict__ d1,
                                                     double *__restrict__ d2, MrShared *shd, MrSys *sys,
                                                     double best0, double *__restrict__ ynorm_out) {
  __shared__ double sh[MB / 64];
  const double yn = sqrt(mr_fold(part, sh));
  const double inv = yn > 0.0 ? 1.0 / yn : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < n; i += (int64_t)MNB * MB) {
    const double vi = y[i] * inv;
    v[i] = vi;
    vprev[i] = 0.0;
    if (v32) v32[i] = (float)vi;
    for (int l = 0; l < nlam; ++l) {
      x[i + l * n] = 0.0;
      d1[i + l * n] = 0.0;
      d2[i + l * n] = 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *ynorm_out = yn;
    shd->beta = yn;
    for (int l = 0; l < nlam; ++l) {
      MrSys s;
      s.c1 = 1.0; s.s1 = 0.0; s.c2 = 1.0; s.s2 = 0.0;
      s.phibar = yn;
      s.tau = s.delta = s.eps = 0.0; s.gamma = 1.0;
      s.best_auc = best0; s.auc = best0;
      s.iters = 0; s.best_iter = 0; s.improved = 0;
      s.state = !isfinite(yn) ? MR_BREAKDOWN : (yn == 0.0 ? MR_DONE : MR_ACTIVE);
      sys[l] = s;
    }
  }
}

// q = w - beta_k v_{k-1}; partials of v.q
template <class TW>
__global__ __launch_bounds__(MB) void mr_alpha_kernel(const TW *__restrict__ w, const double *__restrict__ v,
                                                      const double *__restrict__ vprev, int64_t n,
                                                      const MrShared *shd, double *__restrict__ q,
                                                      double *__restrict__ part) {
  __shared__ double sh[MB / 64];
  const double beta = shd->beta;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < n; i += (int64_t)MNB * MB) {
    const double qi = (double)w[i] - beta * vprev[i];
    q[i] = qi;
    acc += v[i] * qi;
  }
  const double s = mr_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// alpha_k = v.q (every block folds the same partials); q -= alpha_k v; partials of q.q
__global__ __launch_bounds__(MB) void mr_beta_kernel(const double *__restrict__ v, int64_t n,
                                                     const double *__restrict__ part_a,
                                                     double *__restrict__ q, double *__restrict__ part_b,
                                                     double *__restrict__ alpha_out) {
  __shared__ double sh[MB / 64];
  const double alpha = mr_fold(part_a, sh);
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < n; i += (int64_t)MNB * MB) {
    const double qi = q[i] - alpha * v[i];
    q[i] = qi;
    acc += qi * qi;
  }
  const double s = mr_block_sum(acc, sh);
  if (threadIdx.x == 0) part_b[blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
}

// The Givens step of one system from the previous scalars (so) into sn_.
__device__ __forceinline__ void mr_givens(const MrSys &so, MrSys &sn_, double alpha, double beta,
                                          double beta_next) {
  sn_ = so;
  const double eps = so.s2 * beta, dt = so.c2 * beta;
  const double delta = so.c1 * dt + so.s1 * alpha;
  const double gbar = so.c1 * alpha - so.s1 * dt;
  const double gamma = sqrt(gbar * gbar + beta_next * beta_next);
  sn_.eps = eps;
  sn_.delta = delta;
  sn_.gamma = gamma;
  if (!(gamma > 0.0) || !isfinite(gamma)) {
    sn_.tau = 0.0;
    sn_.state = MR_BREAKDOWN;
    return;
  }
  const double cs = gbar / gamma, snr = beta_next / gamma;
  sn_.tau = cs * so.phibar;
  sn_.phibar = -snr * so.phibar;
  sn_.c2 = so.c1;
  sn_.s2 = so.s1;
  sn_.c1 = cs;
  sn_.s1 = snr;
}

// beta_{k+1}, the Givens steps, d_k and a_k of every active system, then the
// next Lanczos vector.  Reads the scalars of parity p (so, sho), writes 1-p.
__global__ __launch_bounds__(MB) void mr_update_kernel(double *__restrict__ v, double *__restrict__ vprev,
                                                       float *__restrict__ v32, const double *__restrict__ q,
                                                       int64_t n, int nlam, const double *__restrict__ lam,
                                                       const double *__restrict__ alpha_in,
                                                       const double *__restrict__ part_b,
                                                       const MrShared *sho, MrShared *shn,
                                                       const MrSys *so, MrSys *sn, double *__restrict__ x,
                                                       double *__restrict__ d1, double *__restrict__ d2) {
  // (elementwise after the fold: any grid; the fold reads the MNB partials)
  __shared__ double sh[MB / 64];
  __shared__ MrSys st[64];
  __shared__ double sdl[64], sep[64], sig[64], stau[64];
  __shared__ int son[64];
  const double beta_next = sqrt(mr_fold(part_b, sh));
  const double alpha = *alpha_in, beta = sho->beta;
  if (threadIdx.x < nlam) {
    const int l = threadIdx.x;
    MrSys s = so[l];
    const bool was = s.state == MR_ACTIVE;
    if (was) mr_givens(so[l], s, alpha + lam[l], beta, beta_next);
    st[l] = s;
    son[l] = was && s.state == MR_ACTIVE;
    sdl[l] = s.delta;
    sep[l] = s.eps;
    sig[l] = s.gamma;
    stau[l] = s.tau;
  }
  __syncthreads();
  const double ib = beta_next > 0.0 ? 1.0 / beta_next : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < n; i += (int64_t)gridDim.x * MB) {
    const double vi = v[i];
    for (int l = 0; l < nlam; ++l) {
      if (!son[l]) continue;
      const int64_t o = i + (int64_t)l * n;
      const double a1 = d1[o];
      const double dk = (vi - sdl[l] * a1 - sep[l] * d2[o]) / sig[l];
      d2[o] = a1;
      d1[o] = dk;
      x[o] += stau[l] * dk;
    }
    const double vn = q[i] * ib;
    vprev[i] = vi;
    v[i] = vn;
    if (v32) v32[i] = (float)vn;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    shn->beta = beta_next;
    for (int l = 0; l < nlam; ++l) sn[l] = st[l];
  }
}

// Validation images: pd_k = (K_val v_k - delta pd_{k-1} - eps pd_{k-2}) / gamma;
// predictions += tau pd_k (systems that stepped in this iteration).
template <class TW>
__global__ __launch_bounds__(MB) void mr_val_kernel(const TW *__restrict__ wv, int64_t nv, int nlam,
                                                    const MrSys *so, const MrSys *sn,
                                                    double *__restrict__ pd1, double *__restrict__ pd2,
                                                    double *__restrict__ pv) {
  __shared__ double sdl[64], sep[64], sig[64], stau[64];
  __shared__ int son[64];
  if (threadIdx.x < nlam) {
    const int l = threadIdx.x;
    son[l] = so[l].state == MR_ACTIVE && sn[l].state == MR_ACTIVE;
    sdl[l] = sn[l].delta;
    sep[l] = sn[l].eps;
    sig[l] = sn[l].gamma;
    stau[l] = sn[l].tau;
  }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < nv; i += (int64_t)gridDim.x * MB) {
    const double w = (double)wv[i];
    for (int l = 0; l < nlam; ++l) {
      if (!son[l]) continue;
      const int64_t o = i + (int64_t)l * nv;
      const double a1 = pd1[o];
      const double dk = (w - sdl[l] * a1 - sep[l] * pd2[o]) / sig[l];
      pd2[o] = a1;
      pd1[o] = dk;
      pv[o] += stau[l] * dk;
    }
  }
}

// lab[q] = q / div (the system of gathered negative q)
__global__ void mr_iota_div_kernel(int32_t *__restrict__ lab, int64_t n, int64_t div) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) lab[q] = (int32_t)(q / div);
}

__global__ void mr_gather_neg_kernel(const double *__restrict__ pv, int64_t nv, int nlam,
                                     const int32_t *__restrict__ neg, int64_t nneg, double *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nneg * nlam) return;
  const int64_t l = q / nneg, j = q - l * nneg;
  out[q] = pv[l * nv + neg[j]];
}

__global__ __launch_bounds__(MB) void mr_auc_kernel(const double *__restrict__ pv, int64_t nv, int nlam,
                                                    const int32_t *__restrict__ pos, int64_t npos,
                                                    const double *__restrict__ sneg, int64_t nneg,
                                                    const MrSys *so, unsigned long long *__restrict__ cnt) {
  __shared__ unsigned long long shc[MB / 64];
  const int64_t ip = (int64_t)blockIdx.x * MB + threadIdx.x;
  for (int l = 0; l < nlam; ++l) {
    if (so[l].state != MR_ACTIVE) continue;  // uniform: only systems that stepped are counted
    unsigned long long c = 0;
    if (ip < npos) {
      const double x = pv[(int64_t)l * nv + pos[ip]];
      const double *a = sneg + (int64_t)l * nneg;
      int64_t lo = 0, hi = nneg;  // first element >= x
      while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
      }
      int64_t lo2 = lo, hi2 = nneg;  // first element > x
      while (lo2 < hi2) {
        const int64_t mid = lo2 + (hi2 - lo2) / 2;
        if (a[mid] <= x) lo2 = mid + 1;
        else hi2 = mid;
      }
      c = (unsigned long long)lo + (unsigned long long)lo2;  // 2 less + equal
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) shc[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[(int64_t)blockIdx.x * nlam + l] = (shc[0] + shc[1]) + (shc[2] + shc[3]);
    __syncthreads();
  }
}

// One thread per system: the AUC from the counts, best / patience, the
// residual test and the iteration cap; *run = any system still active.
__global__ void mr_state_kernel(MrSys *sn, const MrSys *so, int nlam, const unsigned long long *cnt, int nblk,
                                int64_t npos, int64_t nneg, int have_val, int patience, double tol,
                                const double *__restrict__ ynorm, int max_iter,
                                double *__restrict__ auc_hist, int *__restrict__ run) {
  const int l = threadIdx.x;
  if (l < nlam) {
    MrSys s = sn[l];
    s.improved = 0;
    if (so[l].state == MR_ACTIVE) {
      s.iters = so[l].iters + 1;
      if (s.state == MR_ACTIVE) {
        if (have_val) {
          unsigned long long t = 0;
          for (int b = 0; b < nblk; ++b) t += cnt[(int64_t)b * nlam + l];
          s.auc = (npos > 0 && nneg > 0) ? (double)t / (2.0 * (double)npos * (double)nneg) : 0.5;
          if (auc_hist) auc_hist[(int64_t)(s.iters - 1) * nlam + l] = s.auc;
          if (s.auc > s.best_auc) {
            s.best_auc = s.auc;
            s.best_iter = s.iters;
            s.improved = 1;
          }
        }
        const double yn = *ynorm;
        if (fabs(s.phibar) / (yn > 0.0 ? yn : 1.0) < tol) s.state = MR_DONE;
        else if (have_val && patience > 0 && s.iters - s.best_iter >= patience) s.state = MR_STOPPED;
        else if (s.iters >= max_iter) s.state = MR_MAXITER;
      }
    }
    sn[l] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int any = 0;
    for (int k = 0; k < nlam; ++k) any |= sn[k].state == MR_ACTIVE;
    *run = any;
  }
}

// a -> out for systems whose AUC just improved
__global__ void mr_best_kernel(const double *__restrict__ x, int64_t n, int nlam, const MrSys *sn,
                               double *__restrict__ out, int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int l = 0; l < nlam; ++l)
    if (sn[l].improved) out[i + l * ldo] = x[i + (int64_t)l * n];
}

__global__ void mr_copy_kernel(const double *__restrict__ x, int64_t n, int nlam, double *__restrict__ out,
                               int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int l = 0; l < nlam; ++l) out[i + l * ldo] = x[i + (int64_t)l * n];
}

// r = y - (K a + lambda a) per system; partials of r.r (per system, MNB each)
__global__ __launch_bounds__(MB) void mr_resid_kernel(const double *__restrict__ y,
                                                      const double *__restrict__ ka,
                                                      const double *__restrict__ a, int64_t lda,
                                                      const double *__restrict__ lam, int64_t n, int nlam,
                                                      double *__restrict__ part) {
  __shared__ double sh[MB / 64];
  for (int l = 0; l < nlam; ++l) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < n; i += (int64_t)MNB * MB) {
      const double r = y[i] - (ka[i + (int64_t)l * n] + lam[l] * a[i + l * lda]);
      acc += r * r;
    }
    const double s = mr_block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)l * MNB + blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(MB) void mr_fold_kernel(const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double sh[MB / 64];
  const double v = mr_fold(part + (int64_t)blockIdx.x * MNB, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// FP32 copy of a base matrix with row stride ldy >= cols (padding written as
// zeros): rows of whole 64-byte lines start on 16-byte boundaries, so the
// stage-2 kernels stage F1 in vector pieces.
__global__ void mr_to_f32_kernel(const double *__restrict__ x, int64_t ldx, float *__restrict__ y,
                                 int64_t ldy, int64_t rows, int64_t cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ldy) return;
  const int64_t r = idx / ldy, c = idx - r * ldy;
  y[idx] = c < cols ? (float)x[r * ldx + c] : 0.0f;
}

// ---------------------------------------------------------------------------
namespace {
struct PlanHolder {
  gvt_plan *plan = nullptr;
  ~PlanHolder() {
    if (plan) {
      if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
      delete plan;
    }
  }
};
dim3 mg1(int64_t n) { return dim3((unsigned)ceil_div(std::max<int64_t>(n, 1), 256)); }
// elementwise kernels of MB threads, one element per thread (capped grid-stride)
dim3 mgrid(int64_t n) { return dim3((unsigned)std::min<int64_t>(ceil_div(std::max<int64_t>(n, 1), MB), 8192)); }
}  // namespace

int krr_minres_impl(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                    int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                    const double *lambdas, int nlam, double *A, int64_t lda, int max_iter, double tol,
                    int mprec, const gvt_validation *val, int check_every, int64_t *iters_out,
                    double *relres_out, int64_t *best_iter_out, double *best_auc_out, double *auc_hist,
                    hipStream_t s) {
  GVT_REQUIRE(n >= 1 && nlam >= 1 && nlam <= 64, GVT_ERR_ARG, "need n >= 1 and 1 <= nlam <= 64");
  GVT_REQUIRE(D && c && e && y && lambdas && A && iters_out && relres_out, GVT_ERR_ARG, "null argument");
  GVT_REQUIRE(lda >= n, GVT_ERR_ARG, "lda < n");
  GVT_REQUIRE(max_iter >= 1 && tol >= 0 && check_every >= 1, GVT_ERR_ARG, "bad max_iter/tol/check_every");
  GVT_REQUIRE(mprec == GVT_F64 || mprec == GVT_F32, GVT_ERR_UNSUPPORTED,
              "MINRES products run in GVT_F64 or GVT_F32");
  for (int l = 0; l < nlam; ++l)
    GVT_REQUIRE(lambdas[l] >= 0 && std::isfinite(lambdas[l]), GVT_ERR_ARG, "lambda must be >= 0");
  const bool hom = kind == GVT_SYMMETRIC || kind == GVT_ANTISYMMETRIC || kind == GVT_RANKING ||
                   kind == GVT_MLPK;
  if (hom) { T = D; t = d; ldt = ldd; }
  GVT_REQUIRE(T, GVT_ERR_ARG, "null T");
  GVT_REQUIRE(ldd >= d && ldt >= t, GVT_ERR_ARG, "ld < cols");
  const bool have_val = val != nullptr && val->n > 0;
  if (have_val) {
    GVT_REQUIRE(val->a && val->b && val->labels, GVT_ERR_ARG, "validation: null pointer");
    GVT_REQUIRE(val->patience >= 0, GVT_ERR_ARG, "validation: negative patience");
  }
  const int64_t nv = have_val ? val->n : 0;

  PlanHolder ph, pv_h;
  ph.plan = new gvt_plan();
  gvt_plan *P = ph.plan;
  plan_build(P, &kind, 1, d, d, t, t, c, e, n, c, e, n, GVT_FLAG_SYMMETRIC_BASES, s, 1);
  GVT_REQUIRE(!P->dense, GVT_ERR_UNSUPPORTED, "complete-data training grid: use the dense product");
  gvt_plan *PV = nullptr;
  std::vector<int32_t> hpos, hneg;
  if (have_val) {
    pv_h.plan = new gvt_plan();
    PV = pv_h.plan;
    plan_build(PV, &kind, 1, d, d, t, t, val->a, val->b, nv, c, e, n, GVT_FLAG_SYMMETRIC_BASES, s, 1);
    GVT_REQUIRE(!PV->dense, GVT_ERR_UNSUPPORTED, "validation sample: complete data not supported");
    // positive / negative index lists (the labels are read once)
    std::vector<double> lab(nv);
    GVT_HIP_CHECK(hipMemcpyAsync(lab.data(), val->labels, nv * 8, hipMemcpyDeviceToHost, s));
    GVT_HIP_CHECK(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nv; ++i) (lab[i] > 0.5 ? hpos : hneg).push_back((int32_t)i);
  }
  const int64_t npos = (int64_t)hpos.size(), nneg = (int64_t)hneg.size();

  // workspace
  const size_t nn = (size_t)n * nlam;
  DevMem m_v, m_vp, m_q, m_w, m_x, m_d1, m_d2, m_part, m_sc, m_lam, m_v32, m_w32, m_D32, m_T32;
  DevMem m_wv, m_pd1, m_pd2, m_pv, m_pn, m_cnt, m_ka, m_tmp;
  double *v = (double *)m_v.ensure(n * 8), *vprev = (double *)m_vp.ensure(n * 8);
  double *q = (double *)m_q.ensure(n * 8), *w = (double *)m_w.ensure(n * 8);
  double *x = (double *)m_x.ensure(nn * 8), *d1 = (double *)m_d1.ensure(nn * 8);
  double *d2 = (double *)m_d2.ensure(nn * 8);
  double *part = (double *)m_part.ensure((size_t)MNB * 8 * 2 + 256);
  double *part_b = part + MNB;
  // scalars: two MrShared, two MrSys[nlam] sets, alpha, ||y||, run flag
  char *scb = (char *)m_sc.ensure(2 * sizeof(MrShared) + 2 * sizeof(MrSys) * nlam + 256);
  MrShared *shd[2] = {(MrShared *)scb, (MrShared *)scb + 1};
  MrSys *sys[2] = {(MrSys *)(scb + 2 * sizeof(MrShared)), (MrSys *)(scb + 2 * sizeof(MrShared)) + nlam};
  double *alpha = (double *)(scb + 2 * sizeof(MrShared) + 2 * sizeof(MrSys) * nlam);
  double *ynorm = alpha + 1;
  int *run = (int *)(ynorm + 1);
  double *lam = (double *)m_lam.ensure(nlam * 8);
  GVT_HIP_CHECK(hipMemcpyAsync(lam, lambdas, nlam * 8, hipMemcpyHostToDevice, s));
  const bool lowprec = mprec == GVT_F32;
  float *v32 = nullptr, *w32 = nullptr, *D32 = nullptr, *T32 = nullptr, *wv32 = nullptr;
  const int64_t ldd32 = (d + 15) / 16 * 16, ldt32 = hom ? ldd32 : (t + 15) / 16 * 16;
  if (lowprec) {
    v32 = (float *)m_v32.ensure(n * 4);
    w32 = (float *)m_w32.ensure((size_t)(n + nv) * 4);
    wv32 = w32 + n;
    D32 = (float *)m_D32.ensure((size_t)d * ldd32 * 4);
    mr_to_f32_kernel<<<mg1(d * ldd32), 256, 0, s>>>(D, ldd, D32, ldd32, d, d);
    if (!hom) {
      T32 = (float *)m_T32.ensure((size_t)t * ldt32 * 4);
      mr_to_f32_kernel<<<mg1(t * ldt32), 256, 0, s>>>(T, ldt, T32, ldt32, t, t);
    } else {
      T32 = D32;
    }
  }
  double *wv = nullptr, *pd1 = nullptr, *pd2 = nullptr, *pvv = nullptr;
  int32_t *dpos = nullptr, *dneg = nullptr;
  unsigned long long *cnt = nullptr;
  DevMem m_sort;
  double *gneg = nullptr, *sneg = nullptr;
  char *stemp = nullptr;
  size_t sort_bytes = 0;
  double *kneg = nullptr;                                   // negatives sorted by value (all systems)
  int32_t *lab1 = nullptr, *lab2 = nullptr, *lab3 = nullptr;  // system index per gathered negative
  int sys_bits = 1;
  while ((1 << sys_bits) < nlam) ++sys_bits;
  const int64_t auc_blocks = std::max<int64_t>(1, ceil_div(npos, MB));
  if (have_val) {
    wv = (double *)m_wv.ensure(nv * 8);
    pd1 = (double *)m_pd1.ensure((size_t)nv * nlam * 8);
    pd2 = (double *)m_pd2.ensure((size_t)nv * nlam * 8);
    pvv = (double *)m_pv.ensure((size_t)nv * nlam * 8);
    GVT_HIP_CHECK(hipMemsetAsync(pd1, 0, (size_t)nv * nlam * 8, s));
    GVT_HIP_CHECK(hipMemsetAsync(pd2, 0, (size_t)nv * nlam * 8, s));
    GVT_HIP_CHECK(hipMemsetAsync(pvv, 0, (size_t)nv * nlam * 8, s));
    dpos = (int32_t *)m_pn.ensure((size_t)(npos + nneg) * 4 + 256);
    dneg = dpos + npos;
    if (npos) GVT_HIP_CHECK(hipMemcpyAsync(dpos, hpos.data(), npos * 4, hipMemcpyHostToDevice, s));
    if (nneg) GVT_HIP_CHECK(hipMemcpyAsync(dneg, hneg.data(), nneg * 4, hipMemcpyHostToDevice, s));
    cnt = (unsigned long long *)m_cnt.ensure((size_t)auc_blocks * nlam * 8);
    // sorted negatives of every system: the gathered predictions sorted once by
    // value (the system index riding along), then stably by system index, so
    // each system's run is its negatives in the order a sort of that system
    // alone gives (two sorts in place of one per system)
    const int64_t nn2 = std::max<int64_t>(nneg * nlam, 1);
    size_t tb1 = 0, tb2 = 0;
    GVT_HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb1, (const double *)nullptr, (double *)nullptr,
                                                     (const int32_t *)nullptr, (int32_t *)nullptr, (int)nn2, 0,
                                                     64, s));
    GVT_HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, (const int32_t *)nullptr, (int32_t *)nullptr,
                                                     (const double *)nullptr, (double *)nullptr, (int)nn2, 0,
                                                     sys_bits, s));
    sort_bytes = std::max(tb1, tb2);
    const size_t arrays = ((size_t)nn2 * 36 + 255) / 256 * 256;
    char *sb = (char *)m_sort.ensure(arrays + sort_bytes + 256);
    gneg = (double *)sb;
    sneg = gneg + nn2;
    kneg = sneg + nn2;
    lab1 = (int32_t *)(kneg + nn2);
    lab2 = lab1 + nn2;
    lab3 = lab2 + nn2;
    stemp = sb + arrays;
    mr_iota_div_kernel<<<mg1(nn2), 256, 0, s>>>(lab1, nn2, std::max<int64_t>(nneg, 1));
  }
  double *hist_dev = nullptr;
  DevMem m_hist;
  if (have_val && auc_hist) {
    hist_dev = (double *)m_hist.ensure((size_t)max_iter * nlam * 8);
    std::vector<double> nanv((size_t)max_iter * nlam, NAN);
    GVT_HIP_CHECK(hipMemcpyAsync(hist_dev, nanv.data(), nanv.size() * 8, hipMemcpyHostToDevice, s));
    GVT_HIP_CHECK(hipStreamSynchronize(s));
  }
  // A starts at zero (the iterate of the best AUC, or the last iterate)
  for (int l = 0; l < nlam; ++l) GVT_HIP_CHECK(hipMemsetAsync(A + l * lda, 0, n * 8, s));

  mr_norm_kernel<<<MNB, MB, 0, s>>>(y, n, part);
  // a_0 = 0: every prediction ties, AUC 1/2 (or 1/2 by definition with one class empty)
  mr_init_kernel<<<MNB, MB, 0, s>>>(y, n, nlam, part, v, vprev, v32, x, d1, d2, shd[0], sys[0], 0.5, ynorm);
  check_launch(s);

  int par = 0;
  int total = 0;
  std::vector<MrSys> hs(nlam);
  int status = GVT_OK;
  // Products inside iterations are gated by `run`: once every system has
  // stopped, the rest of a block of iterations skips its products.
  GVT_HIP_CHECK(hipMemsetD32Async(run, 1, 1, s));
  auto iteration = [&]() {
    MrShared *sho = shd[par], *shn = shd[1 - par];
    MrSys *so = sys[par], *sn = sys[1 - par];
    P->gate = run;
    if (PV) PV->gate = run;
    if (lowprec) {
      plan_execute(P, GVT_F32, D32, ldd32, T32, ldt32, v32, 1, n, w32, n, s);
      mr_alpha_kernel<float><<<MNB, MB, 0, s>>>(w32, v, vprev, n, sho, q, part);
    } else {
      plan_execute(P, GVT_F64, D, ldd, T, ldt, v, 1, n, w, n, s);
      mr_alpha_kernel<double><<<MNB, MB, 0, s>>>(w, v, vprev, n, sho, q, part);
    }
    if (have_val) {
      // K_val v_k before v moves on
      if (lowprec) plan_execute(PV, GVT_F32, D32, ldd32, T32, ldt32, v32, 1, n, wv32, nv, s);
      else plan_execute(PV, GVT_F64, D, ldd, T, ldt, v, 1, n, wv, nv, s);
    }
    mr_beta_kernel<<<MNB, MB, 0, s>>>(v, n, part, q, part_b, alpha);
    mr_update_kernel<<<mgrid(n), MB, 0, s>>>(v, vprev, v32, q, n, nlam, lam, alpha, part_b, sho, shn, so, sn, x, d1,
                                        d2);
    if (have_val) {
      if (lowprec)
        mr_val_kernel<float><<<mgrid(nv), MB, 0, s>>>(wv32, nv, nlam, so, sn, pd1, pd2, pvv);
      else
        mr_val_kernel<double><<<mgrid(nv), MB, 0, s>>>(wv, nv, nlam, so, sn, pd1, pd2, pvv);
      if (nneg > 0) {
        mr_gather_neg_kernel<<<mg1(nneg * nlam), 256, 0, s>>>(pvv, nv, nlam, dneg, nneg, gneg);
        // (a segmented sort would give each system's run one workgroup)
        const int nn2 = (int)(nneg * nlam);
        size_t tb = sort_bytes;
        GVT_HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(stemp, tb, gneg, kneg, lab1, lab2, nn2, 0, 64, s));
        tb = sort_bytes;
        GVT_HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(stemp, tb, lab2, lab3, kneg, sneg, nn2, 0, sys_bits, s));
      }
      mr_auc_kernel<<<(unsigned)auc_blocks, MB, 0, s>>>(pvv, nv, nlam, dpos, npos, sneg, nneg, so, cnt);
    }
    mr_state_kernel<<<1, 64, 0, s>>>(sn, so, nlam, cnt, (int)auc_blocks, npos, nneg, have_val ? 1 : 0,
                                     have_val ? (int)val->patience : 0, tol, ynorm, max_iter, hist_dev, run);
    if (have_val) mr_best_kernel<<<mg1(n), 256, 0, s>>>(x, n, nlam, sn, A, lda);
    P->gate = nullptr;
    if (PV) PV->gate = nullptr;
    par = 1 - par;
  };
  while (true) {
    GVT_HIP_CHECK(hipMemcpyAsync(hs.data(), sys[par], sizeof(MrSys) * nlam, hipMemcpyDeviceToHost, s));
    GVT_HIP_CHECK(hipStreamSynchronize(s));
    bool any = false;
    for (int l = 0; l < nlam; ++l) {
      any |= hs[l].state == MR_ACTIVE;
      if (hs[l].state == MR_BREAKDOWN) status = GVT_ERR_BREAKDOWN;
    }
    if (!any || status != GVT_OK || total >= max_iter) break;
    const int nk = std::min(check_every, max_iter - total);
    for (int k = 0; k < nk; ++k) iteration();
    total += nk;
    check_launch(s);
  }
  // without a validation sample the result is the last iterate
  if (!have_val) mr_copy_kernel<<<mg1(n), 256, 0, s>>>(x, n, nlam, A, lda);
  // true residuals of the returned solutions with an FP64 product
  double *ka = (double *)m_ka.ensure(nn * 8);
  double *acopy = (double *)m_tmp.ensure(nn * 8 + (size_t)MNB * nlam * 8 + 64 * 8);
  double *rpart = acopy + nn, *rt = rpart + (size_t)MNB * nlam;
  for (int l = 0; l < nlam; ++l)
    GVT_HIP_CHECK(hipMemcpyAsync(acopy + (size_t)l * n, A + l * lda, n * 8, hipMemcpyDeviceToDevice, s));
  plan_execute(P, GVT_F64, D, ldd, T, ldt, acopy, nlam, n, ka, n, s);
  mr_resid_kernel<<<MNB, MB, 0, s>>>(y, ka, A, lda, lam, n, nlam, rpart);
  mr_fold_kernel<<<nlam, MB, 0, s>>>(rpart, rt);
  std::vector<double> hrt(nlam);
  double hyn = 0.0;
  GVT_HIP_CHECK(hipMemcpyAsync(hrt.data(), rt, nlam * 8, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipMemcpyAsync(&hyn, ynorm, 8, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipMemcpyAsync(hs.data(), sys[par], sizeof(MrSys) * nlam, hipMemcpyDeviceToHost, s));
  if (hist_dev)
    GVT_HIP_CHECK(hipMemcpyAsync(auc_hist, hist_dev, (size_t)max_iter * nlam * 8, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  check_launch(s);
  GVT_REQUIRE(std::isfinite(hyn), GVT_ERR_BREAKDOWN, "non-finite labels");
  const double yn = hyn > 0.0 ? hyn : 1.0;
  bool all_done = true;
  for (int l = 0; l < nlam; ++l) {
    iters_out[l] = hs[l].iters;
    relres_out[l] = std::sqrt(hrt[l]) / yn;
    if (best_iter_out) best_iter_out[l] = have_val ? hs[l].best_iter : hs[l].iters;
    if (best_auc_out) best_auc_out[l] = have_val ? hs[l].best_auc : NAN;
    if (hs[l].state == MR_BREAKDOWN) status = GVT_ERR_BREAKDOWN;
    if (hs[l].state == MR_MAXITER || hs[l].state == MR_ACTIVE) all_done = false;
  }
  if (status == GVT_OK && !all_done) status = GVT_NOT_CONVERGED;
  return status;
}

}  // namespace gvt
