// Regularized kernel risk minimisation with other losses (Section 3: the
// risk L(p, y) + (lambda/2) ||f||^2 with p = K a; the GVT speeds up any
// optimiser dominated by products with K, such as truncated Newton; Section 7
// names kernel logistic regression and support vector machines).
//
//   J(a) = L(K a, y) + (lambda / 2) a^T K a,    grad J = K (g + lambda a)
//
//   squared        L = 1/2 sum (y - p)^2            g = p - y,                d = 1
//   logistic       L = sum log(1 + exp(-y p))       g = -y sigma(-y p),       d = sigma(yp) sigma(-yp)
//   squared hinge  L = 1/2 sum max(0, 1 - y p)^2    g = -y max(0, 1 - y p),   d = [y p < 1]
//   hinge          L = sum max(0, 1 - y p)          g = -y [y p < 1]  (subgradient; no Newton)
//
// Truncated Newton: the Newton equation K (D K + lambda I) delta = -grad J is
// met by any delta with (D K + lambda I) delta = -(g + lambda a), an operator
// self-adjoint and positive in the K inner product <x, y>_K = x^T K y.  Each
// step runs conjugate gradients on it in that inner product:
// <z, A z>_K = (K z)^T (d * (K z) + lambda z), <r, r>_K = r^T (K r), one kernel
// product K r per iteration, K z and K delta carried by the recurrences of z
// and delta.  CG stops after max_cg iterations or once sqrt(<r, r>_K) <=
// min(1/2, sqrt(||grad|| / ||grad_0||)) sqrt(<r_0, r_0>_K); then the step
// backtracks t = 1, 1/2, ... (at most 30 halvings) until
// J(a + t delta) <= J(a) + 1e-4 t grad.delta, using p + t K delta, so the line
// search costs no // product.  The outer loop stops when ||grad J|| <= tol ||grad J(0)|| or after
// max_newton steps.  All vectors and scalars are FP64 with fixed-order block
// sums; the products run in FP64 or FP32.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.h"

namespace gvt {

static constexpr int EB = 256;   // block size
static constexpr int ENB = 240;  // reduction grid (fixed for determinism)

__device__ __forceinline__ double e_block_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double e_sigma(double x) {
  if (x >= 0.0) return 1.0 / (1.0 + exp(-x));
  const double ex = exp(x);
  return ex / (1.0 + ex);
}

// Loss value, first and second derivative at prediction p with label y.
__device__ __forceinline__ void e_loss(int loss, double p, double y, double &L, double &g, double &d) {
  if (loss == GVT_LOSS_SQUARED) {
    const double r = p - y;
    L = 0.5 * r * r;
    g = r;
    d = 1.0;
    return;
  }
  const double m = y * p;
  if (loss == GVT_LOSS_LOGISTIC) {
    L = fmax(-m, 0.0) + log1p(exp(-fabs(m)));
    const double s = e_sigma(-m);
    g = -y * s;
    d = s * (1.0 - s);
    return;
  }
  const double h = fmax(0.0, 1.0 - m);
  if (loss == GVT_LOSS_SQHINGE) {
    L = 0.5 * h * h;
    g = -y * h;
    d = h > 0.0 ? 1.0 : 0.0;
    return;
  }
  L = h;  // hinge
  g = h > 0.0 ? -y : 0.0;
  d = 0.0;
}

// From the product pw = K a:
// u = g + lambda a, dv = d; partials [0] of L, [1] of a.p.
template <class TW>
__global__ __launch_bounds__(EB) void e_loss_kernel(int loss, const TW *__restrict__ pw,
                                                    const double *__restrict__ y,
                                                    const double *__restrict__ a, double lam, int64_t n,
                                                    double *__restrict__ p_out, double *__restrict__ u,
                                                    double *__restrict__ dv, double *__restrict__ part) {
  __shared__ double sh[EB / 64];
  double sl = 0.0, sa = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x; i < n; i += (int64_t)ENB * EB) {
    const double p = (double)pw[i];
    double L, g, d;
    e_loss(loss, p, y[i], L, g, d);
    if (p_out) p_out[i] = p;
    if (u) u[i] = g + lam * a[i];
    if (dv) dv[i] = d;
    sl += L;
    sa += a[i] * p;
  }
  const double s0 = e_block_sum(sl, sh), s1 = e_block_sum(sa, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s0;
    part[ENB + blockIdx.x] = s1;
  }
}

// Trial point of the line search: L(p + t Kx) and (a + t x).(p + t Kx) partials.
__global__ __launch_bounds__(EB) void e_trial_kernel(int loss, const double *__restrict__ p,
                                                     const double *__restrict__ kx, const double *__restrict__ a,
                                                     const double *__restrict__ x, const double *__restrict__ y,
                                                     double t, int64_t n, double *__restrict__ part) {
  __shared__ double sh[EB / 64];
  double sl = 0.0, sa = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x; i < n; i += (int64_t)ENB * EB) {
    const double pt = p[i] + t * kx[i];
    double L, g, d;
    e_loss(loss, pt, y[i], L, g, d);
    sl += L;
    sa += (a[i] + t * x[i]) * pt;
  }
  const double s0 = e_block_sum(sl, sh), s1 = e_block_sum(sa, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s0;
    part[ENB + blockIdx.x] = s1;
  }
}

// partials of x.y
template <class TY>
__global__ __launch_bounds__(EB) void e_dot_kernel(const double *__restrict__ x, const TY *__restrict__ y,
                                                   int64_t n, double *__restrict__ part) {
  __shared__ double sh[EB / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x; i < n; i += (int64_t)ENB * EB)
    s += x[i] * (double)y[i];
  const double r = e_block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// fold nsum groups of ENB partials into out[0..nsum)
__global__ __launch_bounds__(EB) void e_fold_kernel(const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double sh[EB / 64];
  const double v = e_block_sum(threadIdx.x < ENB ? part[(int64_t)blockIdx.x * ENB + threadIdx.x] : 0.0, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// az = d * kz + lambda z; partials of kz . az (= <z, A z>_K)
__global__ __launch_bounds__(EB) void e_az_kernel(const double *__restrict__ dv, const double *__restrict__ kz,
                                                  const double *__restrict__ z, double lam, int64_t n,
                                                  double *__restrict__ az, double *__restrict__ part) {
  __shared__ double sh[EB / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x; i < n; i += (int64_t)ENB * EB) {
    const double v = dv[i] * kz[i] + lam * z[i];
    az[i] = v;
    s += kz[i] * v;
  }
  const double r = e_block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// x += al z; kx += al kz; r -= al az
__global__ void e_cgstep_kernel(double al, const double *__restrict__ z, const double *__restrict__ kz,
                                const double *__restrict__ az, int64_t n, double *__restrict__ x,
                                double *__restrict__ kx, double *__restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] += al * z[i];
  kx[i] += al * kz[i];
  r[i] -= al * az[i];
}

// z = r + be z; kz = kr + be kz
__global__ void e_dir_kernel(const double *__restrict__ r, const double *__restrict__ kr, double be, int64_t n,
                             double *__restrict__ z, double *__restrict__ kz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  z[i] = r[i] + be * z[i];
  kz[i] = kr[i] + be * kz[i];
}

// y = alpha x + beta y (FP64; y is not read when beta is 0), optional FP32 copy
__global__ void e_axpby_kernel(double al, const double *__restrict__ x, double be, int64_t n,
                               double *__restrict__ y, float *__restrict__ y32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = be == 0.0 ? al * x[i] : al * x[i] + be * y[i];
  if (y) y[i] = v;
  if (y32) y32[i] = (float)v;
}

// y = (double)x
__global__ void e_widen_kernel(const float *__restrict__ x, int64_t n, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

// FP32 copy of a base matrix with row stride ldy >= cols (padding written as
// zeros): rows of whole 64-byte lines start on 16-byte boundaries, so the
// stage-2 kernels stage F1 in vector pieces.
__global__ void e_f32_kernel(const double *__restrict__ x, int64_t ldx, float *__restrict__ y, int64_t ldy,
                             int64_t rows, int64_t cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ldy) return;
  const int64_t r = idx / ldy, c = idx - r * ldy;
  y[idx] = c < cols ? (float)x[r * ldx + c] : 0.0f;
}

// ---------------------------------------------------------------------------
namespace {
struct EPlan {
  gvt_plan *plan = nullptr;
  ~EPlan() {
    if (plan) {
      if (plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
      delete plan;
    }
  }
};
dim3 eg1(int64_t n) { return dim3((unsigned)ceil_div(std::max<int64_t>(n, 1), 256)); }

// The solver's state: the plan, base matrices (and FP32 copies), work vectors.
struct Erm {
  gvt_plan *P;
  int kind, loss, prec;
  const double *D, *T;
  int64_t d, t, ldd, ldt, n;
  const double *y;
  double lam;
  hipStream_t s;
  float *D32 = nullptr, *T32 = nullptr;
  int64_t ldd32 = 0, ldt32 = 0;  // row strides of the FP32 copies
  double *part = nullptr, *fold = nullptr;  // 2 x ENB partials, 8 fold results
  float *in32 = nullptr, *out32 = nullptr;  // FP32 product staging

  // Y = K X (FP64 vectors; an FP32 product through the staging vectors)
  void K(const double *X, double *Y) {
    if (prec == GVT_F64) {
      plan_execute(P, GVT_F64, D, ldd, T, ldt, X, 1, n, Y, n, s);
    } else {
      e_axpby_kernel<<<eg1(n), 256, 0, s>>>(1.0, X, 0.0, n, nullptr, in32);  // in32 = (float)X
      plan_execute(P, GVT_F32, D32, ldd32, T32, ldt32, in32, 1, n, out32, n, s);
      e_widen_kernel<<<eg1(n), 256, 0, s>>>(out32, n, Y);
    }
  }
  std::vector<double> fetch(int nsum) {
    e_fold_kernel<<<nsum, EB, 0, s>>>(part, fold);
    std::vector<double> h(nsum);
    GVT_HIP_CHECK(hipMemcpyAsync(h.data(), fold, nsum * 8, hipMemcpyDeviceToHost, s));
    GVT_HIP_CHECK(hipStreamSynchronize(s));
    return h;
  }
  double dot(const double *x, const double *y_) {
    e_dot_kernel<double><<<ENB, EB, 0, s>>>(x, y_, n, part);
    return fetch(1)[0];
  }
  // J at a (p = K a into p); u = g + lambda a; dv = d; returns J
  double risk(const double *a, double *p, double *u, double *dv, double *tmp) {
    K(a, tmp);
    e_loss_kernel<double><<<ENB, EB, 0, s>>>(loss, tmp, y, a, lam, n, p, u, dv, part);
    const std::vector<double> h = fetch(2);
    return h[0] + 0.5 * lam * h[1];
  }
};
}  // namespace

static void erm_common_checks(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *&T,
                              int64_t &t, int64_t &ldt, const int32_t *c, const int32_t *e, int64_t n,
                              const double *y, double lambda) {
  GVT_REQUIRE(loss >= GVT_LOSS_SQUARED && loss <= GVT_LOSS_HINGE, GVT_ERR_ARG, "unknown loss");
  GVT_REQUIRE(n >= 1 && D && c && e && y, GVT_ERR_ARG, "null argument or n < 1");
  GVT_REQUIRE(lambda >= 0 && std::isfinite(lambda), GVT_ERR_ARG, "lambda must be >= 0");
  const bool hom = kind == GVT_SYMMETRIC || kind == GVT_ANTISYMMETRIC || kind == GVT_RANKING ||
                   kind == GVT_MLPK;
  if (hom) { T = D; t = d; ldt = ldd; }
  GVT_REQUIRE(T, GVT_ERR_ARG, "null T");
  GVT_REQUIRE(ldd >= d && ldt >= t, GVT_ERR_ARG, "ld < cols");
}

int erm_objective_impl(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                       int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                       const double *a, double lambda, double *grad, double *obj_out, hipStream_t s) {
  erm_common_checks(kind, loss, D, d, ldd, T, t, ldt, c, e, n, y, lambda);
  GVT_REQUIRE(a && obj_out, GVT_ERR_ARG, "null a or obj_out");
  EPlan ep;
  ep.plan = new gvt_plan();
  plan_build(ep.plan, &kind, 1, d, d, t, t, c, e, n, c, e, n, GVT_FLAG_SYMMETRIC_BASES, s, 1);
  GVT_REQUIRE(!ep.plan->dense, GVT_ERR_UNSUPPORTED, "complete-data training grid: use the dense product");
  DevMem m_v, m_part;
  double *vb = (double *)m_v.ensure((size_t)n * 8 * 2);
  double *p = vb, *u = vb + n;
  Erm E{ep.plan, kind, loss, GVT_F64, D, T, d, t, ldd, ldt, n, y, lambda, s};
  E.part = (double *)m_part.ensure((size_t)ENB * 8 * 2 + 8 * 8);
  E.fold = E.part + 2 * ENB;
  double *tmp = grad ? grad : (double *)nullptr;
  DevMem m_tmp;
  if (!tmp) tmp = (double *)m_tmp.ensure((size_t)n * 8);
  *obj_out = E.risk(a, p, u, nullptr, tmp);
  if (grad) E.K(u, grad);
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  check_launch(s);
  GVT_REQUIRE(std::isfinite(*obj_out), GVT_ERR_BREAKDOWN, "non-finite objective");
  return GVT_OK;
}

int erm_newton_impl(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                    int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y, double lambda,
                    double *A, int max_newton, int max_cg, double tol, int mprec, int *steps_out,
                    int *cg_out, double *obj_out, double *gnorm_out, double *gnorm0_out, hipStream_t s) {
  erm_common_checks(kind, loss, D, d, ldd, T, t, ldt, c, e, n, y, lambda);
  GVT_REQUIRE(loss != GVT_LOSS_HINGE, GVT_ERR_UNSUPPORTED, "the hinge loss has no Hessian: use its subgradient");
  GVT_REQUIRE(A && max_newton >= 0 && max_cg >= 1 && tol >= 0, GVT_ERR_ARG, "bad A/max_newton/max_cg/tol");
  GVT_REQUIRE(mprec == GVT_F64 || mprec == GVT_F32, GVT_ERR_UNSUPPORTED, "products run in GVT_F64 or GVT_F32");
  EPlan ep;
  ep.plan = new gvt_plan();
  plan_build(ep.plan, &kind, 1, d, d, t, t, c, e, n, c, e, n, GVT_FLAG_SYMMETRIC_BASES, s, 1);
  GVT_REQUIRE(!ep.plan->dense, GVT_ERR_UNSUPPORTED, "complete-data training grid: use the dense product");
  Erm E{ep.plan, kind, loss, mprec, D, T, d, t, ldd, ldt, n, y, lambda, s};
  DevMem m_vec, m_part, m_32, m_D32, m_T32;
  // p, u (g + lambda a), dv, grad, x, kx, r, kr, z, kz, az, tmp
  double *vb = (double *)m_vec.ensure((size_t)n * 8 * 12);
  double *p = vb, *u = p + n, *dv = u + n, *grad = dv + n, *x = grad + n, *kx = x + n, *r = kx + n;
  double *kr = r + n, *z = kr + n, *kz = z + n, *az = kz + n, *tmp = az + n;
  E.part = (double *)m_part.ensure((size_t)ENB * 8 * 2 + 8 * 8);
  E.fold = E.part + 2 * ENB;
  if (mprec == GVT_F32) {
    float *f = (float *)m_32.ensure((size_t)n * 4 * 2);
    E.in32 = f;
    E.out32 = f + n;
    E.ldd32 = (d + 15) / 16 * 16;
    E.D32 = (float *)m_D32.ensure((size_t)d * E.ldd32 * 4);
    e_f32_kernel<<<eg1(d * E.ldd32), 256, 0, s>>>(D, ldd, E.D32, E.ldd32, d, d);
    const bool hom = T == D;
    if (!hom) {
      E.ldt32 = (t + 15) / 16 * 16;
      E.T32 = (float *)m_T32.ensure((size_t)t * E.ldt32 * 4);
      e_f32_kernel<<<eg1(t * E.ldt32), 256, 0, s>>>(T, ldt, E.T32, E.ldt32, t, t);
    } else {
      E.T32 = E.D32;
      E.ldt32 = E.ldd32;
    }
  }
  GVT_HIP_CHECK(hipMemsetAsync(A, 0, (size_t)n * 8, s));
  int steps = 0, cg_total = 0;
  double J = 0.0, gn = 0.0, g0 = -1.0;
  while (true) {
    J = E.risk(A, p, u, dv, tmp);
    E.K(u, grad);
    gn = std::sqrt(E.dot(grad, grad));
    if (g0 < 0) g0 = gn;
    GVT_REQUIRE(std::isfinite(J) && std::isfinite(gn), GVT_ERR_BREAKDOWN, "non-finite objective or gradient");
    if (steps >= max_newton || gn <= tol * g0 || gn == 0.0) break;
    const double eta = std::min(0.5, std::sqrt(gn / g0));
    // CG on (D K + lambda I) delta = -(g + lambda a) in the K inner product, from 0
    GVT_HIP_CHECK(hipMemsetAsync(x, 0, (size_t)n * 8, s));
    GVT_HIP_CHECK(hipMemsetAsync(kx, 0, (size_t)n * 8, s));
    e_axpby_kernel<<<eg1(n), 256, 0, s>>>(-1.0, u, 0.0, n, r, nullptr);      // r = -(g + lambda a)
    e_axpby_kernel<<<eg1(n), 256, 0, s>>>(-1.0, grad, 0.0, n, kr, nullptr);  // K r = -grad
    e_axpby_kernel<<<eg1(n), 256, 0, s>>>(1.0, r, 0.0, n, z, nullptr);
    e_axpby_kernel<<<eg1(n), 256, 0, s>>>(1.0, kr, 0.0, n, kz, nullptr);
    double rho = E.dot(r, kr);
    const double rho0 = rho;
    bool moved = false;
    for (int k = 0; k < max_cg; ++k) {
      e_az_kernel<<<ENB, EB, 0, s>>>(dv, kz, z, lambda, n, az, E.part);
      const double zaz = E.fetch(1)[0];
      ++cg_total;
      if (!(zaz > 0.0 && rho > 0.0)) break;
      const double al = rho / zaz;
      e_cgstep_kernel<<<eg1(n), 256, 0, s>>>(al, z, kz, az, n, x, kx, r);
      moved = true;
      E.K(r, kr);
      const double rho_new = E.dot(r, kr);
      if (!(rho_new > 0.0) || std::sqrt(rho_new) <= eta * std::sqrt(rho0)) break;
      e_dir_kernel<<<eg1(n), 256, 0, s>>>(r, kr, rho_new / rho, n, z, kz);
      rho = rho_new;
    }
    if (!moved) break;
    // backtracking on J(a + t x) with p + t Kx (no product)
    const double slope = E.dot(grad, x);
    double tt = 1.0;
    for (int k = 0; k < 31; ++k) {
      e_trial_kernel<<<ENB, EB, 0, s>>>(loss, p, kx, A, x, y, tt, n, E.part);
      const std::vector<double> h = E.fetch(2);
      const double Jt = h[0] + 0.5 * lambda * h[1];
      if (Jt <= J + 1e-4 * tt * slope) break;
      tt *= 0.5;
    }
    e_axpby_kernel<<<eg1(n), 256, 0, s>>>(tt, x, 1.0, n, A, nullptr);
    ++steps;
  }
  check_launch(s);
  if (steps_out) *steps_out = steps;
  if (cg_out) *cg_out = cg_total;
  if (obj_out) *obj_out = J;
  if (gnorm_out) *gnorm_out = gn;
  if (gnorm0_out) *gnorm0_out = g0;
  return (gn <= tol * g0 || gn == 0.0) ? GVT_OK : GVT_NOT_CONVERGED;
}

}  // namespace gvt
