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
#include <cmath>
#include <cstring>

#include "plan.h"

namespace gvt {

static constexpr int RB = 256;   // reduction block size
static constexpr int RNB = 240;  // reduction grid (fixed for determinism)
static_assert(RNB <= RB, "partials are folded by one block");

enum CgState { CG_DONE = 0, CG_ACTIVE = 1, CG_PENDING = 2, CG_BREAKDOWN = 3, CG_MAXITER = 4 };

struct CgScalars {
  double rho, pw, alpha, beta, ynorm;
  int state, iters, pad0, pad1;
};

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = RB / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
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

// Fixed-tree fold of the RNB block partials of system l by one 256-thread block.
__device__ __forceinline__ double fold_partials(const double *partial, int nlam, int l, double *sh) {
  const double v = threadIdx.x < RNB ? partial[threadIdx.x * nlam + l] : 0.0;
  return block_sum(v, sh);
}

// w = K p (+ FP32 product cast) + lambda p ; partial dot p.w
template <class TW>
__global__ __launch_bounds__(RB) void cg_pw_kernel(const TW *__restrict__ wraw, double *__restrict__ w,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ lam, int64_t n,
                                                   int nlam, const CgScalars *__restrict__ sc,
                                                   double *__restrict__ partial) {
  __shared__ double sh[RB];
  for (int l = 0; l < nlam; ++l) {
    double acc = 0.0;
    if (sc[l].state == CG_ACTIVE) {
      const double lm = lam[l];
      for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)RNB * RB) {
        const double pi = p[i + l * n];
        const double wi = (double)wraw[i + l * n] + lm * pi;
        w[i + l * n] = wi;
        acc += pi * wi;
      }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x * nlam + l] = s;
  }
}

// one block per system
__global__ __launch_bounds__(RB) void cg_alpha_kernel(CgScalars *sc, const double *__restrict__ partial,
                                                      int nlam) {
  __shared__ double sh[RB];
  const int l = blockIdx.x;
  if (sc[l].state != CG_ACTIVE) return;  // uniform per block
  const double pw = fold_partials(partial, nlam, l, sh);
  if (threadIdx.x != 0) return;
  sc[l].pw = pw;
  if (!(pw > 0.0) || !isfinite(pw)) {
    sc[l].state = CG_BREAKDOWN;
    return;
  }
  sc[l].alpha = sc[l].rho / pw;
}

// a += alpha p; r -= alpha w; partial r.r
__global__ __launch_bounds__(RB) void cg_update_kernel(double *__restrict__ a, int64_t lda,
                                                       double *__restrict__ r,
                                                       const double *__restrict__ p,
                                                       const double *__restrict__ w, int64_t n,
                                                       int nlam, const CgScalars *__restrict__ sc,
                                                       double *__restrict__ partial) {
  __shared__ double sh[RB];
  for (int l = 0; l < nlam; ++l) {
    double acc = 0.0;
    if (sc[l].state == CG_ACTIVE) {
      const double al = sc[l].alpha;
      for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)RNB * RB) {
        a[i + l * lda] += al * p[i + l * n];
        const double ri = r[i + l * n] - al * w[i + l * n];
        r[i + l * n] = ri;
        acc += ri * ri;
      }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x * nlam + l] = s;
  }
}

__global__ __launch_bounds__(RB) void cg_beta_kernel(CgScalars *sc, const double *__restrict__ partial,
                                                     int nlam, double tol, int max_iter, int lowprec) {
  __shared__ double sh[RB];
  const int l = blockIdx.x;
  if (sc[l].state != CG_ACTIVE) return;  // uniform per block
  const double rho_new = fold_partials(partial, nlam, l, sh);
  if (threadIdx.x != 0) return;
  sc[l].iters += 1;
  if (!isfinite(rho_new)) {
    sc[l].state = CG_BREAKDOWN;
    return;
  }
  sc[l].beta = rho_new / sc[l].rho;
  sc[l].rho = rho_new;
  if (sqrt(rho_new) / sc[l].ynorm < tol) {
    sc[l].state = lowprec ? CG_PENDING : CG_DONE;
  } else if (sc[l].iters >= max_iter) {
    sc[l].state = CG_MAXITER;
  }
}

// p = r + beta p  (active systems)
__global__ void cg_p_kernel(double *__restrict__ p, const double *__restrict__ r, int64_t n, int nlam,
                            const CgScalars *__restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int l = 0; l < nlam; ++l)
    if (sc[l].state == CG_ACTIVE) p[i + l * n] = r[i + l * n] + sc[l].beta * p[i + l * n];
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

__global__ void mat_to_f32_kernel(const double *__restrict__ x, int64_t ldx, float *__restrict__ y,
                                  int64_t rows, int64_t cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols, c = idx - r * cols;
  y[idx] = (float)x[r * ldx + c];
}

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
  plan_build(P, &kind, 1, d, d, t, t, c, e, n, c, e, n, GVT_FLAG_SYMMETRIC_BASES, s);
  GVT_REQUIRE(!P->dense, GVT_ERR_UNSUPPORTED, "complete-data training grid: use the dense product");

  // workspace
  DevMem m_r, m_p, m_w, m_wraw, m_p32, m_w32, m_D32, m_T32, m_part, m_sc, m_lam, m_tmp;
  const size_t nv = (size_t)n * nlam;
  double *r = (double *)m_r.ensure(nv * 8);
  double *p = (double *)m_p.ensure(nv * 8);
  double *w = (double *)m_w.ensure(nv * 8);
  double *wraw = (double *)m_wraw.ensure(nv * 8);
  double *part = (double *)m_part.ensure((size_t)RNB * nlam * 8);
  CgScalars *sc = (CgScalars *)m_sc.ensure(sizeof(CgScalars) * nlam);
  double *lam = (double *)m_lam.ensure(nlam * 8);
  double *tmp = (double *)m_tmp.ensure(64 * 8);
  float *p32 = nullptr, *w32 = nullptr, *D32 = nullptr, *T32 = nullptr;
  GVT_HIP_CHECK(hipMemcpyAsync(lam, lambdas, nlam * 8, hipMemcpyHostToDevice, s));
  if (mprec == GVT_F32) {
    p32 = (float *)m_p32.ensure(nv * 4);
    w32 = (float *)m_w32.ensure(nv * 4);
    D32 = (float *)m_D32.ensure((size_t)d * d * 4);
    mat_to_f32_kernel<<<g1(d * d), 256, 0, s>>>(D, ldd, D32, d, d);
    if (!hom) {
      T32 = (float *)m_T32.ensure((size_t)t * t * 4);
      mat_to_f32_kernel<<<g1(t * t), 256, 0, s>>>(T, ldt, T32, t, t);
    } else {
      T32 = D32;
    }
  }
  auto matvec64 = [&](const double *X, double *Y) {
    plan_execute(P, GVT_F64, D, ldd, T, ldt, X, nlam, n, Y, n, s);
  };

  // ||y||
  dot_partial_kernel<<<RNB, RB, 0, s>>>(y, 0, y, 0, n, 1, part);
  fold_kernel<<<1, RB, 0, s>>>(part, 1, tmp);
  double ynorm2 = 0.0;
  GVT_HIP_CHECK(hipMemcpyAsync(&ynorm2, tmp, 8, hipMemcpyDeviceToHost, s));
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  const double ynorm = std::sqrt(ynorm2);
  GVT_REQUIRE(std::isfinite(ynorm), GVT_ERR_BREAKDOWN, "non-finite labels");

  // init: a = A0 or 0; r = y - (K + lambda) a; p = r; rho = r.r
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
  } else {
    bcast_col_kernel<<<g1(n), 256, 0, s>>>(y, r, n, n, nlam);
    dot_partial_kernel<<<RNB, RB, 0, s>>>(r, n, r, n, n, nlam, part);
  }
  fold_kernel<<<nlam, RB, 0, s>>>(part, nlam, tmp);
  std::vector<double> rho0(nlam);
  GVT_HIP_CHECK(hipMemcpyAsync(rho0.data(), tmp, nlam * 8, hipMemcpyDeviceToHost, s));
  copy_cols_kernel<<<g1(n), 256, 0, s>>>(r, n, p, n, n, nlam, -1, nullptr);
  GVT_HIP_CHECK(hipStreamSynchronize(s));
  for (int l = 0; l < nlam; ++l) {
    std::memset(&hs[l], 0, sizeof(CgScalars));
    hs[l].rho = rho0[l];
    hs[l].ynorm = ynorm;
    hs[l].state = (std::sqrt(rho0[l]) / ynorm < tol) ? CG_DONE : CG_ACTIVE;
  }
  GVT_HIP_CHECK(hipMemcpyAsync(sc, hs.data(), sizeof(CgScalars) * nlam, hipMemcpyHostToDevice, s));

  const int lowprec = mprec == GVT_F32 ? 1 : 0;
  auto iteration = [&]() {
    if (lowprec) {
      to_f32_kernel<<<g1((int64_t)nv), 256, 0, s>>>(p, p32, (int64_t)nv);
      plan_execute(P, GVT_F32, D32, d, T32, t, p32, nlam, n, w32, n, s);
      cg_pw_kernel<float><<<RNB, RB, 0, s>>>(w32, w, p, lam, n, nlam, sc, part);
    } else {
      matvec64(p, wraw);
      cg_pw_kernel<double><<<RNB, RB, 0, s>>>(wraw, w, p, lam, n, nlam, sc, part);
    }
    cg_alpha_kernel<<<nlam, RB, 0, s>>>(sc, part, nlam);
    cg_update_kernel<<<RNB, RB, 0, s>>>(A, lda, r, p, w, n, nlam, sc, part);
    cg_beta_kernel<<<nlam, RB, 0, s>>>(sc, part, nlam, tol, max_iter, lowprec);
    cg_p_kernel<<<g1(n), 256, 0, s>>>(p, r, n, nlam, sc);
  };

  // warm-up layout of plan workspaces (allocation must not happen inside a capture)
  // by running one iteration eagerly, then capture blocks of check_every iterations.
  // graphs need a capturable (non-null) stream
  const bool use_graph = s != nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int status = GVT_OK;
  int total_iter = 0;
  bool first = true;
  while (true) {
    bool any_active = false;
    for (int l = 0; l < nlam; ++l) any_active |= hs[l].state == CG_ACTIVE;
    if (!any_active) {
      // certify systems whose low-precision recurrence claims convergence
      bool pending = false;
      for (int l = 0; l < nlam; ++l) pending |= hs[l].state == CG_PENDING;
      if (!pending) break;
      copy_cols_kernel<<<g1(n), 256, 0, s>>>(A, lda, w, n, n, nlam, -1, nullptr);
      matvec64(w, wraw);
      residual_kernel<<<RNB, RB, 0, s>>>(y, wraw, A, lda, lam, n, nlam, w, part);
      fold_kernel<<<nlam, RB, 0, s>>>(part, nlam, tmp);
      std::vector<double> rt(nlam);
      GVT_HIP_CHECK(hipMemcpyAsync(rt.data(), tmp, nlam * 8, hipMemcpyDeviceToHost, s));
      GVT_HIP_CHECK(hipStreamSynchronize(s));
      for (int l = 0; l < nlam; ++l) {
        if (hs[l].state != CG_PENDING) continue;
        if (std::sqrt(rt[l]) / ynorm < tol) {
          hs[l].state = CG_DONE;
        } else if (hs[l].iters >= max_iter) {
          hs[l].state = CG_MAXITER;
        } else {
          hs[l].state = CG_ACTIVE;  // restart from the true residual
          hs[l].rho = rt[l];
        }
      }
      // r = w (true residual) and p = r for restarted systems
      GVT_HIP_CHECK(hipMemcpyAsync(sc, hs.data(), sizeof(CgScalars) * nlam, hipMemcpyHostToDevice, s));
      copy_cols_kernel<<<g1(n), 256, 0, s>>>(w, n, r, n, n, nlam, CG_ACTIVE, sc);
      copy_cols_kernel<<<g1(n), 256, 0, s>>>(w, n, p, n, n, nlam, CG_ACTIVE, sc);
      continue;
    }
    if (first) {
      // one eager iteration lays out every workspace (no allocation may happen
      // inside a capture); then capture a block of check_every iterations
      iteration();
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
  bool all_done = true;
  for (int l = 0; l < nlam; ++l) {
    iters_out[l] = hs[l].iters;
    relres_out[l] = std::sqrt(rt[l]) / ynorm;
    if (hs[l].state == CG_BREAKDOWN) status = GVT_ERR_BREAKDOWN;
    if (hs[l].state != CG_DONE) all_done = false;
  }
  if (status == GVT_OK && !all_done) status = GVT_NOT_CONVERGED;
  return status;
}

}  // namespace gvt
