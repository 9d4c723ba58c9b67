// extern "C" entry points declared in include/gvt.h.
#include <algorithm>
#include <cstdarg>
#include <iterator>
#include <map>
#include <mutex>

#include "plan.h"

namespace gvt {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}
void clear_error() { g_last_error.clear(); }

// Released device blocks are kept for reuse instead of freed: hipMalloc costs
// tens of microseconds per call, and a ridge solve (plan, workspaces, CG
// vectors) makes a dozen of them.  A block goes back to its device's cache
// only after that device has finished all queued work, as hipFree would wait,
// so no stream can still be using it when it is handed out again.  A request
// takes the smallest cached block of at least its size and at most twice it;
// each device's cache holds at most kBlockCacheMax bytes (the largest blocks
// beyond that are freed), and an allocation that fails empties the cache and
// tries once more.
namespace {
constexpr size_t kBlockCacheMax = (size_t)4 << 30;
struct BlockCache {
  std::multimap<size_t, void *> by_size;
  size_t held = 0;
};
struct BlockState {
  std::mutex mu;
  std::map<int, BlockCache> cache;  // per device
  std::map<void *, int> dev_of;     // device of each block handed out
};
// never destroyed: blocks may come back while the process exits
BlockState &blocks() {
  static BlockState *s = new BlockState;
  return *s;
}

size_t block_round(size_t n) {
  const size_t g = n >= ((size_t)1 << 20) ? ((size_t)64 << 10) : 256;
  return (n + g - 1) / g * g;
}

void cache_drop_all(BlockCache &c) {
  for (auto &kv : c.by_size) (void)hipFree(kv.second);
  c.by_size.clear();
  c.held = 0;
}
}  // namespace

void *dev_block_get(size_t want, size_t *got) {
  int dev = 0;
  GVT_HIP_CHECK(hipGetDevice(&dev));
  const size_t n = block_round(want);
  BlockState &B = blocks();
  std::lock_guard<std::mutex> lk(B.mu);
  BlockCache &c = B.cache[dev];
  auto it = c.by_size.lower_bound(n);
  if (it != c.by_size.end() && it->first <= 2 * n) {
    void *p = it->second;
    *got = it->first;
    c.held -= it->first;
    c.by_size.erase(it);
    B.dev_of[p] = dev;
    return p;
  }
  void *p = nullptr;
  if (hipMalloc(&p, n) != hipSuccess) {
    (void)hipGetLastError();
    GVT_HIP_CHECK(hipDeviceSynchronize());
    cache_drop_all(c);
    if (hipMalloc(&p, n) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{GVT_ERR_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
  }
  *got = n;
  B.dev_of[p] = dev;
  return p;
}

void dev_block_put(void *p, size_t got) {
  BlockState &B = blocks();
  int dev = -1;
  {
    std::lock_guard<std::mutex> lk(B.mu);
    auto d = B.dev_of.find(p);
    if (d != B.dev_of.end()) {
      dev = d->second;
      B.dev_of.erase(d);
    }
  }
  int cur = 0;
  if (dev < 0 || hipGetDevice(&cur) != hipSuccess) {
    (void)hipFree(p);
    return;
  }
  if (cur != dev) (void)hipSetDevice(dev);
  // The device finishes what may still read or write the block (every stream,
  // as hipFree waits).  The wait holds no lock, so other threads' requests and
  // releases go on meanwhile; the block is not in the cache until it is idle.
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(p);
  } else {
    std::vector<void *> drop;
    {
      std::lock_guard<std::mutex> lk(B.mu);
      BlockCache &c = B.cache[dev];
      c.by_size.emplace(got, p);
      c.held += got;
      while (c.held > kBlockCacheMax && !c.by_size.empty()) {
        auto last = std::prev(c.by_size.end());
        drop.push_back(last->second);
        c.held -= last->first;
        c.by_size.erase(last);
      }
    }
    for (void *q : drop) (void)hipFree(q);
  }
  if (cur != dev) (void)hipSetDevice(cur);
}

// Pinned staging buffer shared by every plan upload of the process (grows on
// demand; gvt_empty_cache frees it).
static std::mutex g_stage_mu;
static void *g_stage = nullptr;
static size_t g_stage_bytes = 0;

// Frees every cached device block on every device and the staging buffer;
// returns the device bytes freed.  Cached blocks are idle (each came back
// after its device had drained), and blocks in use by plans are not cached.
static size_t empty_caches() {
  size_t freed = 0;
  {
    BlockState &B = blocks();
    std::lock_guard<std::mutex> lk(B.mu);
    int cur = 0;
    GVT_HIP_CHECK(hipGetDevice(&cur));
    struct Restore {
      int dev;
      ~Restore() { (void)hipSetDevice(dev); }
    } restore{cur};
    for (auto &kv : B.cache) {
      if (kv.second.by_size.empty()) continue;
      GVT_HIP_CHECK(hipSetDevice(kv.first));
      freed += kv.second.held;
      cache_drop_all(kv.second);
    }
  }
  std::lock_guard<std::mutex> lk(g_stage_mu);
  if (g_stage) (void)hipHostFree(g_stage);
  g_stage = nullptr;
  g_stage_bytes = 0;
  return freed;
}

void Uploads::commit(DevMem &blob) {
  size_t total = 0;
  for (auto &it : items) total += (it.bytes + 255) & ~size_t(255);
  blob.ensure(total ? total : 256);
  size_t off = 0;
  for (auto &it : items) {
    it.m->view(static_cast<char *>(blob.p) + off, it.bytes);
    off += (it.bytes + 255) & ~size_t(255);
  }
  if (total) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (g_stage_bytes < total) {
      if (g_stage) (void)hipHostFree(g_stage);
      g_stage = nullptr;
      g_stage_bytes = 0;
      const size_t want = std::max<size_t>(total, (size_t)4 << 20);
      GVT_HIP_CHECK(hipHostMalloc(&g_stage, want, hipHostMallocDefault));
      g_stage_bytes = want;
    }
    off = 0;
    for (auto &it : items) {
      if (it.bytes) std::memcpy(static_cast<char *>(g_stage) + off, it.data, it.bytes);
      off += (it.bytes + 255) & ~size_t(255);
    }
    GVT_HIP_CHECK(hipMemcpy(blob.p, g_stage, total, hipMemcpyHostToDevice));
  }
  items.clear();
}

int krr_cg_impl(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                const double *lambdas, int nlam, double *A, int64_t lda, const double *A0,
                int64_t lda0, int max_iter, double tol, int mprec, int check_every,
                int64_t *iters_out, double *relres_out, hipStream_t s);
int krr_minres_impl(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                    int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                    const double *lambdas, int nlam, double *A, int64_t lda, int max_iter, double tol,
                    int mprec, const gvt_validation *val, int check_every, int64_t *iters_out,
                    double *relres_out, int64_t *best_iter_out, double *best_auc_out, double *auc_hist,
                    hipStream_t s);
int erm_objective_impl(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                       int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                       const double *a, double lambda, double *grad, double *obj_out, hipStream_t s);
int erm_newton_impl(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                    int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y, double lambda,
                    double *A, int max_newton, int max_cg, double tol, int mprec, int *steps_out,
                    int *cg_out, double *obj_out, double *gnorm_out, double *gnorm0_out, hipStream_t s);
int krr_cg_batched_impl(int kind, const gvt_krr_problem *pr, int nprob, const double *lambdas,
                        int nlam, int max_iter, double tol, int mprec, int check_every,
                        int64_t *iters_out, double *relres_out, hipStream_t s);

}  // namespace gvt

using namespace gvt;

extern "C" {

const char *gvt_last_error(void) { return g_last_error.c_str(); }

int gvt_version(void) { return 100; }

int gvt_empty_cache(int64_t *freed_bytes) {
  return guarded([&]() {
    const size_t f = empty_caches();
    if (freed_bytes) *freed_bytes = (int64_t)f;
    return GVT_OK;
  });
}

int gvt_plan_create(gvt_plan_t *plan, const int *kinds, int nkinds, int64_t d_rows, int64_t d_cols,
                    int64_t t_rows, int64_t t_cols, const int32_t *out_a, const int32_t *out_b,
                    int64_t n_out, const int32_t *in_c, const int32_t *in_e, int64_t n_in,
                    int flags, void *stream) {
  return guarded([&]() {
    GVT_REQUIRE(plan, GVT_ERR_ARG, "null plan pointer");
    *plan = nullptr;
    gvt_plan *P = new gvt_plan();
    try {
      plan_build(P, kinds, nkinds, d_rows, d_cols, t_rows, t_cols, out_a, out_b, n_out, in_c, in_e,
                 n_in, flags, (hipStream_t)stream);
      GVT_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    } catch (...) {
      delete P;
      throw;
    }
    *plan = P;
    return GVT_OK;
  });
}

int gvt_plan_destroy(gvt_plan_t plan) {
  return guarded([&]() {
    if (!plan) return GVT_OK;
    (void)hipStreamSynchronize(plan->last_stream);
    delete plan;
    return GVT_OK;
  });
}

int gvt_plan_execute(gvt_plan_t plan, int prec, const void *D, int64_t ldd, const void *T,
                     int64_t ldt, const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu,
                     void *stream) {
  return guarded([&]() {
    plan_execute(plan, prec, D, ldd, T, ldt, V, nrhs, ldv, U, ldu, (hipStream_t)stream);
    return GVT_OK;
  });
}

int gvt_plan_profile(gvt_plan_t plan, int prec, const void *D, int64_t ldd, const void *T,
                     int64_t ldt, const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu,
                     int reps, double *stage_ms, void *stream) {
  return guarded([&]() {
    plan_profile(plan, prec, D, ldd, T, ldt, V, nrhs, ldv, U, ldu, reps, stage_ms,
                 (hipStream_t)stream);
    return GVT_OK;
  });
}

int gvt_plan_info(gvt_plan_t plan, double *info) {
  return guarded([&]() {
    GVT_REQUIRE(plan && info, GVT_ERR_ARG, "null argument");
    info[0] = plan->cost_fma;
    info[1] = plan->dense ? 1.0 : 0.0;
    info[2] = (double)plan->terms.size();
    info[3] = (double)plan->sbufs.size();
    int64_t srows = 0, skeys = 0;
    if (!plan->sbufs.empty()) {
      srows = (int64_t)plan->sbufs[0].rows.size();
      skeys = nkeys_of(plan, plan->sbufs[0].key);
    }
    info[4] = (double)srows;
    info[5] = (double)skeys;
    info[6] = plan->sbufs.empty() ? -1.0 : (double)plan->sbufs[0].key;
    info[7] = (double)plan->uniq[0];
    info[8] = (double)plan->uniq[1];
    info[9] = (double)plan->uniq[2];
    info[10] = (double)plan->uniq[3];
    return GVT_OK;
  });
}

static int oneshot(int prec, const int *kinds, int nkinds, const void *D, int64_t d_rows,
                   int64_t d_cols, int64_t ldd, const void *T, int64_t t_rows, int64_t t_cols,
                   int64_t ldt, const int32_t *out_a, const int32_t *out_b, int64_t n_out,
                   const int32_t *in_c, const int32_t *in_e, int64_t n_in, const void *V,
                   int64_t nrhs, int64_t ldv, void *U, int64_t ldu, int flags, void *stream) {
  return guarded([&]() {
    hipStream_t s = (hipStream_t)stream;
    gvt_plan P;
    plan_build(&P, kinds, nkinds, d_rows, d_cols, t_rows, t_cols, out_a, out_b, n_out, in_c, in_e,
               n_in, flags, s, (int)std::min<int64_t>(nrhs, 8));
    plan_execute(&P, prec, D, ldd, T, ldt, V, nrhs, ldv, U, ldu, s);
    GVT_HIP_CHECK(hipStreamSynchronize(s));
    return GVT_OK;
  });
}

int gvt_matvec(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm, const void *N,
               int64_t n_rows, int64_t n_cols, int64_t ldn, const int32_t *out_a,
               const int32_t *out_b, int64_t n_out, const int32_t *in_c, const int32_t *in_e,
               int64_t n_in, const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu,
               void *stream) {
  const int kind = GVT_KRONECKER;
  return oneshot(prec, &kind, 1, M, m_rows, m_cols, ldm, N, n_rows, n_cols, ldn, out_a, out_b,
                 n_out, in_c, in_e, n_in, V, nrhs, ldv, U, ldu, 0, stream);
}

int gvt_pairwise_matvec(int prec, const int *kinds, int nkinds, const void *D, int64_t d_rows,
                        int64_t d_cols, int64_t ldd, const void *T, int64_t t_rows, int64_t t_cols,
                        int64_t ldt, const int32_t *out_a, const int32_t *out_b, int64_t n_out,
                        const int32_t *in_c, const int32_t *in_e, int64_t n_in, const void *V,
                        int64_t nrhs, int64_t ldv, void *U, int64_t ldu, int flags, void *stream) {
  return oneshot(prec, kinds, nkinds, D, d_rows, d_cols, ldd, T, t_rows, t_cols, ldt, out_a, out_b,
                 n_out, in_c, in_e, n_in, V, nrhs, ldv, U, ldu, flags, stream);
}

int gvt_dense_matvec(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm,
                     const void *N, int64_t n_rows, int64_t n_cols, int64_t ldn, const void *V,
                     int64_t ldv, void *U, int64_t ldu, void *stream) {
  return guarded([&]() {
    GVT_REQUIRE(prec == GVT_F64 || prec == GVT_F32 || prec == GVT_BF16X3 || prec == GVT_BF16X6, GVT_ERR_ARG,
                "unknown precision");
    GVT_REQUIRE(m_rows >= 0 && m_cols >= 0 && n_rows >= 0 && n_cols >= 0, GVT_ERR_ARG,
                "negative size");
    GVT_REQUIRE(ldm >= m_cols && ldn >= n_cols && ldv >= n_cols && ldu >= n_rows, GVT_ERR_ARG,
                "leading dimension too small");
    GVT_REQUIRE((m_rows == 0 || n_rows == 0) || (M && N && V && U), GVT_ERR_ARG, "null pointer");
    dense_matvec(prec, M, m_rows, m_cols, ldm, N, n_rows, n_cols, ldn, V, ldv, U, ldu, nullptr,
                 (hipStream_t)stream);
    return GVT_OK;
  });
}

int gvt_plan_uses_tiles(gvt_plan_t plan, int prec) {
  return guarded([&]() {
    GVT_REQUIRE(plan, GVT_ERR_ARG, "null plan");
    return plan_uses_tiles(plan, prec) || plan_uses_gtiles(plan, prec) ? 1 : 0;
  });
}

int gvt_base_kernel(int kind, int prec, const void *X, int64_t nx, int64_t ldx, const void *Y,
                    int64_t ny, int64_t ldy, int64_t dim, double gamma, void *K, int64_t ldk,
                    void *stream) {
  return guarded([&]() {
    GVT_REQUIRE(kind == GVT_BASE_LINEAR || kind == GVT_BASE_GAUSSIAN, GVT_ERR_ARG, "unknown base kernel");
    GVT_REQUIRE(prec == GVT_F64 || prec == GVT_F32, GVT_ERR_ARG, "base kernels are GVT_F64 or GVT_F32");
    GVT_REQUIRE(nx >= 0 && ny >= 0 && dim >= 0, GVT_ERR_ARG, "negative size");
    GVT_REQUIRE(Y != nullptr || ny == nx, GVT_ERR_ARG, "Y = NULL needs ny == nx");
    GVT_REQUIRE(ldx >= dim && (Y == nullptr || ldy >= dim) && ldk >= ny, GVT_ERR_ARG,
                "leading dimension too small");
    GVT_REQUIRE(nx == 0 || ny == 0 || (K && (dim == 0 || (X))), GVT_ERR_ARG, "null pointer");
    GVT_REQUIRE(std::isfinite(gamma), GVT_ERR_ARG, "gamma is not finite");
    base_kernel(kind, prec, X, nx, ldx, Y, ny, ldy, dim, gamma, K, ldk, (hipStream_t)stream);
    return GVT_OK;
  });
}

int gvt_tanimoto_kernel(int prec, const uint64_t *X, int64_t nx, int64_t ldx, const uint64_t *Y,
                        int64_t ny, int64_t ldy, int64_t nbits, void *K, int64_t ldk, void *stream) {
  return guarded([&]() {
    GVT_REQUIRE(prec == GVT_F64 || prec == GVT_F32, GVT_ERR_ARG, "Tanimoto kernels are GVT_F64 or GVT_F32");
    GVT_REQUIRE(nx >= 0 && ny >= 0 && nbits >= 0, GVT_ERR_ARG, "negative size");
    GVT_REQUIRE(Y != nullptr || ny == nx, GVT_ERR_ARG, "Y = NULL needs ny == nx");
    const int64_t words = (nbits + 63) / 64;
    GVT_REQUIRE(ldx >= words && (Y == nullptr || ldy >= words) && ldk >= ny, GVT_ERR_ARG,
                "leading dimension too small");
    GVT_REQUIRE(nx == 0 || ny == 0 || (X && K), GVT_ERR_ARG, "null pointer");
    tanimoto_kernel_matrix(prec, X, nx, ldx, Y, ny, ldy, nbits, K, ldk, (hipStream_t)stream);
    return GVT_OK;
  });
}

int gvt_dense_matvec_checked(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm,
                             const void *N, int64_t n_rows, int64_t n_cols, int64_t ldn,
                             const void *V, int64_t ldv, void *U, int64_t ldu, double max_relerr,
                             double *relerr_out, int *prec_out, void *stream) {
  return guarded([&]() {
    GVT_REQUIRE(prec == GVT_F64 || prec == GVT_F32 || prec == GVT_BF16X3 || prec == GVT_BF16X6, GVT_ERR_ARG,
                "unknown precision");
    GVT_REQUIRE(m_rows >= 0 && m_cols >= 0 && n_rows >= 0 && n_cols >= 0, GVT_ERR_ARG,
                "negative size");
    GVT_REQUIRE(ldm >= m_cols && ldn >= n_cols && ldv >= n_cols && ldu >= n_rows, GVT_ERR_ARG,
                "leading dimension too small");
    GVT_REQUIRE((m_rows == 0 || n_rows == 0) || (M && N && V && U), GVT_ERR_ARG, "null pointer");
    GVT_REQUIRE(relerr_out && prec_out && max_relerr >= 0.0, GVT_ERR_ARG,
                "null output or negative bound");
    const hipStream_t s = (hipStream_t)stream;
    int p = prec;
    double est = 0.0;
    for (;;) {
      dense_matvec(p, M, m_rows, m_cols, ldm, N, n_rows, n_cols, ldn, V, ldv, U, ldu, nullptr, s);
      est = dense_sample_relerr(p, M, m_rows, m_cols, ldm, N, n_rows, n_cols, ldn, V, ldv, U, ldu, s);
      // a sampled estimate: escalate once it reaches half the bound
      if (max_relerr <= 0.0 || !(est > 0.5 * max_relerr)) break;
      if (p == GVT_BF16X3) p = GVT_BF16X6;
      else if (p == GVT_BF16X6) p = GVT_F32;
      else break;
    }
    *relerr_out = est;
    *prec_out = p;
    return (max_relerr > 0.0 && !(est <= max_relerr)) ? GVT_TOL_NOT_MET : GVT_OK;
  });
}

int gvt_dense_matvec_noalloc(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm,
                             const void *N, int64_t n_rows, int64_t n_cols, int64_t ldn,
                             const void *V, int64_t ldv, void *U, int64_t ldu, void *stream) {
  return guarded([&]() {
    GVT_REQUIRE(prec == GVT_F64 || prec == GVT_F32 || prec == GVT_BF16X3 || prec == GVT_BF16X6, GVT_ERR_ARG,
                "unknown precision");
    GVT_REQUIRE(m_rows >= 0 && m_cols >= 0 && n_rows >= 0 && n_cols >= 0, GVT_ERR_ARG,
                "negative size");
    GVT_REQUIRE(ldm >= m_cols && ldn >= n_cols && ldv >= n_cols && ldu >= n_rows, GVT_ERR_ARG,
                "leading dimension too small");
    GVT_REQUIRE((m_rows == 0 || n_rows == 0) || (M && N && V && U), GVT_ERR_ARG, "null pointer");
    const size_t need = dense_workspace_bytes(prec, m_rows, m_cols, n_rows, n_cols);
    if (need == 0) return GVT_OK;
    if (need > kDenseScratchBytes) {
      set_error("gvt_dense_matvec_noalloc: this product needs %zu bytes of workspace, more than the "
                "%zu bytes of the static workspace", need, kDenseScratchBytes);
      return GVT_ERR_ARG;
    }
    dense_matvec(prec, M, m_rows, m_cols, ldm, N, n_rows, n_cols, ldn, V, ldv, U, ldu,
                 dense_scratch_ptr(), (hipStream_t)stream);
    return GVT_OK;
  });
}

int gvt_krr_cg(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
               int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
               const double *lambdas, int nlam, double *A, int64_t lda, const double *A0,
               int64_t lda0, int max_iter, double tol, int matvec_prec, int check_every,
               int64_t *iters_out, double *relres_out, void *stream) {
  return guarded([&]() {
    return krr_cg_impl(kind, D, d, ldd, T, t, ldt, c, e, n, y, lambdas, nlam, A, lda, A0, lda0,
                       max_iter, tol, matvec_prec, check_every, iters_out, relres_out,
                       (hipStream_t)stream);
  });
}

int gvt_krr_minres(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                   int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                   const double *lambdas, int nlam, double *A, int64_t lda, int max_iter, double tol,
                   int matvec_prec, const gvt_validation *val, int check_every, int64_t *iters_out,
                   double *relres_out, int64_t *best_iter_out, double *best_auc_out,
                   double *auc_hist, void *stream) {
  return guarded([&]() {
    return krr_minres_impl(kind, D, d, ldd, T, t, ldt, c, e, n, y, lambdas, nlam, A, lda, max_iter, tol,
                           matvec_prec, val, check_every, iters_out, relres_out, best_iter_out,
                           best_auc_out, auc_hist, (hipStream_t)stream);
  });
}

int gvt_erm_objective(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T,
                      int64_t t, int64_t ldt, const int32_t *c, const int32_t *e, int64_t n,
                      const double *y, const double *a, double lambda, double *grad, double *obj_out,
                      void *stream) {
  return guarded([&]() {
    return erm_objective_impl(kind, loss, D, d, ldd, T, t, ldt, c, e, n, y, a, lambda, grad, obj_out,
                              (hipStream_t)stream);
  });
}

int gvt_erm_newton(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T,
                   int64_t t, int64_t ldt, const int32_t *c, const int32_t *e, int64_t n,
                   const double *y, double lambda, double *A, int max_newton, int max_cg, double tol,
                   int matvec_prec, int *steps_out, int *cg_iters_out, double *obj_out,
                   double *gnorm_out, double *gnorm0_out, void *stream) {
  return guarded([&]() {
    return erm_newton_impl(kind, loss, D, d, ldd, T, t, ldt, c, e, n, y, lambda, A, max_newton, max_cg, tol,
                           matvec_prec, steps_out, cg_iters_out, obj_out, gnorm_out, gnorm0_out,
                           (hipStream_t)stream);
  });
}

int gvt_krr_cg_batched(int kind, const gvt_krr_problem *problems, int nprob, const double *lambdas,
                       int nlam, int max_iter, double tol, int matvec_prec, int check_every,
                       int64_t *iters_out, double *relres_out, void *stream) {
  return guarded([&]() {
    return krr_cg_batched_impl(kind, problems, nprob, lambdas, nlam, max_iter, tol, matvec_prec,
                               check_every, iters_out, relres_out, (hipStream_t)stream);
  });
}

}  // extern "C"
