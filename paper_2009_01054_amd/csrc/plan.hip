// Plan construction and execution.
//
// A plan turns (kinds, base-matrix shapes, output pairs, input pairs) into a
// term program: Corollary 1 writes every pairwise kernel as a sum of
// Kronecker products whose index selectors come from the commutation and
// unification rules R(d,t)P = R(t,d), R(d,t)Q = R(d,d).  Each two-factor term
// is applied with the generalized vec trick (Theorem 1) in whichever stage
// order is cheaper; one-factor terms (a base matrix times an all-ones
// factor) collapse to segment sums, a GEMV and a gather; the Cartesian
// kernel's identity factors become sparse key matches.  Identical stage-1
// scatters, segment sums, GEMVs and terms are shared across all kinds of the
// plan.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include <chrono>
#include <cstdlib>
#include <exception>
#include <thread>

#include "plan.h"
#include "tuning.h"

namespace gvt {

// GVT_PLAN_TIMING=1 prints the host time of each plan phase to stderr.
struct PhaseTimer {
  bool on = std::getenv("GVT_PLAN_TIMING") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void lap(const char *what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[gvt plan] %-24s %8.3f ms\n", what,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

int64_t rows_of(const gvt_plan *P, int f) { return f == FD ? P->d_rows : P->t_rows; }
int64_t cols_of(const gvt_plan *P, int f) { return f == FD ? P->d_cols : P->t_cols; }
int64_t nkeys_of(const gvt_plan *P, int key) { return key == SC ? P->d_cols : P->t_cols; }

static bool kind_homogeneous(int k) {
  return k == GVT_SYMMETRIC || k == GVT_ANTISYMMETRIC || k == GVT_RANKING || k == GVT_MLPK;
}

namespace {

struct RawTerm {
  int type;
  int a0, a1, a2, a3, a4, a5;  // meaning depends on type
  bool operator<(const RawTerm &o) const {
    return std::tie(type, a0, a1, a2, a3, a4, a5) <
           std::tie(o.type, o.a0, o.a1, o.a2, o.a3, o.a4, o.a5);
  }
};

// G(fdot, fsc; x, y; key, other): u_i = sum_j fdot[x_i, key_j] fsc[y_i, other_j] v_j
RawTerm G(int fdot, int fsc, int x, int y, int key, int other) {
  return RawTerm{TG, fdot, fsc, x, y, key, other};
}
// O(f, sq; x, key): u_i = sum_j f[x_i, key_j]^{1|2} v_j
RawTerm O(int f, int sq, int x, int key) { return RawTerm{TO, f, sq, x, key, 0, 0}; }
// M(f; x, outkey, key, other): u_i = sum_{j: key_j == outkey_i} f[x_i, other_j] v_j
RawTerm M(int f, int x, int outkey, int key, int other) {
  return RawTerm{TM, f, x, outkey, key, other, 0};
}

// Corollary 1 term lists (readings: anti-symmetric follows the sign of its
// Table 4b function, i.e. (I - P)(D x D); MLPK uses (I - Q)^T on the right).
std::vector<std::pair<RawTerm, double>> expand_kind(int kind, bool hom) {
  const int FTm = hom ? FD : FT;
  switch (kind) {
    case GVT_KRONECKER:  // D (x) T
      return {{G(FD, FTm, SA, SB, SC, SE), 1.0}};
    case GVT_LINEAR:  // D (x) 1 + 1 (x) T
      return {{O(FD, 0, SA, SC), 1.0}, {O(FTm, 0, SB, SE), 1.0}};
    case GVT_POLY2D:  // Q(D x D)Q^T + 2 D x T + PQ(T x T)Q^T P
      return {{O(FD, 1, SA, SC), 1.0}, {G(FD, FTm, SA, SB, SC, SE), 2.0}, {O(FTm, 1, SB, SE), 1.0}};
    case GVT_CARTESIAN:  // D (x) I + I (x) T
      return {{M(FD, SA, SB, SE, SC), 1.0}, {M(FTm, SB, SA, SC, SE), 1.0}};
    case GVT_SYMMETRIC:  // (P + I)(D x D)
      return {{G(FD, FD, SA, SB, SC, SE), 1.0}, {G(FD, FD, SB, SA, SC, SE), 1.0}};
    case GVT_ANTISYMMETRIC:  // (I - P)(D x D)
      return {{G(FD, FD, SA, SB, SC, SE), 1.0}, {G(FD, FD, SB, SA, SC, SE), -1.0}};
    case GVT_RANKING:  // (I - P)(D x 1)(I - P)
      return {{O(FD, 0, SA, SC), 1.0}, {O(FD, 0, SA, SE), -1.0},
              {O(FD, 0, SB, SC), -1.0}, {O(FD, 0, SB, SE), 1.0}};
    case GVT_MLPK:  // (I + P)(I - Q)(D x D)(I - Q)^T(I + P), ten terms
      return {{O(FD, 1, SA, SC), 1.0},  {O(FD, 1, SA, SE), 1.0},
              {O(FD, 1, SB, SC), 1.0},  {O(FD, 1, SB, SE), 1.0},
              {G(FD, FD, SA, SB, SC, SE), 2.0},  {G(FD, FD, SB, SA, SC, SE), 2.0},
              {G(FD, FD, SA, SA, SC, SE), -2.0}, {G(FD, FD, SA, SB, SC, SC), -2.0},
              {G(FD, FD, SB, SB, SC, SE), -2.0}, {G(FD, FD, SA, SB, SE, SE), -2.0}};
    default:
      throw Error{GVT_ERR_ARG, "unknown kind " + std::to_string(kind)};
  }
}

void counting_sort(const std::vector<int32_t> &key, int64_t nkeys, std::vector<int32_t> &perm,
                   std::vector<int64_t> &seg) {
  const int64_t n = (int64_t)key.size();
  seg.assign(nkeys + 1, 0);
  for (int64_t j = 0; j < n; ++j) seg[key[j] + 1]++;
  for (int64_t k = 0; k < nkeys; ++k) seg[k + 1] += seg[k];
  std::vector<int64_t> pos(seg.begin(), seg.end() - 1);
  perm.resize(n);
  for (int64_t j = 0; j < n; ++j) perm[pos[key[j]]++] = (int32_t)j;
}

int64_t count_unique(const std::vector<int32_t> &v, int64_t range) {
  std::vector<char> seen(range, 0);
  int64_t u = 0;
  for (int32_t x : v)
    if (!seen[x]) { seen[x] = 1; ++u; }
  return u;
}

// Stage-2 tuning targets (tuning.h): outputs per F1 row per tile that each
// RHS class aims for (a pass over a tile serves a fixed number of outputs per
// row, and every pass re-copies the tile's S rows).  Overridable for tuning
// sweeps.
double stage2_target(int cls) {
  const char *ev = std::getenv(cls ? "GVT_STAGE2_TARGET_R8" : "GVT_STAGE2_TARGET_R1");
  if (ev) {
    const double v = std::atof(ev);
    if (v > 0) return v;
  }
  return cls ? kStage2TargetR8 : kStage2TargetR1;
}

// Where the index work of a plan runs: on the device for large index sets,
// where sorting on the host costs more than the launches; GVT_PLAN_DEVICE=0/1
// forces either side.
constexpr int64_t kDevicePlanMinPairs = 1 << 16;
bool device_plan(int64_t n_in, int64_t n_out) {
  const char *ev = std::getenv("GVT_PLAN_DEVICE");
  if (ev && *ev) return std::atoi(ev) != 0;
  return n_in + n_out >= kDevicePlanMinPairs;
}

// Stage-2 tile classes a plan builds up front: those of the first RHS block
// of `rhs_hint` right-hand sides under the FP64 and the FP32 cap.
std::vector<int> hint_classes(const gvt_plan *P, int rhs_hint) {
  const int a = tile_class(rhs_block(rhs_hint, P->max_rhs[0]));
  const int b = tile_class(rhs_block(rhs_hint, P->max_rhs[1]));
  return a == b ? std::vector<int>{a} : std::vector<int>{a, b};
}

// Host tasks of a plan build: on their own threads for large inputs, inline
// for small ones (where starting a thread costs more than the task).
struct TaskGroup {
  bool par;
  std::vector<std::thread> th;
  explicit TaskGroup(bool parallel) : par(parallel) {}
  template <class F> void run(F f) {
    if (par) th.emplace_back(std::move(f));
    else f();
  }
  void join() {
    for (auto &t : th) t.join();
    th.clear();
  }
  ~TaskGroup() { join(); }
};

}  // namespace

int stage2_block_rows(const gvt_plan *P, const TermSpec &t, int cls) {
  const SBufSpec &sb = P->sbufs[t.sbuf];
  const double nsr = (double)std::max<size_t>(sb.rows.size(), 1);
  const double nx = (double)std::max<int64_t>(P->uniq[t.x], 1);
  const double rho = (double)P->n_out / (nx * nsr);  // outputs per (F1 row, S row)
  double rows = rho > 0 ? stage2_target(cls) / rho : kStage2MaxS;
  int ysz = (int)std::ceil(std::min<double>(std::max<double>(rows, 8.0), kStage2MaxS) / 8.0) * 8;
  return std::min(ysz, kStage2MaxS);
}

namespace {

// Stage-2 tiles of term `ts` for RHS class `cls`.
//  class 0 (1-2 RHS): groups of kStage2Rows consecutive F1 rows x blocks of
//    S rows staged in LDS; per output the compact S row.
//  class 1 (4-8 RHS): groups of kStage2Rows consecutive compact S rows x
//    blocks of F1 rows staged in LDS; per output the F1 row.
// The staged block is at most stage2_block_rows() rows high; more than four
// blocks are rounded up to a multiple of 8, so that an XCD can keep one slice
// of the staged matrix in its L2 (always in class 1; class 0 picks the order
// at launch, by F1 block or by S block; the padding blocks are empty tiles).
// One stable counting sort on (tile, group row) orders the outputs; the order
// inside a group row does not matter.
// With `up` the arrays join the plan's upload, else they are copied into the
// tile set's own allocation at once.
struct TileHost {
  int bsz = 0, nsb = 0;
  int64_t ntiles = 0;
  std::vector<int32_t> perm, stg, tstg, tmax;
  std::vector<int64_t> toff;
  std::vector<uint8_t> grow;
};

struct TileGeom {
  int bsz = 0;
  TileDims d{};
};

TileGeom tile_geom(const gvt_plan *P, const TermSpec &ts, int cls) {
  TileGeom g;
  const SBufSpec &sb = P->sbufs[ts.sbuf];
  g.bsz = stage2_block_rows(P, ts, cls);
  const int64_t nsr = std::max<int64_t>((int64_t)sb.rows.size(), 1);
  const int64_t nxr = std::max<int64_t>(rows_of(P, ts.fdot), 1);
  const int64_t ngrp_rows = cls ? nsr : nxr;   // grouped dimension
  const int64_t nstg_rows = cls ? nxr : nsr;   // staged dimension
  int64_t nsb = ceil_div(nstg_rows, (int64_t)g.bsz);
  if (nsb > 4) nsb = 8 * ceil_div(nsb, (int64_t)8);
  g.d.nsb = nsb;
  g.d.sbs = ceil_div(nstg_rows, nsb);
  g.d.ntiles = ceil_div(ngrp_rows, kStage2Rows) * nsb;
  g.d.nstg_rows = nstg_rows;
  g.d.rows_per_tile = kStage2Rows;
  g.d.swap = cls != 0;
  GVT_REQUIRE(g.d.ntiles * kStage2Rows < INT32_MAX, GVT_ERR_ARG, "too many stage-2 tiles");
  return g;
}

TileHost compute_tiles(const gvt_plan *P, const TermSpec &ts, int cls) {
  TileHost o;
  const SBufSpec &sb = P->sbufs[ts.sbuf];
  const std::vector<int32_t> &hx = P->h_out[ts.x == SA ? 0 : 1];
  const std::vector<int32_t> &hy = P->h_out[ts.y == SA ? 0 : 1];
  const int64_t n_out = P->n_out;
  const TileGeom g = tile_geom(P, ts, cls);
  const int64_t nsb = g.d.nsb, sbs = g.d.sbs, ntiles = g.d.ntiles, nstg_rows = g.d.nstg_rows;
  std::vector<int32_t> stg_of(n_out), tkey(n_out);
  for (int64_t i = 0; i < n_out; ++i) {
    const int32_t yr = sb.rowmap[hy[i]], xv = hx[i];
    const int32_t grp = cls ? yr : xv;
    stg_of[i] = cls ? xv : yr;
    const int64_t tile_id = (grp / kStage2Rows) * nsb + stg_of[i] / sbs;
    tkey[i] = (int32_t)(tile_id * kStage2Rows + grp % kStage2Rows);
  }
  std::vector<int64_t> sgk;
  counting_sort(tkey, ntiles * kStage2Rows, o.perm, sgk);
  o.stg.resize(n_out);
  for (int64_t q = 0; q < n_out; ++q) o.stg[q] = stg_of[o.perm[q]];
  o.toff.resize((size_t)ntiles * (kStage2Rows + 1));
  o.tstg.resize((size_t)2 * ntiles);
  o.tmax.assign(ntiles, 0);
  o.grow.resize((size_t)ntiles * kStage2Rows);
  for (int64_t tt = 0; tt < ntiles; ++tt) {
    const int64_t sbk = tt % nsb;
    o.tstg[2 * tt] = (int32_t)std::min<int64_t>(sbk * sbs, nstg_rows);
    o.tstg[2 * tt + 1] = (int32_t)std::max<int64_t>(0, std::min<int64_t>(sbs, nstg_rows - sbk * sbs));
    for (int g2 = 0; g2 <= kStage2Rows; ++g2)
      o.toff[(size_t)tt * (kStage2Rows + 1) + g2] = sgk[(size_t)tt * kStage2Rows + g2];
    int64_t c[kStage2Rows];
    for (int g2 = 0; g2 < kStage2Rows; ++g2) {
      c[g2] = sgk[(size_t)tt * kStage2Rows + g2 + 1] - sgk[(size_t)tt * kStage2Rows + g2];
      o.tmax[tt] = std::max<int32_t>(o.tmax[tt], (int32_t)c[g2]);
    }
    // group order: rows by descending output count, ties by row
    for (int g2 = 0; g2 < kStage2Rows; ++g2) {
      int rank = 0;
      for (int h = 0; h < kStage2Rows; ++h) rank += c[h] > c[g2] || (c[h] == c[g2] && h < g2);
      o.grow[(size_t)tt * kStage2Rows + rank] = (uint8_t)g2;
    }
  }
  o.bsz = g.bsz;
  o.ntiles = ntiles;
  o.nsb = (int)nsb;
  return o;
}

// Device arrays of known sizes laid out in one allocation.
struct DevLayout {
  std::vector<std::pair<DevMem *, size_t>> items;
  void add(DevMem &m, size_t bytes) { items.push_back({&m, bytes}); }
  void commit(DevMem &blob) {
    size_t total = 0;
    for (auto &it : items) total += (it.second + 255) & ~size_t(255);
    blob.ensure(total ? total : 256);
    size_t off = 0;
    for (auto &it : items) {
      it.first->view(static_cast<char *>(blob.p) + off, it.second);
      off += (it.second + 255) & ~size_t(255);
    }
    items.clear();
  }
};

// Device-built tiles: the arrays' sizes, then the kernels that fill them.
void dev_tiles_layout(TileSet &tl, const TileGeom &g, int64_t n_out, DevLayout &L) {
  tl.ysz = g.bsz;
  tl.ntiles = g.d.ntiles;
  tl.nyb = (int)g.d.nsb;
  L.add(tl.perm, (size_t)n_out * 4);
  L.add(tl.yrows, (size_t)n_out * 4);
  L.add(tl.tileoff, (size_t)g.d.ntiles * (kStage2Rows + 1) * 8);
  L.add(tl.tiley, (size_t)g.d.ntiles * 2 * 4);
  L.add(tl.tilemax, (size_t)g.d.ntiles * 4);
  L.add(tl.grow, (size_t)g.d.ntiles * kStage2Rows);
}

void dev_tiles_fill(gvt_plan *P, const TermSpec &ts, TileSet &tl, const TileGeom &g, hipStream_t s) {
  const SBufSpec &sb = P->sbufs[ts.sbuf];
  dev_tiles(P->idx[ts.x].as<int32_t>(), P->idx[ts.y].as<int32_t>(), sb.d_rowmap.as<int32_t>(),
            P->n_out, g.d, tl.perm.as<int32_t>(), tl.yrows.as<int32_t>(), tl.tileoff.as<int64_t>(),
            tl.tiley.as<int32_t>(), tl.tilemax.as<int32_t>(), tl.grow.as<uint8_t>(), P->scratch, s);
  tl.built = true;
}

// With `up` the arrays join the plan's upload, else they are copied into the
// tile set's own allocation at once.
void install_tiles(TileSet &tl, TileHost &&o, Uploads *up) {
  tl.ysz = o.bsz;
  tl.ntiles = o.ntiles;
  tl.nyb = o.nsb;
  Uploads local;
  Uploads &u = up ? *up : local;
  u.add(tl.perm, std::move(o.perm));
  u.add(tl.yrows, std::move(o.stg));
  u.add(tl.tileoff, std::move(o.toff));
  u.add(tl.tiley, std::move(o.tstg));
  u.add(tl.tilemax, std::move(o.tmax));
  u.add(tl.grow, std::move(o.grow));
  if (!up) local.commit(tl.blob);
  tl.built = true;
}

}  // namespace

void plan_ensure_tiles(gvt_plan *P, int cls, hipStream_t s) {
  bool need = false;
  for (const TermSpec &t : P->terms) need = need || (t.type == TG && !t.tiles[cls].built);
  if (!need || P->n_out == 0) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    throw Error{GVT_ERR_ARG,
                "the first product with a new RHS block size builds stage-2 tiles and cannot be "
                "captured; run it once before capturing"};
  for (TermSpec &t : P->terms) {
    if (t.type != TG || t.tiles[cls].built) continue;
    if (P->on_device) {
      TileSet &tl = t.tiles[cls];
      const TileGeom g = tile_geom(P, t, cls);
      DevLayout L;
      dev_tiles_layout(tl, g, P->n_out, L);
      L.commit(tl.blob);
      dev_tiles_fill(P, t, tl, g, s);
    } else {
      install_tiles(t.tiles[cls], compute_tiles(P, t, cls), nullptr);
    }
  }
}

void plan_build(gvt_plan *P, const int *kinds, int nkinds, int64_t d_rows, int64_t d_cols,
                int64_t t_rows, int64_t t_cols, const int32_t *a, const int32_t *b, int64_t n_out,
                const int32_t *c, const int32_t *e, int64_t n_in, int flags, hipStream_t s,
                int rhs_hint) {
  GVT_REQUIRE(kinds && nkinds >= 1, GVT_ERR_ARG, "kinds must be a non-empty host array");
  GVT_REQUIRE(nkinds <= kMaxCombineOut, GVT_ERR_ARG, "at most 8 kinds per plan");
  GVT_REQUIRE(d_rows >= 0 && d_cols >= 0 && t_rows >= 0 && t_cols >= 0 && n_out >= 0 && n_in >= 0,
              GVT_ERR_ARG, "negative size");
  GVT_REQUIRE(n_out <= INT32_MAX && n_in <= INT32_MAX, GVT_ERR_ARG, "too many pairs for int32 positions");
  GVT_REQUIRE((n_out == 0 || (a && b)) && (n_in == 0 || (c && e)), GVT_ERR_ARG, "null index array");
  GVT_REQUIRE(!((flags & GVT_FLAG_ORDER_A) && (flags & GVT_FLAG_ORDER_B)), GVT_ERR_ARG,
              "ORDER_A and ORDER_B are exclusive");
  refresh_launch_knobs();
  {
    const char *both = std::getenv("GVT_MAX_RHS_BLOCK");
    const char *ev[2] = {std::getenv("GVT_MAX_RHS_BLOCK_F64"), std::getenv("GVT_MAX_RHS_BLOCK_F32")};
    const int tuned[2] = {kMaxRhsBlockF64, kMaxRhsBlockF32};
    for (int k = 0; k < 2; ++k) {
      const int mr = ev[k] && *ev[k] ? std::atoi(ev[k]) : both && *both ? std::atoi(both) : tuned[k];
      P->max_rhs[k] = (mr == 1 || mr == 2 || mr == 4 || mr == 8) ? mr : 8;
    }
  }
  P->kinds.assign(kinds, kinds + nkinds);
  P->flags = flags;
  bool hom = false;
  for (int k : P->kinds) {
    GVT_REQUIRE(k >= GVT_KRONECKER && k <= GVT_MLPK, GVT_ERR_ARG, "unknown kind");
    hom = hom || kind_homogeneous(k);
  }
  if (hom) {
    GVT_REQUIRE(t_rows == d_rows && t_cols == d_cols, GVT_ERR_KIND,
                "homogeneous kinds need T with the shape of D (T is taken to be D)");
  }
  if (flags & GVT_FLAG_SYMMETRIC_BASES) {
    GVT_REQUIRE(d_rows == d_cols && t_rows == t_cols, GVT_ERR_KIND,
                "GVT_FLAG_SYMMETRIC_BASES needs square base matrices");
  }
  P->homogeneous = hom;
  P->d_rows = d_rows; P->d_cols = d_cols; P->t_rows = t_rows; P->t_cols = t_cols;
  P->n_out = n_out; P->n_in = n_in;
  P->last_stream = s;

  PhaseTimer tm;
  const bool alias = n_out == n_in && a == c && b == e;
  const int64_t cnt[4] = {n_out, n_out, n_in, n_in};
  const int64_t lim[4] = {d_rows, t_rows, d_cols, t_cols};
  static const char *nm[4] = {"out_a", "out_b", "in_c", "in_e"};
  // first index outside [0, lim) per array (-1: none), then the error naming
  // the array and limit the value violates (aliased arrays carry two limits)
  int64_t bad[4] = {-1, -1, -1, -1};
  auto report_bad = [&](int i, int32_t v) {
    int which = i;
    if (alias && (v < 0 || v >= lim[i + 2]) && !(v < 0 || v >= lim[i])) which = i + 2;
    throw Error{GVT_ERR_INDEX, std::string(nm[which]) + "[" + std::to_string(bad[i]) + "] = " +
                                   std::to_string(v) + " outside [0, " + std::to_string(lim[which]) +
                                   ")"};
  };
  const bool dense_candidate = nkinds == 1 && P->kinds[0] == GVT_KRONECKER && n_in == d_cols * t_cols &&
                               n_out == d_rows * t_rows && n_in > 0 && n_out > 0;
  P->on_device = device_plan(n_in, n_out);
  std::vector<int32_t> h[4];
  std::vector<uint8_t> seen_dev[4];  // device-built plans: which values occur, per array
  if (P->on_device) {
    // ---- the plan's own device copies of the indices, validation and unique
    // marks by one kernel; the only host synchronisation of the build -------
    const int narr = alias ? 2 : 4;
    const int32_t *src[4] = {a, b, c, e};
    DevLayout L;
    for (int i = 0; i < narr; ++i) L.add(P->idx[i], (size_t)cnt[i] * 4);
    L.commit(P->idxblob);
    for (int i = 0; i < narr; ++i)
      if (cnt[i])
        GVT_HIP_CHECK(hipMemcpyAsync(P->idx[i].p, src[i], cnt[i] * 4, hipMemcpyDeviceToDevice, s));
    if (alias) {
      P->idx[2].view(P->idx[0].p, P->idx[0].bytes);
      P->idx[3].view(P->idx[1].p, P->idx[1].bytes);
    }
    const int32_t *x[4];
    int64_t L2[4], range[4];
    for (int i = 0; i < narr; ++i) {
      x[i] = P->idx[i].as<int32_t>();
      L2[i] = alias ? std::min(lim[i], lim[i + 2]) : lim[i];
      range[i] = alias ? std::max(lim[i], lim[i + 2]) : lim[i];
    }
    ProbeResult pr;
    dev_probe(x, cnt, L2, range, narr, dense_candidate ? t_rows : 0, dense_candidate ? t_cols : 0,
              P->scratch, pr, s);
    tm.lap("indices: device probe");
    for (int i = 0; i < narr; ++i) {
      if (pr.bad[i] < 0) continue;
      bad[i] = pr.bad[i];
      int32_t v = 0;
      GVT_HIP_CHECK(hipMemcpy(&v, x[i] + bad[i], 4, hipMemcpyDeviceToHost));
      report_bad(i, v);
    }
    for (int i = 0; i < narr; ++i) {
      int64_t u = 0;
      for (uint8_t f : pr.seen[i]) u += f;
      P->uniq[i] = u;
      seen_dev[i] = std::move(pr.seen[i]);
    }
    if (alias) {
      P->uniq[2] = P->uniq[0];
      P->uniq[3] = P->uniq[1];
    }
    P->dense = dense_candidate && pr.nat;
  } else {
    // ---- indices to host, validation, unique counts (Table 1) -------------
    // When the output pairs are the input pairs (training products), the two
    // index arrays are copied and checked once.
    const int32_t *src[4] = {a, b, c, e};
    for (int i = 0; i < (alias ? 2 : 4); ++i) {
      h[i].resize(cnt[i]);
      if (cnt[i])
        GVT_HIP_CHECK(hipMemcpyAsync(h[i].data(), src[i], cnt[i] * sizeof(int32_t),
                                     hipMemcpyDeviceToHost, s));
    }
    GVT_HIP_CHECK(hipStreamSynchronize(s));
    tm.lap("indices to host");
    auto check = [&](int i) {
      const int i2 = alias ? i + 2 : -1;  // the aliased input array, with its own limit
      const int64_t Lm = i2 >= 0 ? std::min(lim[i], lim[i2]) : lim[i];
      const std::vector<int32_t> &v = h[i];
      for (int64_t j = 0; j < (int64_t)v.size(); ++j)
        if (v[j] < 0 || v[j] >= Lm) { bad[i] = j; return; }
      P->uniq[i] = count_unique(v, Lm > 0 ? std::max(lim[i], i2 >= 0 ? lim[i2] : 0) : 0);
    };
    {
      TaskGroup tg(n_in + n_out >= (1 << 16));
      const int na = alias ? 2 : 4;
      for (int i = 1; i < na; ++i) tg.run([&, i]() { check(i); });
      check(0);
      tg.join();
    }
    for (int i = 0; i < (alias ? 2 : 4); ++i)
      if (bad[i] >= 0) report_bad(i, h[i][bad[i]]);
    if (alias) {
      h[2] = h[0];
      h[3] = h[1];
      P->uniq[2] = P->uniq[0];
      P->uniq[3] = P->uniq[1];
    }
    // complete data: both pair sets are the full grid in natural order
    if (dense_candidate) {
      bool nat = true;
      for (int64_t j = 0; j < n_in && nat; ++j)
        nat = h[2][j] == (int32_t)(j / t_cols) && h[3][j] == (int32_t)(j % t_cols);
      for (int64_t i = 0; i < n_out && nat; ++i)
        nat = h[0][i] == (int32_t)(i / t_rows) && h[1][i] == (int32_t)(i % t_rows);
      P->dense = nat;
    }
  }
  tm.lap("validate + unique");
  Uploads up;
  if (!P->on_device) {
    P->h_out[0] = h[0];
    P->h_out[1] = h[1];
  }

  if (P->dense) {
    P->outputs.assign(1, {});
    P->cost_fma = (double)d_rows * d_cols * t_cols + (double)d_rows * t_cols * t_rows;
    return;
  }

  // ---- term expansion, stage-order choice, common subexpressions ----------
  const double n_in_d = (double)n_in, n_out_d = (double)n_out;
  auto selval_uniq = [&](int sel) { return (double)P->uniq[sel]; };
  std::map<std::tuple<int, int, int>, int> sbuf_index;  // (fsc, key, other) -> sbuf
  std::map<RawTerm, int> term_index;
  std::map<std::tuple<int, int, int>, int> gemv_index;
  std::vector<RawTerm> raw_terms;

  auto g_cost = [&](const RawTerm &t) {
    const int y = t.a3, key = t.a4, other = t.a5;
    const double s1 = (key == other) ? selval_uniq(y) * (double)nkeys_of(P, key)
                                     : selval_uniq(y) * n_in_d;
    return s1 + n_out_d * (double)nkeys_of(P, key);
  };
  const int prefer_key = (flags & GVT_FLAG_ORDER_A) ? SC
                         : (flags & GVT_FLAG_ORDER_B) ? SE
                         : (d_cols >= t_cols ? SC : SE);
  const bool forced = (flags & (GVT_FLAG_ORDER_A | GVT_FLAG_ORDER_B)) != 0;

  auto canon_g = [&](RawTerm t) {
    // the same term with the two Kronecker factors exchanged (Lemma: P(D x T)P^T = T x D)
    RawTerm sw = G(t.a1, t.a0, t.a3, t.a2, t.a5, t.a4);
    if (forced) {
      if (t.a4 == prefer_key) return t;
      if (sw.a4 == prefer_key) return sw;
      return t;
    }
    double c1 = g_cost(t), c2 = g_cost(sw);
    if (c1 < c2) return t;
    if (c2 < c1) return sw;
    const bool has1 = sbuf_index.count({t.a1, t.a4, t.a5}) > 0;
    const bool has2 = sbuf_index.count({sw.a1, sw.a4, sw.a5}) > 0;
    if (has1 != has2) return has1 ? t : sw;
    if (t.a4 == prefer_key) return t;
    if (sw.a4 == prefer_key) return sw;
    return t;
  };

  P->outputs.assign(nkinds, {});
  for (int kk = 0; kk < nkinds; ++kk) {
    for (auto &tc : expand_kind(P->kinds[kk], hom)) {
      RawTerm t = tc.first;
      if (t.type == TG) {
        t = canon_g(t);
        sbuf_index.emplace(std::make_tuple(t.a1, t.a4, t.a5), (int)sbuf_index.size());
      }
      auto it = term_index.find(t);
      int id;
      if (it == term_index.end()) {
        id = (int)raw_terms.size();
        term_index.emplace(t, id);
        raw_terms.push_back(t);
      } else {
        id = it->second;
      }
      // merge repeated terms within a kind
      bool merged = false;
      for (auto &oc : P->outputs[kk])
        if (oc.first == id) { oc.second += tc.second; merged = true; }
      if (!merged) P->outputs[kk].push_back({id, tc.second});
    }
  }

  // ---- materialise sorts, S buffers, gemvs and terms ----------------------
  auto sel_host = [&](int sel) -> const std::vector<int32_t> & { return h[sel]; };
  auto sel_dev = [&](int sel) -> const int32_t * { return P->idx[sel].as<int32_t>(); };
  bool insort_needed[2] = {false, false};
  bool outord_needed[2] = {false, false};  // outputs grouped by a / by b (match terms)
  auto need_insort = [&](int key) { insort_needed[key == SC ? 0 : 1] = true; };
  // sort by other index first, then stably by key: segments ordered by other inside
  struct SortHost {
    std::vector<int32_t> perm, inv, other;
    std::vector<int64_t> seg;
  } sort_host[2];
  auto build_insort = [&](int ks) {
    const int key = ks == 0 ? SC : SE, okey = ks == 0 ? SE : SC;
    SortHost &o = sort_host[ks];
    std::vector<int32_t> perm_o;
    std::vector<int64_t> seg_o;
    counting_sort(h[okey], nkeys_of(P, okey), perm_o, seg_o);
    std::vector<int32_t> key_o(n_in);
    for (int64_t p = 0; p < n_in; ++p) key_o[p] = h[key][perm_o[p]];
    counting_sort(key_o, nkeys_of(P, key), o.perm, o.seg);
    for (int64_t p = 0; p < n_in; ++p) o.perm[p] = perm_o[o.perm[p]];
    o.inv.resize(n_in);
    for (int64_t p = 0; p < n_in; ++p) o.inv[o.perm[p]] = (int32_t)p;
    o.other.resize(n_in);
    for (int64_t p = 0; p < n_in; ++p) o.other[p] = h[okey][o.perm[p]];
  };

  tm.lap("term expansion");
  // S buffers in creation order
  P->sbufs.resize(sbuf_index.size());
  for (auto &kv : sbuf_index) {
    SBufSpec &sb = P->sbufs[kv.second];
    std::tie(sb.fsc, sb.key, sb.other) = kv.first;
    sb.degenerate = sb.key == sb.other;
    sb.rowmap.assign(rows_of(P, sb.fsc), -1);
  }
  // rows needed per S buffer
  for (const RawTerm &t : raw_terms) {
    if (t.type != TG) continue;
    SBufSpec &sb = P->sbufs[sbuf_index.at({t.a1, t.a4, t.a5})];
    if (P->on_device) {
      const std::vector<uint8_t> &seen = seen_dev[alias && t.a3 >= 2 ? t.a3 - 2 : t.a3];
      const size_t nr = std::min(seen.size(), sb.rowmap.size());
      for (size_t v = 0; v < nr; ++v)
        if (seen[v]) sb.rowmap[v] = 0;
    } else {
      for (int32_t v : sel_host(t.a3)) sb.rowmap[v] = 0;
    }
  }
  for (SBufSpec &sb : P->sbufs) {
    // a nearly contiguous row set (at most 1/8 of its span missing) is widened
    // to the whole span, so that stage 1 can walk it several rows per lane;
    // the added rows are computed and never read
    sb.nneed = 0;
    for (int32_t m : sb.rowmap) sb.nneed += m >= 0;
    if (!sb.degenerate && stage1_wide_enabled()) {
      int64_t lo = -1, hi = -1, cnt = 0;
      for (int64_t r = 0; r < (int64_t)sb.rowmap.size(); ++r)
        if (sb.rowmap[r] >= 0) { lo = lo < 0 ? r : lo; hi = r; ++cnt; }
      if (cnt > 0 && (hi - lo + 1 - cnt) * 8 <= hi - lo + 1)
        for (int64_t r = lo; r <= hi; ++r) sb.rowmap[r] = 0;
    }
    sb.rows.clear();
    for (int64_t r = 0; r < (int64_t)sb.rowmap.size(); ++r)
      if (sb.rowmap[r] >= 0) { sb.rowmap[r] = (int32_t)sb.rows.size(); sb.rows.push_back((int32_t)r); }
    sb.row0 = !sb.rows.empty() && sb.rows.back() - sb.rows.front() + 1 == (int64_t)sb.rows.size()
                  ? sb.rows.front() : -1;
    up.add(sb.d_rows, sb.rows);
    if (P->on_device) up.add(sb.d_rowmap, sb.rowmap);
    need_insort(sb.key);  // scatter segments, or the segment sums of a degenerate buffer
  }
  tm.lap("S rows");
  P->terms.resize(raw_terms.size());
  P->cost_fma = 0.0;
  for (size_t ti = 0; ti < raw_terms.size(); ++ti) {
    const RawTerm &t = raw_terms[ti];
    TermSpec &ts = P->terms[ti];
    ts.type = t.type;
    if (t.type == TG) {
      ts.fdot = t.a0; ts.x = t.a2; ts.y = t.a3;
      ts.sbuf = sbuf_index.at({t.a1, t.a4, t.a5});
      P->cost_fma += g_cost(t);
    } else if (t.type == TO) {
      auto gk = std::make_tuple(t.a0, t.a1, t.a3);
      auto it = gemv_index.find(gk);
      if (it == gemv_index.end()) {
        it = gemv_index.emplace(gk, (int)P->gemvs.size()).first;
        P->gemvs.push_back(GemvSpec{t.a0, t.a1, t.a3});
        need_insort(t.a3);
        P->cost_fma += (double)rows_of(P, t.a0) * (double)nkeys_of(P, t.a3) + n_in_d;
      }
      ts.gemv = it->second;
      ts.f = t.a0; ts.x = t.a2;
    } else {
      ts.f = t.a0; ts.x = t.a1; ts.outkey = t.a2; ts.key = t.a3;
      need_insort(ts.key);
      outord_needed[ts.x == SA ? 0 : 1] = true;
      P->cost_fma += n_out_d * (n_in_d / std::max<double>(1.0, (double)nkeys_of(P, ts.key)));
    }
  }
  // two-factor terms as dense-tile groups (gvt_plan::tgroups): a term keyed
  // (e, c) is the same operator with F_A, F_B and the gather indices swapped
  {
    bool ok = true;
    std::vector<TileGroup> groups;
    for (size_t ti = 0; ti < P->terms.size() && ok; ++ti) {
      const TermSpec &ts = P->terms[ti];
      if (ts.type != TG) continue;
      const SBufSpec &sb = P->sbufs[ts.sbuf];
      int fa, fb, pp, qq;
      if (sb.key == SC && sb.other == SE) {
        fa = ts.fdot; fb = sb.fsc; pp = ts.x; qq = ts.y;
      } else if (sb.key == SE && sb.other == SC) {
        fa = sb.fsc; fb = ts.fdot; pp = ts.y; qq = ts.x;
      } else {
        ok = false;
        break;
      }
      ok = cols_of(P, fa) == nkeys_of(P, SC) && cols_of(P, fb) == nkeys_of(P, SE);
      size_t g = 0;
      while (g < groups.size() && !(groups[g].fa == fa && groups[g].fb == fb)) ++g;
      if (g == groups.size()) groups.push_back(TileGroup{fa, fb, {}});
      groups[g].terms.push_back(TileTerm{(int)ti, pp, qq});
    }
    if (ok && n_in > 0 && n_out > 0) P->tgroups = std::move(groups);
  }
  // S-buffer stage-1 cost (shared scatters counted once)
  for (const SBufSpec &sb : P->sbufs)
    P->cost_fma += sb.degenerate ? (double)sb.nneed * nkeys_of(P, sb.key) : (double)sb.nneed * n_in_d;
  // stage-2 costs were included in g_cost together with a per-term stage-1; remove those
  for (const RawTerm &t : raw_terms)
    if (t.type == TG) {
      const int y = t.a3, key = t.a4, other = t.a5;
      P->cost_fma -= (key == other) ? selval_uniq(y) * (double)nkeys_of(P, key)
                                    : selval_uniq(y) * n_in_d;
    }
  if (P->on_device) {
    // ---- sorts and tile orders on the device: sizes first (one allocation),
    // then the small host arrays, then the kernels, all queued on s --------
    const std::vector<int> hcls = hint_classes(P, rhs_hint);
    DevLayout L;
    for (int ks = 0; ks < 2; ++ks) {
      if (!insort_needed[ks]) continue;
      InputSort &is = P->insort[ks];
      is.nkeys = nkeys_of(P, ks == 0 ? SC : SE);
      is.nother = nkeys_of(P, ks == 0 ? SE : SC);
      L.add(is.perm, (size_t)n_in * 4);
      L.add(is.inv, (size_t)n_in * 4);
      L.add(is.other, (size_t)n_in * 4);
      L.add(is.seg, (size_t)(is.nkeys + 1) * 8);
    }
    for (int xs = 0; xs < 2; ++xs) {
      if (!outord_needed[xs] || n_out == 0) continue;
      OutOrder &oo = P->outord[xs];
      oo.nrows = xs == 0 ? d_rows : t_rows;
      L.add(oo.perm, (size_t)n_out * 4);
      L.add(oo.off, (size_t)(oo.nrows + 1) * 8);
    }
    struct DevTiles {
      TermSpec *ts;
      int cls;
      TileGeom g;
    };
    std::vector<DevTiles> tiles;
    for (TermSpec &ts : P->terms)
      if (ts.type == TG && n_out > 0)
        for (int cls : hcls) {
          tiles.push_back({&ts, cls, tile_geom(P, ts, cls)});
          dev_tiles_layout(ts.tiles[cls], tiles.back().g, n_out, L);
        }
    size_t sneed = 0;
    for (int ks = 0; ks < 2; ++ks)
      if (insort_needed[ks])
        sneed = std::max(sneed, dev_input_sort_bytes(P->insort[ks].nkeys, P->insort[ks].nother, n_in));
    for (int xs = 0; xs < 2; ++xs)
      if (outord_needed[xs] && n_out > 0) sneed = std::max(sneed, dev_group_rows_bytes(n_out));
    for (auto &tk : tiles)
      sneed = std::max(sneed, dev_tiles_bytes(n_out, tk.g.d.ntiles * tk.g.d.rows_per_tile));
    dev_reserve(P->scratch, sneed, s);
    L.commit(P->devblob);
    up.commit(P->blob);
    for (int ks = 0; ks < 2; ++ks) {
      if (!insort_needed[ks]) continue;
      InputSort &is = P->insort[ks];
      const int key = ks == 0 ? SC : SE, okey = ks == 0 ? SE : SC;
      dev_input_sort(P->idx[key].as<int32_t>(), is.nkeys, P->idx[okey].as<int32_t>(), is.nother, n_in,
                     is.perm.as<int32_t>(), is.other.as<int32_t>(), is.seg.as<int64_t>(),
                     P->scratch, s);
      dev_invert(is.perm.as<int32_t>(), n_in, is.inv.as<int32_t>(), s);
      is.built = true;
    }
    for (int xs = 0; xs < 2; ++xs) {
      if (!outord_needed[xs] || n_out == 0) continue;
      OutOrder &oo = P->outord[xs];
      dev_group_rows(P->idx[xs == 0 ? SA : SB].as<int32_t>(), oo.nrows, n_out, oo.perm.as<int32_t>(),
                     oo.off.as<int64_t>(), P->scratch, s);
      oo.built = true;
    }
    for (auto &tk : tiles) dev_tiles_fill(P, *tk.ts, tk.ts->tiles[tk.cls], tk.g, s);
    tm.lap("device sorts queued");
  } else {
    // input sorts and stage-2 tiles are independent host work: one thread each
    {
      struct HostTiles {
        TermSpec *ts;
        int cls;
        TileHost t;
      };
      std::vector<HostTiles> tiles;
      for (TermSpec &ts : P->terms)
        if (ts.type == TG && n_out > 0)
          for (int cls : hint_classes(P, rhs_hint)) tiles.push_back({&ts, cls, TileHost{}});
      TaskGroup tg(n_in + n_out >= (1 << 16));
      std::vector<std::exception_ptr> errs(tiles.size() + 2);
      auto guard = [&](size_t slot, auto fn) {
        try {
          fn();
        } catch (...) {
          errs[slot] = std::current_exception();
        }
      };
      for (int ks = 0; ks < 2; ++ks)
        if (insort_needed[ks] && n_in > 0)
          tg.run([&, ks]() { guard(ks, [&]() { build_insort(ks); }); });
      std::vector<int32_t> oo_perm[2];
      std::vector<int64_t> oo_off[2];
      for (int xs = 0; xs < 2; ++xs)
        if (outord_needed[xs] && n_out > 0)
          tg.run([&, xs]() {
            counting_sort(h[xs == 0 ? SA : SB], xs == 0 ? d_rows : t_rows, oo_perm[xs], oo_off[xs]);
          });
      for (size_t k = 0; k < tiles.size(); ++k)
        tg.run([&, k]() {
          guard(2 + k, [&]() { tiles[k].t = compute_tiles(P, *tiles[k].ts, tiles[k].cls); });
        });
      tg.join();
      for (auto &ep : errs)
        if (ep) std::rethrow_exception(ep);
      for (int ks = 0; ks < 2; ++ks) {
        if (!insort_needed[ks]) continue;
        InputSort &is = P->insort[ks];
        is.nkeys = nkeys_of(P, ks == 0 ? SC : SE);
        is.nother = nkeys_of(P, ks == 0 ? SE : SC);
        if (n_in > 0) {
          up.add(is.perm, std::move(sort_host[ks].perm));
          up.add(is.inv, std::move(sort_host[ks].inv));
          up.add(is.other, std::move(sort_host[ks].other));
          up.add(is.seg, std::move(sort_host[ks].seg));
        } else {
          up.add(is.seg, std::vector<int64_t>(is.nkeys + 1, 0));
        }
        is.built = true;
      }
      for (auto &tk : tiles) install_tiles(tk.ts->tiles[tk.cls], std::move(tk.t), &up);
      for (int xs = 0; xs < 2; ++xs) {
        if (!outord_needed[xs] || n_out == 0) continue;
        OutOrder &oo = P->outord[xs];
        oo.nrows = xs == 0 ? d_rows : t_rows;
        up.add(oo.perm, std::move(oo_perm[xs]));
        up.add(oo.off, std::move(oo_off[xs]));
        oo.built = true;
      }
    }
    tm.lap("input sorts + term orderings");
    bool need_idx = nkinds == 1 && kinds[0] == GVT_KRONECKER;  // dense tiles gather by (a, b)
    for (const TermSpec &t : P->terms) need_idx = need_idx || t.type != TG;
    need_idx = need_idx || !P->tgroups.empty();  // multi-term dense tiles gather by (a, b)
    if (need_idx)
      for (int i = 0; i < 4; ++i) up.add(P->idx[i], h[i]);
    up.commit(P->blob);
    tm.lap("upload");
  }
  P->direct = nkinds == 1 && P->outputs[0].size() == 1 && P->outputs[0][0].second == 1.0 &&
              P->terms[P->outputs[0][0].first].type == TG;
  P->gtiles_ok = !P->direct && !P->tgroups.empty();
  {
    const TermSpec &t0 = P->terms[P->outputs[0][0].first];
    P->tiles_ok = P->direct && kinds[0] == GVT_KRONECKER && n_in > 0 && n_out > 0 && t0.sbuf >= 0 &&
                  !P->sbufs[t0.sbuf].degenerate;
    P->tiles_mode = (flags & GVT_FLAG_DENSE_TILES) ? 1 : (flags & GVT_FLAG_NO_DENSE_TILES) ? -1 : 0;
    if (const char *ev = std::getenv("GVT_DENSE_TILES")) P->tiles_mode = std::atoi(ev) != 0 ? 1 : -1;
  }
  for (auto &o : P->outputs)
    GVT_REQUIRE(o.size() <= (size_t)kMaxCombineTerms, GVT_ERR_ARG, "too many terms");
  GVT_REQUIRE(P->terms.size() <= (size_t)kMaxCombineTerms, GVT_ERR_ARG,
              "the kinds of one plan may use at most 16 distinct terms");
  (void)sel_dev;
}

// ---------------------------------------------------------------------------
namespace {

template <class T> int prec_slot() { return sizeof(T) == 8 ? 0 : 1; }

// Row stride of a stage-1 buffer in elements: keys x RHS padded to whole
// 1 KB chunks (stage 2 copies rows chunk by chunk).  The padding is zero.
template <class T> int64_t sbuf_ld(const gvt_plan *P, int i, int R) {
  return sbuf_row_ld<T>(nkeys_of(P, P->sbufs[i].key), R);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <class T> void layout_workspace(gvt_plan *P, int R) {
  Workspace &W = P->ws[prec_slot<T>()];
  if (W.R == R && W.need) return;
  size_t off = 0;
  auto take = [&](size_t elems) {
    const size_t o = off;
    off = align256(off + elems * sizeof(T));
    return (int64_t)o;
  };
  W.vs = {-1, -1};
  W.sv = {-1, -1};
  W.trans = {-1, -1};
  for (int k = 0; k < 2; ++k)
    if (P->insort[k].built) {
      W.vs[k] = take((size_t)P->n_in * R);
      W.sv[k] = take((size_t)P->insort[k].nkeys * R);
    }
  if (!(P->flags & GVT_FLAG_SYMMETRIC_BASES)) {
    for (const SBufSpec &sb : P->sbufs)
      if (!sb.degenerate && W.trans[sb.fsc] < 0)
        W.trans[sb.fsc] = take((size_t)rows_of(P, sb.fsc) * cols_of(P, sb.fsc));
  }
  W.sbuf.assign(P->sbufs.size(), -1);
  for (size_t i = 0; i < P->sbufs.size(); ++i)
    W.sbuf[i] = take(P->sbufs[i].rows.size() * (size_t)sbuf_ld<T>(P, (int)i, R));
  W.gemv.assign(P->gemvs.size(), -1);
  for (size_t i = 0; i < P->gemvs.size(); ++i) W.gemv[i] = take((size_t)rows_of(P, P->gemvs[i].f) * R);
  W.tvec.assign(P->terms.size(), -1);
  if (!P->direct)
    for (size_t i = 0; i < P->terms.size(); ++i) W.tvec[i] = take((size_t)P->n_out * R);
  W.need = off;
  W.R = R;
  W.pool.ensure(off);
}

template <class T> T *wsp(gvt_plan *P, int64_t off) {
  return off < 0 ? nullptr
                 : reinterpret_cast<T *>(static_cast<char *>(P->ws[prec_slot<T>()].pool.p) + off);
}

inline void mark(gvt_plan *P, int stage, int edge, hipStream_t s) {
  if (P->prof) GVT_HIP_CHECK(hipEventRecord(P->prof[stage * 2 + edge], s));
}

}  // namespace
template <class T>
void execute_gtiles(gvt_plan *P, int gprec, const T *const *F, const int64_t *ldF, const T *V, int R,
                    int64_t ldv, T *const *tvec, hipStream_t s);
namespace {

// One block of R RHS through the term program.  gprec != 0: the two-factor
// terms go through dense tiles in that precision (gvt_plan::tgroups) instead
// of stages 1 and 2.
template <class T>
void execute_block(gvt_plan *P, const T *D, int64_t ldd, const T *Tm, int64_t ldt, const T *V,
                   int R, int64_t ldv, T *U, int64_t ldu, int64_t block_stride, hipStream_t s,
                   int gprec) {
  layout_workspace<T>(P, R);
  Workspace &W = P->ws[prec_slot<T>()];
  const T *F[2] = {D, P->homogeneous ? D : Tm};
  const int64_t ldF[2] = {ldd, P->homogeneous ? ldd : ldt};
  const int32_t *dev_sel[4] = {P->idx[0].as<int32_t>(), P->idx[1].as<int32_t>(),
                               P->idx[2].as<int32_t>(), P->idx[3].as<int32_t>()};

  // input vector in key order, and segment sums where one-factor / degenerate terms need them
  mark(P, ST_PREP, 0, s);
  bool need_sv[2] = {false, false};
  for (const GemvSpec &g : P->gemvs) need_sv[g.key == SC ? 0 : 1] = true;
  for (const SBufSpec &sb : P->sbufs)
    if (sb.degenerate) need_sv[sb.key == SC ? 0 : 1] = true;
  for (int k = 0; k < 2; ++k) {
    const InputSort &is = P->insort[k];
    if (!is.built) continue;
    if (!P->prepacked)
      launch_pack_v<T>(V, ldv, is.perm.as<int32_t>(), P->n_in, R, wsp<T>(P, W.vs[k]), s, P->gate);
    if (need_sv[k])
      launch_segsum<T>(is.seg.as<int64_t>(), wsp<T>(P, W.vs[k]), is.nkeys, R, wsp<T>(P, W.sv[k]), s);
  }
  // one-factor products g = F^{o(1|2)} s
  for (size_t i = 0; i < P->gemvs.size(); ++i) {
    const GemvSpec &g = P->gemvs[i];
    const int ks = g.key == SC ? 0 : 1;
    launch_gemv<T>(F[g.f], ldF[g.f], rows_of(P, g.f), nkeys_of(P, g.key), g.sq != 0,
                   wsp<T>(P, W.sv[ks]), R, wsp<T>(P, W.gemv[i]), s);
  }
  mark(P, ST_PREP, 1, s);
  // stage 1 (shared scatters)
  mark(P, ST_STAGE1, 0, s);
  bool transposed[2] = {false, false};
  for (size_t i = 0; i < P->sbufs.size() && !gprec; ++i) {
    const SBufSpec &sb = P->sbufs[i];
    const int ks = sb.key == SC ? 0 : 1;
    const InputSort &is = P->insort[ks];
    T *S = wsp<T>(P, W.sbuf[i]);
    const int64_t ldS = sbuf_ld<T>(P, (int)i, R);
    if (sb.degenerate) {
      launch_colscale<T>(F[sb.fsc], ldF[sb.fsc], sb.d_rows.as<int32_t>(), (int64_t)sb.rows.size(),
                         wsp<T>(P, W.sv[ks]), is.nkeys, R, S, ldS, s);
      continue;
    }
    const T *Fc;
    int64_t ldc;
    if (P->flags & GVT_FLAG_SYMMETRIC_BASES) {
      Fc = F[sb.fsc];
      ldc = ldF[sb.fsc];
    } else {
      T *Ft = wsp<T>(P, W.trans[sb.fsc]);
      if (!transposed[sb.fsc]) {
        launch_transpose<T>(F[sb.fsc], ldF[sb.fsc], rows_of(P, sb.fsc), cols_of(P, sb.fsc), Ft,
                            rows_of(P, sb.fsc), s);
        transposed[sb.fsc] = true;
      }
      Fc = Ft;
      ldc = rows_of(P, sb.fsc);
    }
    launch_stage1<T>(Fc, ldc, sb.d_rows.as<int32_t>(), (int64_t)sb.rows.size(), sb.row0,
                     is.seg.as<int64_t>(), is.other.as<int32_t>(), is.nother, wsp<T>(P, W.vs[ks]),
                     is.nkeys, R, S, ldS, s, P->gate);
  }
  mark(P, ST_STAGE1, 1, s);
  // two-factor terms: stage 2
  mark(P, ST_STAGE2, 0, s);
  if (gprec) {
    std::vector<T *> tv(P->terms.size(), nullptr);
    for (size_t ti = 0; ti < P->terms.size(); ++ti) tv[ti] = wsp<T>(P, W.tvec[ti]);
    execute_gtiles<T>(P, gprec, F, ldF, V, R, ldv, tv.data(), s);
  }
  // (under plan_profile the launches repeat back to back, so the stage's events
  // bracket several launches and the per-launch figure carries no event
  // overhead; every stage-2 kernel overwrites its outputs)
  const int s2rep = P->prof && !gprec ? kProfileStage2Repeat : 1;
  for (int rep = 0; rep < s2rep; ++rep)
  for (size_t ti = 0; ti < P->terms.size() && !gprec; ++ti) {
    const TermSpec &t = P->terms[ti];
    if (t.type == TG) {
      const SBufSpec &sb = P->sbufs[t.sbuf];
      T *out = P->direct ? U : wsp<T>(P, W.tvec[ti]);
      const int64_t ldi = P->direct ? 1 : R, ldr = P->direct ? ldu : 1;
      const TileSet &tl = t.tiles[tile_class(R)];
      if (tile_class(R) == 0 && R == 1 &&
          launch_stage2_dual<T>(F[t.fdot], ldF[t.fdot], rows_of(P, t.fdot), tl.tileoff.as<int64_t>(),
                                tl.tiley.as<int32_t>(), tl.ntiles, tl.nyb, tl.yrows.as<int32_t>(),
                                tl.perm.as<int32_t>(), wsp<T>(P, W.sbuf[t.sbuf]), sbuf_ld<T>(P, t.sbuf, R),
                                (int64_t)sb.rows.size(), nkeys_of(P, sb.key), P->n_out, T(1), out, ldi, s,
                                P->gate)) {
        // low output density: dual tiles
      } else if (tile_class(R) == 0)
        launch_stage2<T>(F[t.fdot], ldF[t.fdot], rows_of(P, t.fdot), tl.tileoff.as<int64_t>(),
                         tl.tiley.as<int32_t>(), tl.tilemax.as<int32_t>(), tl.grow.as<uint8_t>(),
                         tl.ntiles, tl.nyb, tl.yrows.as<int32_t>(), tl.perm.as<int32_t>(),
                         wsp<T>(P, W.sbuf[t.sbuf]), sbuf_ld<T>(P, t.sbuf, R), (int64_t)sb.rows.size(),
                         nkeys_of(P, sb.key), R, T(1), out, ldi, ldr, s, P->gate);
      else
        launch_stage2y<T>(F[t.fdot], ldF[t.fdot], tl.tileoff.as<int64_t>(), tl.tiley.as<int32_t>(),
                          tl.tilemax.as<int32_t>(), tl.grow.as<uint8_t>(), tl.ntiles, tl.nyb,
                          tl.yrows.as<int32_t>(),
                          tl.perm.as<int32_t>(), wsp<T>(P, W.sbuf[t.sbuf]), sbuf_ld<T>(P, t.sbuf, R),
                          (int64_t)sb.rows.size(), nkeys_of(P, sb.key), R, T(1), out, ldi, ldr, s,
                          P->gate);
    }
  }
  mark(P, ST_STAGE2, 1, s);
  // one-factor and match terms, then the per-kind combination
  mark(P, ST_OTHER, 0, s);
  for (size_t ti = 0; ti < P->terms.size(); ++ti) {
    const TermSpec &t = P->terms[ti];
    if (t.type == TG) {
      continue;
    } else if (t.type == TO) {
      launch_gather_rows<T>(wsp<T>(P, W.gemv[t.gemv]), dev_sel[t.x], P->n_out, R,
                            wsp<T>(P, W.tvec[ti]), s);
    } else {
      const int ks = t.key == SC ? 0 : 1;
      const InputSort &is = P->insort[ks];
      const OutOrder &oo = P->outord[t.x == SA ? 0 : 1];
      launch_match<T>(F[t.f], ldF[t.f], cols_of(P, t.f), dev_sel[t.x], dev_sel[t.outkey], P->n_out,
                      oo.perm.as<int32_t>(), oo.off.as<int64_t>(), oo.nrows, is.seg.as<int64_t>(),
                      is.other.as<int32_t>(), wsp<T>(P, W.vs[ks]), is.nkeys, R,
                      wsp<T>(P, W.tvec[ti]), s);
    }
  }
  if (!P->direct) {
    CombineArgs<T> ca;
    ca.nterms = (int)P->terms.size();
    ca.nout = (int)P->outputs.size();
    for (size_t ti = 0; ti < P->terms.size(); ++ti) ca.t[ti] = wsp<T>(P, W.tvec[ti]);
    for (size_t o = 0; o < P->outputs.size(); ++o)
      for (auto &tc : P->outputs[o]) ca.coef[o][tc.first] = (T)tc.second;
    launch_combine<T>(ca, P->n_out, R, U, ldu, block_stride, s);
  }
  mark(P, ST_OTHER, 1, s);
}

template <class T>
void execute_t(gvt_plan *P, const T *D, int64_t ldd, const T *Tm, int64_t ldt, const T *V,
               int64_t nrhs, int64_t ldv, T *U, int64_t ldu, hipStream_t s, int gprec = 0) {
  const int64_t block_stride = nrhs * ldu;
  if (P->n_out == 0) return;
  if (P->n_in == 0) {
    launch_fill<T>(U, P->n_out, nrhs * (int64_t)P->outputs.size(), ldu, T(0), s);
    return;
  }
  GVT_REQUIRE(!P->prepacked || rhs_block(nrhs, P->max_rhs[prec_slot<T>()]) == nrhs, GVT_ERR_ARG,
              "internal: a prepacked input is one whole RHS block");
  int64_t r0 = 0;
  while (r0 < nrhs) {
    const int64_t left = nrhs - r0;
    const int R = rhs_block(left, P->max_rhs[prec_slot<T>()]);
    plan_ensure_tiles(P, tile_class(R), s);
    execute_block<T>(P, D, ldd, Tm, ldt, V + r0 * ldv, R, ldv, U + r0 * ldu, ldu, block_stride, s, gprec);
    r0 += R;
  }
}

}  // namespace

// ---- dense tiles ---------------------------------------------------------------
// Vmat[c, e] = sum of v_j over the pairs j = (c, e).  One thread per position
// of the sorted input pairs (key segments, the other index ascending inside
// each): a position that starts a run of equal (key, other) sums the run in
// sorted order and stores it; the others store nothing.
template <class T>
__global__ void tiles_scatter_kernel(const int32_t *__restrict__ perm, const int32_t *__restrict__ other,
                                     const int32_t *__restrict__ keyidx, int64_t n, const T *__restrict__ v,
                                     int key_is_c, int64_t tcols, T *__restrict__ Vmat) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t o = other[p], k = keyidx[perm[p]];
  if (p > 0 && other[p - 1] == o && keyidx[perm[p - 1]] == k) return;  // inside a run
  T acc = v[perm[p]];
  for (int64_t q = p + 1; q < n && other[q] == o && keyidx[perm[q]] == k; ++q) acc += v[perm[q]];
  const int64_t c = key_is_c ? k : o, e = key_is_c ? o : k;
  Vmat[c * tcols + e] = acc;
}

template <class T>
__global__ void tiles_zero_kernel(T *__restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = T(0);
}

// u[i] = Umat[a_i, b_i]
template <class T>
__global__ void tiles_gather_kernel(const T *__restrict__ Umat, int64_t ldum, const int32_t *__restrict__ a,
                                    const int32_t *__restrict__ b, int64_t n, T *__restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) u[i] = Umat[(int64_t)a[i] * ldum + b[i]];
}

// u[i * stride] = Umat[p_i, q_i]
template <class T>
__global__ void tiles_gather_term_kernel(const T *__restrict__ Umat, int64_t ldum, const int32_t *__restrict__ p,
                                         const int32_t *__restrict__ q, int64_t n, T *__restrict__ u,
                                         int64_t stride) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) u[i * stride] = Umat[(int64_t)p[i] * ldum + q[i]];
}

// Time estimates per RHS of a dense product of the plan's shapes against the
// gather path's Theorem 1 flops (ngroups dense products).  A GEMM with few
// 128 x 128 output tiles leaves matrix cores idle: its rate scales with
// min(1, tiles / kTilesFull).
static bool dense_beats_gather(const gvt_plan *P, int prec, int64_t fa_rows, int64_t fb_rows, int ngroups) {
  const double es = prec == GVT_F64 ? 8.0 : 4.0;
  const double rate = prec == GVT_F64 ? kTilesRateF64 : kTilesRateF32;
  auto gemm_s = [&](double m, double n, double k) {
    const double tiles = std::ceil(m / 128.0) * std::ceil(n / 128.0);
    return 2.0 * m * n * k / (rate * std::min(1.0, tiles / kTilesFull));
  };
  const double bytes = es * (2.0 * P->d_cols * P->t_cols + 2.0 * fa_rows * fb_rows + fa_rows * P->t_cols);
  const double t_dense = ngroups * (gemm_s((double)fa_rows, (double)P->t_cols, (double)P->d_cols) +
                                    gemm_s((double)fa_rows, (double)fb_rows, (double)P->t_cols) + bytes / 4.0e12);
  const double t_gather = 2.0 * P->cost_fma / (prec == GVT_F64 ? kGatherRateF64 : kGatherRateF32);
  return t_dense < t_gather;
}

bool plan_uses_gtiles(const gvt_plan *P, int prec) {
  if (!P->gtiles_ok || P->tiles_mode < 0) return false;
  if (P->tiles_mode > 0 || prec == GVT_BF16X3 || prec == GVT_BF16X6) return true;
  int64_t ra = 0, rb = 0;
  for (const TileGroup &g : P->tgroups) {
    ra = std::max(ra, rows_of(P, g.fa));
    rb = std::max(rb, rows_of(P, g.fb));
  }
  return dense_beats_gather(P, prec, ra, rb, (int)P->tgroups.size());
}

// The two-factor terms of a multi-term plan as dense tiles: per RHS column r
// and operator group, Vmat[c, e] from v (duplicates summed in the sorted
// order), Umat = F_A Vmat F_B^T in precision gprec, and each term's outputs
// gathered into column r of its term vector (row stride R).
template <class T>
void execute_gtiles(gvt_plan *P, int gprec, const T *const *F, const int64_t *ldF, const T *V, int R,
                    int64_t ldv, T *const *tvec, hipStream_t s) {
  const int ks = P->insort[0].built ? 0 : 1;  // either input sort yields Vmat[c, e]
  const InputSort &is = P->insort[ks];
  GVT_REQUIRE(is.built, GVT_ERR_ARG, "internal: dense tiles without an input sort");
  int64_t ra = 0, rb = 0;
  for (const TileGroup &g : P->tgroups) {
    ra = std::max(ra, rows_of(P, g.fa));
    rb = std::max(rb, rows_of(P, g.fb));
  }
  const int64_t nv = P->d_cols * P->t_cols, nu = ra * rb;
  const size_t al = 256;
  const size_t vb = ((size_t)nv * sizeof(T) + al - 1) / al * al, ub = ((size_t)nu * sizeof(T) + al - 1) / al * al;
  const size_t wb = dense_workspace_bytes(gprec, ra, P->d_cols, rb, P->t_cols);
  char *base = static_cast<char *>(P->tiles_ws.ensure(vb + ub + wb));
  T *Vmat = reinterpret_cast<T *>(base), *Umat = reinterpret_cast<T *>(base + vb);
  void *wsd = base + vb + ub;
  for (int r = 0; r < R; ++r) {
    tiles_zero_kernel<T><<<(unsigned)std::min<int64_t>(ceil_div(nv, 256), 4096), 256, 0, s>>>(Vmat, nv);
    tiles_scatter_kernel<T><<<(unsigned)ceil_div(P->n_in, 256), 256, 0, s>>>(
        is.perm.as<int32_t>(), is.other.as<int32_t>(), P->idx[ks == 0 ? SC : SE].as<int32_t>(), P->n_in,
        V + r * ldv, ks == 0 ? 1 : 0, P->t_cols, Vmat);
    for (const TileGroup &g : P->tgroups) {
      const int64_t na = rows_of(P, g.fa), nb = rows_of(P, g.fb);
      dense_matvec(gprec, F[g.fa], na, P->d_cols, ldF[g.fa], F[g.fb], nb, P->t_cols, ldF[g.fb], Vmat,
                   P->t_cols, Umat, nb, wsd, s);
      for (const TileTerm &tt : g.terms)
        tiles_gather_term_kernel<T><<<(unsigned)ceil_div(P->n_out, 256), 256, 0, s>>>(
            Umat, nb, P->idx[tt.p].as<int32_t>(), P->idx[tt.q].as<int32_t>(), P->n_out, tvec[tt.ti] + r,
            (int64_t)R);
    }
  }
}
template void execute_gtiles<double>(gvt_plan *, int, const double *const *, const int64_t *, const double *, int,
                                     int64_t, double *const *, hipStream_t);
template void execute_gtiles<float>(gvt_plan *, int, const float *const *, const int64_t *, const float *, int,
                                    int64_t, float *const *, hipStream_t);

bool plan_uses_tiles(const gvt_plan *P, int prec) {
  if (!P->tiles_ok || P->tiles_mode < 0) return false;
  if (P->tiles_mode > 0 || prec == GVT_BF16X3 || prec == GVT_BF16X6) return true;
  return dense_beats_gather(P, prec, P->d_rows, P->t_rows, 1);
}

template <class T>
static void execute_tiles(gvt_plan *P, int prec, const void *D, int64_t ldd, const void *Tm, int64_t ldt,
                          const T *V, int64_t nrhs, int64_t ldv, T *U, int64_t ldu, hipStream_t s) {
  const TermSpec &t0 = P->terms[P->outputs[0][0].first];
  const SBufSpec &sb = P->sbufs[t0.sbuf];
  const int ks = sb.key == SC ? 0 : 1;
  const InputSort &is = P->insort[ks];
  GVT_REQUIRE(is.built, GVT_ERR_ARG, "internal: dense tiles without the input sort");
  const int64_t nv = P->d_cols * P->t_cols, nu = P->d_rows * P->t_rows;
  const size_t al = 256;
  const size_t vb = ((size_t)nv * sizeof(T) + al - 1) / al * al, ub = ((size_t)nu * sizeof(T) + al - 1) / al * al;
  const size_t wb = dense_workspace_bytes(prec, P->d_rows, P->d_cols, P->t_rows, P->t_cols);
  char *base = static_cast<char *>(P->tiles_ws.ensure(vb + ub + wb));
  T *Vmat = reinterpret_cast<T *>(base), *Umat = reinterpret_cast<T *>(base + vb);
  void *wsd = base + vb + ub;
  for (int64_t r = 0; r < nrhs; ++r) {
    tiles_zero_kernel<T><<<(unsigned)std::min<int64_t>(ceil_div(nv, 256), 4096), 256, 0, s>>>(Vmat, nv);
    tiles_scatter_kernel<T><<<(unsigned)ceil_div(P->n_in, 256), 256, 0, s>>>(
        is.perm.as<int32_t>(), is.other.as<int32_t>(), P->idx[sb.key].as<int32_t>(), P->n_in, V + r * ldv,
        sb.key == SC ? 1 : 0, P->t_cols, Vmat);
    dense_matvec(prec, D, P->d_rows, P->d_cols, ldd, Tm, P->t_rows, P->t_cols, ldt, Vmat, P->t_cols, Umat,
                 P->t_rows, wsd, s);
    tiles_gather_kernel<T><<<(unsigned)ceil_div(P->n_out, 256), 256, 0, s>>>(
        Umat, P->t_rows, P->idx[0].as<int32_t>(), P->idx[1].as<int32_t>(), P->n_out, U + r * ldu);
  }
}

void plan_execute(gvt_plan *P, int prec, const void *D, int64_t ldd, const void *T, int64_t ldt,
                  const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu, hipStream_t s) {
  GVT_REQUIRE(P, GVT_ERR_ARG, "null plan");
  GVT_REQUIRE(!P->prof || nrhs <= 8, GVT_ERR_ARG, "stage profile covers one RHS block (nrhs <= 8)");
  GVT_REQUIRE(nrhs >= 1, GVT_ERR_ARG, "nrhs must be >= 1");
  GVT_REQUIRE(prec == GVT_F64 || prec == GVT_F32 || prec == GVT_BF16X3 || prec == GVT_BF16X6, GVT_ERR_ARG, "unknown precision");
  GVT_REQUIRE(ldu >= P->n_out && ldv >= P->n_in, GVT_ERR_ARG, "ldv < n_in or ldu < n_out");
  GVT_REQUIRE(P->n_out == 0 || U, GVT_ERR_ARG, "null U");
  GVT_REQUIRE(P->n_in == 0 || V, GVT_ERR_ARG, "null V");
  const bool needT = !P->homogeneous && P->n_in > 0 && P->n_out > 0;
  GVT_REQUIRE(D || P->n_in == 0 || P->n_out == 0, GVT_ERR_ARG, "null D");
  GVT_REQUIRE(!needT || T, GVT_ERR_ARG, "null T (heterogeneous kinds need T)");
  GVT_REQUIRE(ldd >= P->d_cols, GVT_ERR_ARG, "ldd < d_cols");
  GVT_REQUIRE(!needT || ldt >= P->t_cols, GVT_ERR_ARG, "ldt < t_cols");
  P->last_stream = s;
  if (P->dense) {
    // complete data: each RHS column is vec(Vmat) with Vmat d_cols x t_cols row-major
    for (int64_t r = 0; r < nrhs; ++r) {
      const size_t es = prec == GVT_F64 ? 8 : 4;
      dense_matvec(prec, D, P->d_rows, P->d_cols, ldd, T, P->t_rows, P->t_cols, ldt,
                   static_cast<const char *>(V) + r * ldv * es, P->t_cols,
                   static_cast<char *>(U) + r * ldu * es, P->t_rows, nullptr, s);
    }
    return;
  }
  if (plan_uses_tiles(P, prec)) {
    if (prec == GVT_F64)
      execute_tiles<double>(P, prec, D, ldd, T, ldt, (const double *)V, nrhs, ldv, (double *)U, ldu, s);
    else
      execute_tiles<float>(P, prec, D, ldd, T, ldt, (const float *)V, nrhs, ldv, (float *)U, ldu, s);
    check_launch(s);
    return;
  }
  const bool gt = plan_uses_gtiles(P, prec);
  GVT_REQUIRE(gt || prec == GVT_F64 || prec == GVT_F32, GVT_ERR_UNSUPPORTED,
              "split-bf16 products are provided on the matrix-core paths only (complete data, dense tiles "
              "of two-factor terms keyed by (c, e))");
  if (prec == GVT_F64)
    execute_t<double>(P, (const double *)D, ldd, (const double *)T, ldt, (const double *)V, nrhs,
                      ldv, (double *)U, ldu, s, gt ? prec : 0);
  else
    execute_t<float>(P, (const float *)D, ldd, (const float *)T, ldt, (const float *)V, nrhs, ldv,
                     (float *)U, ldu, s, gt ? prec : 0);
  check_launch(s);
}

namespace {
template <class T> int pack_targets_t(gvt_plan *P, int R, void **vs, const int32_t **inv) {
  layout_workspace<T>(P, R);
  Workspace &W = P->ws[prec_slot<T>()];
  int k = 0;
  for (int ks = 0; ks < 2; ++ks) {
    if (!P->insort[ks].built) continue;
    vs[k] = wsp<T>(P, W.vs[ks]);
    inv[k] = P->insort[ks].inv.as<int32_t>();
    ++k;
  }
  return k;
}
}  // namespace

int plan_pack_targets(gvt_plan *P, int prec, int R, void **vs, const int32_t **inv) {
  GVT_REQUIRE(P && !P->dense && (prec == GVT_F64 || prec == GVT_F32), GVT_ERR_ARG,
              "pack targets exist for gather-path plans in F64 or F32");
  GVT_REQUIRE(rhs_block(R, rhs_cap(P, prec)) == R, GVT_ERR_ARG, "R is not a whole RHS block of the plan");
  return prec == GVT_F64 ? pack_targets_t<double>(P, R, vs, inv) : pack_targets_t<float>(P, R, vs, inv);
}

void plan_pack(gvt_plan *P, int prec, const void *V, int64_t ldv, int R, hipStream_t s) {
  void *vs[2];
  const int32_t *inv[2];
  const int nk = plan_pack_targets(P, prec, R, vs, inv);
  int k = 0;
  for (int ks = 0; ks < 2 && k < nk; ++ks) {
    if (!P->insort[ks].built) continue;
    if (prec == GVT_F64)
      launch_pack_v<double>((const double *)V, ldv, P->insort[ks].perm.as<int32_t>(), P->n_in, R,
                            (double *)vs[k], s);
    else
      launch_pack_v<float>((const float *)V, ldv, P->insort[ks].perm.as<int32_t>(), P->n_in, R,
                           (float *)vs[k], s);
    ++k;
  }
}

void plan_profile(gvt_plan *P, int prec, const void *D, int64_t ldd, const void *T, int64_t ldt,
                  const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu, int reps,
                  double *stage_ms, hipStream_t s) {
  GVT_REQUIRE(P && stage_ms && reps >= 1, GVT_ERR_ARG, "bad profile arguments");
  GVT_REQUIRE(!P->dense, GVT_ERR_UNSUPPORTED, "stage profile is for the gather path");
  std::vector<hipEvent_t> ev(2 * kStages);
  for (auto &e : ev) GVT_HIP_CHECK(hipEventCreate(&e));
  for (int k = 0; k < kStages; ++k) stage_ms[k] = 0.0;
  struct Cleanup {
    gvt_plan *P;
    std::vector<hipEvent_t> &ev;
    ~Cleanup() {
      P->prof = nullptr;
      for (auto &e : ev) (void)hipEventDestroy(e);
    }
  } cleanup{P, ev};
  P->prof = ev.data();
  for (int r = 0; r < reps; ++r) {
    plan_execute(P, prec, D, ldd, T, ldt, V, nrhs, ldv, U, ldu, s);
    GVT_HIP_CHECK(hipStreamSynchronize(s));
    for (int k = 0; k < kStages; ++k) {
      float ms = 0.f;
      GVT_HIP_CHECK(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
      stage_ms[k] += ms;
    }
  }
  for (int k = 0; k < kStages; ++k) stage_ms[k] /= reps;
  if (!plan_uses_gtiles(P, prec)) stage_ms[ST_STAGE2] /= kProfileStage2Repeat;
}

}  // namespace gvt
