// Plan object: index preprocessing + the per-kind Kronecker term program.
#pragma once

#include <array>

#include "common.h"
#include "kernels.h"
#include "plan_dev.h"

namespace gvt {

// Index selectors: output-side a, b; input-side c, e.
enum Sel { SA = 0, SB = 1, SC = 2, SE = 3 };
// Base matrices.
enum Mat { FD = 0, FT = 1 };

struct InputSort {  // input pairs sorted by one index (key segments), then by the other
  bool built = false;
  int64_t nkeys = 0;
  int64_t nother = 0;  // range of the other index
  DevMem perm;   // int32[n_in]: sorted position -> input index j
  DevMem inv;    // int32[n_in]: input index j -> sorted position (inverse of perm)
  DevMem other;  // int32[n_in]: the other index of the pair at that position
  DevMem seg;    // int64[nkeys + 1]: segment offsets
};

struct OutOrder {  // output pairs grouped by one output-side index
  bool built = false;
  int64_t nrows = 0;  // range of the grouping index
  DevMem perm;        // int32[n_out]: position -> output index i
  DevMem off;         // int64[nrows + 1]: first position of each index value
};

struct SBufSpec {  // one stage-1 result S = scatter of F_sc by `key` with column index `other`
  int fsc = FD, key = SC, other = SE;
  bool degenerate = false;       // key == other: S[y, k] = F[y, k] * segsum[k]
  std::vector<int32_t> rowmap;   // F_sc row -> compact S row (-1: not needed)
  std::vector<int32_t> rows;     // compact S rows -> F_sc row
  int64_t row0 = -1;             // rows[i] = row0 + i for all i (contiguous), else -1
  int64_t nneed = 0;             // rows the terms read (rows may add a few to close gaps)
  DevMem d_rows;
  DevMem d_rowmap;               // device copy of rowmap (device-built plans)
};

enum TermType { TG = 0, TO = 1, TM = 2 };

// Stage-2 tiles of one two-factor term for one S-row block size.  Outputs are
// ordered by (x block, S-row block, x, S row); tiles are numbered
// x_block * nyb + y_block.
struct TileSet {
  bool built = false;
  int ysz = 0;          // S rows per block (<= kStage2MaxS)
  DevMem perm, yrows;   // int32[n_out] per position
  DevMem tileoff;       // int64[ntiles * (kStage2Rows + 1)]: start of each x row in a tile
  DevMem tiley;         // int32[2 * ntiles]: first S row and S-row count of the tile
  DevMem tilemax;       // int32[ntiles]: largest per-row output count in the tile
  DevMem grow;          // uint8[ntiles * kStage2Rows]: the group row each group of a tile
                        // works on, rows by descending output count (ties by row)
  int64_t ntiles = 0;
  int nyb = 0;
  DevMem blob;          // the arrays' allocation when built after the plan
};

// RHS classes with their own stage-2 tiles: [0] blocks of 1-2 RHS, [1] of 4-8.
constexpr int kTileClasses = 2;
inline int tile_class(int R) { return R >= 4 ? 1 : 0; }

struct TermSpec {
  int type = TG;
  // G (two-factor Kronecker term):  u_i = sum_k F_dot[x_i, k] S[y_i, k]
  int fdot = FD, x = SA, y = SB, sbuf = -1;
  TileSet tiles[kTileClasses];
  // O (one-factor term):  u_i = g[x_i], g = F^{o(1|2)} segsum_key
  int gemv = -1;
  // M (Cartesian sparse match):  u_i = sum_{j: key_j = outkey_i} F[x_i, other_j] v_j
  int f = FD, outkey = SB, key = SE;
  bool operator==(const TermSpec &) const = delete;
};

// Multi-term dense tiles: a two-factor term u_i = sum_j F_dot[x_i, key_j]
// F_sc[y_i, other_j] v_j keyed (c, e) or (e, c) is the gather of
// Umat = F_A Vmat F_B^T at (p_i, q_i), with Vmat[c, e] = sum of v over the
// pairs (c, e); terms with the same F_A, F_B share Umat.
struct TileTerm {
  int ti, p, q;  // term index, output selectors (SA / SB) of Umat's row and column
};
struct TileGroup {
  int fa, fb;  // Umat = F[fa] Vmat F[fb]^T
  std::vector<TileTerm> terms;
};

struct GemvSpec {
  int f = FD, sq = 0, key = SC;
};

struct Workspace {
  DevMem pool;
  size_t need = 0;
  int R = 0;
  // offsets into pool (bytes); -1 = unused
  std::array<int64_t, 2> vs{{-1, -1}}, sv{{-1, -1}}, trans{{-1, -1}};
  std::vector<int64_t> sbuf, gemv, tvec;
};

}  // namespace gvt

struct gvt_plan {
  std::vector<int> kinds;
  bool homogeneous = false;
  bool dense = false;
  int flags = 0;
  int64_t d_rows = 0, d_cols = 0, t_rows = 0, t_cols = 0, n_out = 0, n_in = 0;
  std::array<int64_t, 4> uniq{{0, 0, 0, 0}};
  gvt::DevMem blob;    // one device allocation holding the uploaded index arrays below
  // Device-built plans (large index sets): the index work runs on the GPU;
  // idx always holds the plan's own copies of a, b, c, e, devblob the sorted
  // arrays and tile orders, scratch the sort buffers.
  bool on_device = false;
  gvt::DevMem idxblob, devblob;
  gvt::DevScratch scratch;
  gvt::DevMem idx[4];  // device copies of a, b, c, e (int32), when a term reads them
  gvt::InputSort insort[2];   // [0]: by c (other = e), [1]: by e (other = c)
  gvt::OutOrder outord[2];    // [0]: grouped by a, [1]: grouped by b
  std::vector<int32_t> h_out[2];  // host copies of a, b (host-built plans: tiles built on demand)
  std::vector<gvt::SBufSpec> sbufs;
  std::vector<gvt::GemvSpec> gemvs;
  std::vector<gvt::TermSpec> terms;
  std::vector<std::vector<std::pair<int, double>>> outputs;  // per kind: (term, coef)
  bool direct = false;  // single kind, single G term with coefficient 1
  // Device flag gating the two-factor product kernels (see launch_pack_v);
  // set by a solver around the products it may want to skip, else null.
  const int *gate = nullptr;
  // Set by a solver whose own kernels have already written the input vector
  // in key order (plan_pack_targets): the products then skip their pack.
  bool prepacked = false;
  // Largest block of right-hand sides one product pass carries (1, 2, 4 or
  // 8), for FP64 [0] and FP32 [1] products: the tuned kMaxRhsBlockF64/F32,
  // or GVT_MAX_RHS_BLOCK (both) / GVT_MAX_RHS_BLOCK_F64 / _F32 when the plan
  // is built.
  int max_rhs[2] = {8, 8};
  gvt::Workspace ws[2];  // per precision (F64, F32)
  hipStream_t last_stream = nullptr;
  // Theorem 1 cost of the chosen term program (FMA count per RHS), for reporting
  double cost_fma = 0.0;
  // Dense tiles for dense-but-incomplete data: a plan of one Kronecker term may
  // run its product as the complete-data contraction M Vmat N^T on matrix
  // cores, with v scattered into a zero grid Vmat (duplicates summed in the
  // sorted order) and the outputs gathered from Umat.  mode: 0 chosen per call
  // by the cost model (tuning.h), 1 always, -1 never.
  bool tiles_ok = false;
  int tiles_mode = 0;
  gvt::DevMem tiles_ws;  // Vmat, Umat and the dense product's workspace
  // The same for plans of several terms (not direct): every two-factor term
  // goes through one dense product per operator group (TileGroup) and a
  // gather into its term vector; one-factor and match terms and the per-kind
  // combination stay on the gather path.  Possible when every two-factor term
  // is keyed by (c, e) or (e, c); the same mode and cost model decide.
  std::vector<gvt::TileGroup> tgroups;
  bool gtiles_ok = false;
  // optional stage timing: events recorded at stage-group boundaries
  hipEvent_t *prof = nullptr;  // [kStages][2] start/stop, or null
};

namespace gvt {
// stage groups reported by gvt_plan_profile
enum Stage { ST_PREP = 0, ST_STAGE1 = 1, ST_STAGE2 = 2, ST_OTHER = 3, kStages = 4 };
// back-to-back repeats of a product's stage-2 launches under gvt_plan_profile
constexpr int kProfileStage2Repeat = 8;
int64_t rows_of(const gvt_plan *P, int f);
int64_t cols_of(const gvt_plan *P, int f);
int64_t nkeys_of(const gvt_plan *P, int key);
// rhs_hint: the number of right-hand sides the caller expects; the stage-2
// tiles of its class are built now, those of the other class on first use.
void plan_build(gvt_plan *P, const int *kinds, int nkinds, int64_t d_rows, int64_t d_cols,
                int64_t t_rows, int64_t t_cols, const int32_t *a, const int32_t *b, int64_t n_out,
                const int32_t *c, const int32_t *e, int64_t n_in, int flags, hipStream_t s,
                int rhs_hint = 1);
// Build the stage-2 tiles of RHS class `cls` for every two-factor term (no-op
// when built).  Synchronous host work and a copy: not allowed while `s` is
// being captured.
void plan_ensure_tiles(gvt_plan *P, int cls, hipStream_t s);
// The RHS cap of a plan for products in precision prec (GVT_F64 or GVT_F32).
inline int rhs_cap(const gvt_plan *P, int prec) { return P->max_rhs[prec == GVT_F64 ? 0 : 1]; }
// RHS block of a product pass for `left` remaining right-hand sides.
inline int rhs_block(int64_t left, int max_rhs) {
  const int64_t m = left < max_rhs ? left : max_rhs;
  return m >= 8 ? 8 : m >= 4 ? 4 : m >= 2 ? 2 : 1;
}
// S rows per stage-2 block for a term: from the tuning target of the class
// (or the GVT_STAGE2_TARGET_R1 / GVT_STAGE2_TARGET_R8 environment override).
int stage2_block_rows(const gvt_plan *P, const TermSpec &t, int cls);
void plan_execute(gvt_plan *P, int prec, const void *D, int64_t ldd, const void *T, int64_t ldt,
                  const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu, hipStream_t s);
// Whether a product in precision prec takes the dense-tile form (see tiles_ok),
// and whether a multi-term product runs its two-factor terms as dense tiles
// (see gtiles_ok).
bool plan_uses_tiles(const gvt_plan *P, int prec);
bool plan_uses_gtiles(const gvt_plan *P, int prec);
// Where a product with one block of R right-hand sides (R a block size the
// plan runs whole: rhs_block(R, max_rhs) == R) reads its input in key order:
// for each input sort k < the returned count, element (j, r) of the input
// goes to vs[k][inv[k][j] * R + r].  Lays out the precision's workspace for R.
int plan_pack_targets(gvt_plan *P, int prec, int R, void **vs, const int32_t **inv);
// The pack alone: V (n_in x R, column stride ldv) into those places.
void plan_pack(gvt_plan *P, int prec, const void *V, int64_t ldv, int R, hipStream_t s);
void plan_profile(gvt_plan *P, int prec, const void *D, int64_t ldd, const void *T, int64_t ldt,
                  const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu, int reps,
                  double *stage_ms, hipStream_t s);
}  // namespace gvt
