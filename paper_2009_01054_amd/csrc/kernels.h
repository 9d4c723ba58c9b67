// Launcher declarations for the library's kernels (internal).
#pragma once

#include "common.h"

namespace gvt {

constexpr int kMaxCombineTerms = 16;
// Stage-2 tiles: kStage2Rows consecutive F1 rows x at most kStage2MaxS S rows.
constexpr int kStage2Rows = 32;
constexpr int kStage2MaxS = 64;
constexpr double kL2BytesPerXcd = 4.0 * 1024 * 1024;  // gfx950: 4 MB of L2 per XCD
constexpr double kMallBytes = 256.0 * 1024 * 1024;    // MI355X: 256 MB memory-side cache
constexpr int kMaxCombineOut = 8;

// Row stride (elements) of a stage-1 buffer: nkeys x R values padded to whole
// 1 KB chunks, the unit in which stage 2 copies S rows into LDS.
template <class T> __host__ __device__ inline int64_t sbuf_row_ld(int64_t nkeys, int R) {
  const int64_t chunk = 1024 / (int64_t)sizeof(T);
  return (nkeys * R + chunk - 1) / chunk * chunk;
}

template <class T> struct CombineArgs {
  int nterms = 0;
  int nout = 0;
  const T *t[kMaxCombineTerms] = {};
  T coef[kMaxCombineOut][kMaxCombineTerms] = {};
};

// gate (optional device flag): when it reads 0 at run time, the launch does
// nothing.  The product kernels of two-factor terms take one, so a captured
// iteration whose systems have all stopped skips its product.
template <class T>
void launch_pack_v(const T *V, int64_t ldv, const int32_t *perm, int64_t n, int R, T *vs,
                   hipStream_t s, const int *gate = nullptr);
template <class T>
void launch_segsum(const int64_t *seg, const T *vs, int64_t nkeys, int R, T *out, hipStream_t s);
// Re-read the environment overrides of the tuned launch shapes (called when a
// plan is built).
void refresh_launch_knobs();
bool stage1_wide_enabled();  // the several-rows-per-lane stage-1 walk is on

// Stage 1: the segment walk over the key segments of the sorted input pairs.
// row0 >= 0 states that rows[i] = row0 + i for every i, which allows the walk
// with several rows per lane; -1 otherwise.
template <class T>
void launch_stage1(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows, int64_t row0,
                   const int64_t *seg, const int32_t *other, int64_t nother, const T *vs,
                   int64_t nkeys, int R, T *S, int64_t ldS, hipStream_t s,
                   const int *gate = nullptr);
template <class T>
void launch_colscale(const T *F, int64_t ldf, const int32_t *rows, int64_t nrows, const T *sv,
                     int64_t nkeys, int R, T *S, int64_t ldS, hipStream_t s);
template <class T>
void launch_stage2(const T *F1, int64_t ld1, int64_t nx, const int64_t *tileoff, const int32_t *tiley,
                   const int32_t *tilemax, const uint8_t *grow, int64_t ntiles, int nyb,
                   const int32_t *yrows, const int32_t *perm, const T *S, int64_t ldS, int64_t nsrows,
                   int64_t nkeys, int R, T coef, T *out, int64_t ldi, int64_t ldr, hipStream_t s,
                   const int *gate = nullptr);
// Stage 2 with one RHS over dual tiles (128 F1 rows x two S-row blocks of the
// same tiles, both operands staged in LDS) at low output density; returns
// false, launching nothing, where it does not apply.
template <class T>
bool launch_stage2_dual(const T *F1, int64_t ld1, int64_t nx, const int64_t *tileoff, const int32_t *tiley,
                        int64_t ntiles, int nyb, const int32_t *yrows, const int32_t *perm, const T *S,
                        int64_t ldS, int64_t nsrows, int64_t nkeys, int64_t n_out, T coef, T *out, int64_t ldi,
                        hipStream_t s, const int *gate = nullptr);
// Stage 2 with S-row grouped tiles (blocks of R = 4 or 8 RHS).
template <class T>
void launch_stage2y(const T *F1, int64_t ld1, const int64_t *tileoff, const int32_t *tilex,
                    const int32_t *tilemax, const uint8_t *grow, int64_t ntiles, int nxb,
                    const int32_t *xrows, const int32_t *perm, const T *S, int64_t ldS, int64_t nsr,
                    int64_t nkeys, int R, T coef, T *out, int64_t ldi, int64_t ldr, hipStream_t s,
                    const int *gate = nullptr);
template <class T>
void launch_gemv(const T *F, int64_t ldf, int64_t nrows, int64_t ncols, bool sq, const T *sv, int R,
                 T *g, hipStream_t s);
template <class T>
void launch_gather_rows(const T *g, const int32_t *sel, int64_t n, int R, T *t, hipStream_t s);
// Cartesian match terms.  With outputs grouped by F row (operm/xoff over
// nxrows rows) and a row of at most 64 KB, one block stages its row in LDS;
// otherwise one 16-lane group per output gathers from global memory.
template <class T>
void launch_match(const T *F, int64_t ldf, int64_t ncols, const int32_t *xsel, const int32_t *ksel,
                  int64_t n, const int32_t *operm, const int64_t *xoff, int64_t nxrows,
                  const int64_t *seg, const int32_t *other, const T *vs, int64_t nkeys, int R, T *t,
                  hipStream_t s);
template <class T>
void launch_transpose(const T *F, int64_t ldf, int64_t rows, int64_t cols, T *Ft, int64_t ldt,
                      hipStream_t s);
template <class T>
void launch_combine(const CombineArgs<T> &a, int64_t n, int R, T *U, int64_t ldu,
                    int64_t block_stride, hipStream_t s);
template <class T>
void launch_fill(T *U, int64_t rows, int64_t cols, int64_t ld, T val, hipStream_t s);

// ---- grouped launches over many independent single-term products ----------
// One descriptor per problem holds everything a Kronecker-term product
// u = stage2(F1, stage1(Fc, V)) needs; one launch covers the blocks of all
// problems through a work list of (problem, local block) items.
template <class T> struct GroupDesc {
  // input vector (RHS r at V + r * ldv) and its key-ordered copy
  const T *V;
  int64_t ldv;
  const int32_t *perm_in;
  int64_t n_in;
  T *vs;
  // stage 1
  const T *Fc;
  int64_t ldc;
  const int32_t *rows;
  int64_t nrows;
  const int64_t *seg;
  const int32_t *other;
  int64_t nkeys;
  int64_t row0;  // >= 0: S row i is F2 row row0 + i, walked several rows per lane
  T *S;         // row stride sbuf_row_ld<T>(nkeys, R) for an R-column RHS block
  int64_t nkb;  // stage-1 key blocks
  // stage 1 over an F2 slice resident in LDS (slice != 0): nother F2 columns,
  // nkr key ranges of kpr keys per row block
  int64_t nother, kpr, nkr;
  int slice;
  // stage 2, one tile set per RHS class ([0]: blocks of 1-2 RHS, F1-row groups;
  // [1]: blocks of 4-8 RHS, S-row groups, where tiley holds each tile's F1-row
  // block, yrows each output's F1 row and nyb the number of F1-row blocks)
  const T *F1;
  int64_t ld1;
  int64_t nx;
  const int64_t *tileoff[2];
  const int32_t *tiley[2];
  const int32_t *tilemax[2];
  const uint8_t *grow[2];  // per tile, the group row of each group (descending output count)
  const int32_t *yrows[2];
  const int32_t *perm_out[2];
  int64_t nyb[2];
  T *U;  // RHS r at U + r * ldu
  int64_t ldu;
};

struct GroupItem {
  int32_t p;   // problem
  int32_t li;  // block within the problem
};

// Work items per problem for each grouped launch, in the problem's natural block order.
int64_t group_pack_blocks(int64_t n_in);
// Stage 1: picks the problem's walk (over an F2 slice in LDS, or several rows
// per lane, when its S rows are the contiguous range starting at F2 row
// row0 >= 0; else one row per lane), sets d.slice, d.row0, d.nkb (d.kpr, d.nkr)
// and returns the problem's blocks (n_in, nkeys, nrows and nother set).
// Problems with d.slice set go in the work list of launch_group_stage1_slice.
template <class T>
int64_t group_stage1_setup(GroupDesc<T> &d, int64_t row0);
// Dynamic LDS the slice walk of a problem needs.
template <class T> inline size_t group_stage1_slice_lds(const GroupDesc<T> &d) {
  return d.slice ? (size_t)d.nother * 256 : 0;
}

// active[p] == 0 skips problem p (null: every problem runs).  r0: first RHS of the block.
template <class T>
void launch_group_pack(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                       int64_t r0, const uint8_t *active, hipStream_t s);
template <class T>
void launch_group_stage1(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                         const uint8_t *active, hipStream_t s);
// lds: the largest group_stage1_slice_lds of the listed problems.
template <class T>
void launch_group_stage1_slice(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                               const uint8_t *active, size_t lds, hipStream_t s);
template <class T>
void launch_group_stage2(const GroupDesc<T> *desc, const GroupItem *items, int64_t nitems, int R,
                         int64_t r0, const uint8_t *active, hipStream_t s);

// Dense complete-data path (matrix cores).  ws: workspace of at least
// dense_workspace_bytes (W or the split bf16 pieces); null = the product
// allocates it stream-ordered.
size_t dense_workspace_bytes(int prec, int64_t mr, int64_t mc, int64_t nr, int64_t nc);
void dense_matvec(int prec, const void *M, int64_t mr, int64_t mc, int64_t ldm, const void *N,
                  int64_t nr, int64_t nc, int64_t ldn, const void *V, int64_t ldv, void *U,
                  int64_t ldu, void *ws, hipStream_t s);
// Base kernel matrices from features (linear / Gaussian Gram products on
// matrix cores, Tanimoto by popcount).  Y null: Y = X, exactly symmetric K.
void base_kernel(int kind, int prec, const void *X, int64_t nx, int64_t ldx, const void *Y, int64_t ny,
                 int64_t ldy, int64_t dim, double gamma, void *K, int64_t ldk, hipStream_t s);
void tanimoto_kernel_matrix(int prec, const uint64_t *X, int64_t nx, int64_t ldx, const uint64_t *Y,
                            int64_t ny, int64_t ldy, int64_t nbits, void *K, int64_t ldk, hipStream_t s);
// ||U_S - U_S,ref||_F / ||U_S,ref||_F over up to 16 evenly spaced rows S of
// Umat = M Vmat N^T, with U_S,ref recomputed in FP64 from the stored operands
// (double for GVT_F64, float otherwise).  Synchronises s.
double dense_sample_relerr(int prec, const void *M, int64_t mr, int64_t mc, int64_t ldm, const void *N,
                           int64_t nr, int64_t nc, int64_t ldn, const void *V, int64_t ldv,
                           const void *U, int64_t ldu, hipStream_t s);
// Workspace of gvt_dense_matvec_noalloc: kDenseScratchBytes of static device
// memory per device; the pointer is this device's copy.
constexpr size_t kDenseScratchBytes = (size_t)64 << 20;
void *dense_scratch_ptr();

}  // namespace gvt
