// Launcher declarations for the library's kernels (internal).
#pragma once

#include "common.h"

namespace gvt {

constexpr int kMaxCombineTerms = 16;
// Stage-2 tiles: kStage2Rows consecutive F1 rows x at most kStage2MaxS S rows.
constexpr int kStage2Rows = 32;
constexpr int kStage2MaxS = 64;
constexpr int kMaxCombineOut = 8;

template <class T> struct CombineArgs {
  int nterms = 0;
  int nout = 0;
  const T *t[kMaxCombineTerms] = {};
  T coef[kMaxCombineOut][kMaxCombineTerms] = {};
};

template <class T>
void launch_pack_v(const T *V, int64_t ldv, const int32_t *perm, int64_t n, int R, T *vs,
                   hipStream_t s);
template <class T>
void launch_segsum(const int64_t *seg, const T *vs, int64_t nkeys, int R, T *out, hipStream_t s);
template <class T>
void launch_stage1(const T *Fc, int64_t ldc, const int32_t *rows, int64_t nrows, const int64_t *seg,
                   const int32_t *other, const T *vs, int64_t nkeys, int R, T *S, int64_t ldS,
                   hipStream_t s);
template <class T>
void launch_colscale(const T *F, int64_t ldf, const int32_t *rows, int64_t nrows, const T *sv,
                     int64_t nkeys, int R, T *S, int64_t ldS, hipStream_t s);
template <class T>
void launch_stage2(const T *F1, int64_t ld1, int64_t nx, const int64_t *tileoff, const int32_t *tiley,
                   const int32_t *tilemax, int64_t ntiles, int nyb, const int32_t *yrows,
                   const int32_t *perm, const T *S, int64_t ldS, int64_t nkeys, int R, T coef, T *out,
                   int64_t ldi, int64_t ldr, hipStream_t s);
template <class T>
void launch_gemv(const T *F, int64_t ldf, int64_t nrows, int64_t ncols, bool sq, const T *sv, int R,
                 T *g, hipStream_t s);
template <class T>
void launch_gather_rows(const T *g, const int32_t *sel, int64_t n, int R, T *t, hipStream_t s);
template <class T>
void launch_match(const T *F, int64_t ldf, const int32_t *xsel, const int32_t *ksel, int64_t n,
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

// Dense complete-data path (matrix cores).
void dense_matvec(int prec, const void *M, int64_t mr, int64_t mc, int64_t ldm, const void *N,
                  int64_t nr, int64_t nc, int64_t ldn, const void *V, int64_t ldv, void *U,
                  int64_t ldu, hipStream_t s);

}  // namespace gvt
