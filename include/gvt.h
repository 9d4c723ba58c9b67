/*
 * gvt.h — C ABI of the MI355X (gfx950) generalized-vec-trick library.
 *
 * The library computes matrix-vector products with pairwise kernel matrices
 * without forming them (Viljanen, Airola, Pahikkala, "Generalized vec trick
 * for fast learning of pairwise kernel models"):
 *
 *   u = R(a, b) K R(c, e)^T v
 *
 * where (a_i, b_i), i < n_out, are the output pairs, (c_j, e_j), j < n_in,
 * the input (training) pairs, R(.,.) the sampling operators of Section 3, and
 * K the operator of a pairwise kernel written as a sum of Kronecker products
 * (Corollary 1).  Each Kronecker term is applied with the generalized vec
 * trick of Theorem 1 in O(min(qbar n + m nbar, mbar n + q nbar)) time.  The
 * library also solves the kernel ridge regression system of Section 3
 * eq. (1), (K + lambda I) a = y, by conjugate gradients on that operator.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller unless a
 *    parameter says "host".  The library never frees them and keeps no
 *    reference after the call returns (plans keep their own copies).
 *  - Matrices are row-major with a leading dimension (elements between row
 *    starts) >= the number of columns.  Base matrices: D is d_rows x d_cols
 *    (rows: output-side drugs, columns: input-side drugs), T is
 *    t_rows x t_cols (same for targets).  Index a_i < d_rows, b_i < t_rows,
 *    c_j < d_cols, e_j < t_cols; all indices are 0-based int32.
 *  - Vectors with several right-hand sides are column-major: V is
 *    n_in x nrhs with column stride ldv >= n_in, U is n_out x nrhs with column
 *    stride ldu >= n_out.
 *  - Element type follows the precision: GVT_F64 uses double for D, T, V, U;
 *    GVT_F32 uses float.  GVT_BF16X3 (bf16 split products with FP32
 *    accumulation on matrix cores) uses float storage and is available on the
 *    matrix-core paths only: complete data, and dense tiles of two-factor
 *    terms (gvt_plan_uses_tiles); a plan's other terms then run in FP32.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and the call returns without synchronising unless stated.
 *  - Threads: calls from several host threads may run at once, on streams of
 *    their own, as long as each plan is used by one stream at a time (a plan
 *    owns the workspaces its products write).  The library's only shared state
 *    is its cache of device blocks and its upload staging buffer, both locked.
 *    Giving a device block back (the end of a solve or of a one-shot product,
 *    gvt_plan_destroy, a plan workspace that grows) waits until the device has
 *    finished the work queued on all its streams, as hipFree does; no lock is
 *    held during that wait, so other threads' calls proceed meanwhile.
 *  - Errors: 0 = success, > 0 = warning (results written), < 0 = error.
 *    gvt_last_error() returns a message for the calling thread's last error.
 *    Error paths never leave kernels running on the stream.
 *  - Results are deterministic: repeated calls with the same inputs give
 *    bitwise identical outputs (no floating-point atomics).
 *  - Launch shapes come from tuned constants compiled into the library.
 *    Environment variables read when a plan is built override them for
 *    tuning sweeps: GVT_STAGE1_SLICE (0/1: stage 1 reads a contiguous row
 *    range's F2 columns from a slice held in LDS where it fits),
 *    GVT_STAGE1_SLICE_WGS (workgroups of such a launch), GVT_STAGE1_WIDE (0/1:
 *    stage 1 holds 16 bytes of consecutive rows per lane over a contiguous row
 *    range), GVT_STAGE1_KPW (1, 2, 4 keys per wave), GVT_STAGE2_TARGET_R1 /
 *    _R8 (stage-2 outputs per group row and tile), GVT_STAGE2_XCD (0/1: stage-2
 *    tiles dealt to the XCDs by S block / by F1 block; unset: by working set),
 *    GVT_STAGE2_DUAL (0/1: stage 2 with one RHS stages both operands of
 *    128 x 128 tiles in LDS; unset: at low output density),
 *    GVT_STAGE2Y_PIPELINED (0/1, default 1: stage 2 of 4-RHS blocks copies
 *    the next key chunk while it walks the current one),
 *    GVT_MAX_RHS_BLOCK[_F64|_F32] (largest RHS block of a pass),
 *    GVT_PLAN_DEVICE (0/1: plan index work on the host / device),
 *    GVT_PLAN_LIBRARY_SORT (1: device plans sort with hipCUB's radix sort
 *    instead of the library's own).  All of them
 *    but the RHS block give the same products bit for bit (the block size
 *    changes which lanes sum which keys); GVT_PLAN_TIMING=1 prints the host
 *    time of each plan phase.
 */
#ifndef GVT_H
#define GVT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GVT_OK 0
#define GVT_NOT_CONVERGED 1     /* CG hit max_iter; results are written      */
#define GVT_TOL_NOT_MET 2       /* estimated error above the requested bound;
                                   results are written                        */
#define GVT_ERR_ARG (-1)        /* null pointer, negative size, ld < cols... */
#define GVT_ERR_INDEX (-2)      /* an index is out of range                  */
#define GVT_ERR_KIND (-3)       /* kind/base-matrix mismatch (homogeneous)   */
#define GVT_ERR_HIP (-4)        /* HIP runtime failure                       */
#define GVT_ERR_NOMEM (-5)      /* device allocation failed                  */
#define GVT_ERR_BREAKDOWN (-6)  /* CG breakdown: p.w <= 0 or non-finite      */
#define GVT_ERR_UNSUPPORTED (-7)/* precision/path combination not provided   */

/* ---- arithmetic -------------------------------------------------------- */
#define GVT_F64 0
#define GVT_F32 1
#define GVT_BF16X3 2
#define GVT_BF16X6 3   /* three-way bf16 split, six products (dense path only) */

/* ---- pairwise kernels (Table 4b / Corollary 1) ------------------------ */
#define GVT_KRONECKER 0     /* D (x) T ; the pairwise Gaussian is this kind on Gaussian bases */
#define GVT_LINEAR 1        /* D (x) 1 + 1 (x) T                                          */
#define GVT_POLY2D 2        /* Q(D(x)D)Q^T + 2 D(x)T + PQ(T(x)T)Q^T P                     */
#define GVT_CARTESIAN 3     /* D (x) I + I (x) T                                          */
#define GVT_SYMMETRIC 4     /* (P + I)(D (x) D)                       homogeneous         */
#define GVT_ANTISYMMETRIC 5 /* (I - P)(D (x) D)  (sign of the Table 4b function) homog.   */
#define GVT_RANKING 6       /* (I - P)(D (x) 1)(I - P)                homogeneous         */
#define GVT_MLPK 7          /* (I + P)(I - Q)(D (x) D)(I - Q)^T (I + P)  homogeneous      */

/* ---- base kernels from features (Section 5) ----------------------------- */
#define GVT_BASE_LINEAR 0   /* k(x, y) = <x, y>                  */
#define GVT_BASE_GAUSSIAN 1 /* k(x, y) = exp(-gamma ||x - y||^2) */

/* ---- losses of the regularized risk (Section 3) ------------------------- */
#define GVT_LOSS_SQUARED 0  /* 1/2 sum (y - p)^2                    */
#define GVT_LOSS_LOGISTIC 1 /* sum log(1 + exp(-y p)), y in {-1, 1}  */
#define GVT_LOSS_SQHINGE 2  /* 1/2 sum max(0, 1 - y p)^2             */
#define GVT_LOSS_HINGE 3    /* sum max(0, 1 - y p) (subgradient)     */

/* ---- plan flags ---------------------------------------------------------- */
#define GVT_FLAG_SYMMETRIC_BASES 1 /* D and T are square and symmetric (training
                                      kernels): the library may read a column as
                                      the equal row instead of transposing      */
#define GVT_FLAG_ORDER_A 2         /* force stage order A (scatter by drug)      */
#define GVT_FLAG_ORDER_B 4         /* force stage order B (scatter by target)    */
#define GVT_FLAG_DENSE_TILES 8     /* single Kronecker term: always run products
                                      as M Vmat N^T on matrix cores (dense tiles) */
#define GVT_FLAG_NO_DENSE_TILES 16 /* never use dense tiles (gather path only)   */

typedef struct gvt_plan *gvt_plan_t;

/*
 * gvt_plan_create — index preprocessing shared by every product over the
 * same pair sets (Theorem 1; Table 1 unique counts).
 *
 * Validates every index, counts unique drugs/targets per sample, chooses the
 * cheaper stage order of Theorem 1 per Kronecker term (ties: order A when
 * d_cols >= t_cols, else B), sorts the input pairs into key segments and
 * groups the output pairs, and expands each kind into its Kronecker terms
 * with common subexpressions shared across the `nkinds` kinds.
 *
 * kinds[nkinds] (host): GVT_* kind codes; one output block per kind.
 * Homogeneous kinds need t_rows == d_rows and t_cols == d_cols (T is
 * ignored; pass the D shape).  Index arrays are device pointers, read once
 * (the call synchronises `stream`; the plan keeps no pointer to them).
 * Index sets of 65536 pairs or more (n_in + n_out) are validated, counted
 * and sorted on the device, smaller ones on the host; both give the same
 * plan (environment GVT_PLAN_DEVICE=0/1 forces either).  *plan receives an
 * opaque handle owned by the caller; release it with gvt_plan_destroy.
 * n_in == 0 or n_out == 0 is valid (products then write zeros / nothing).
 * Errors: GVT_ERR_ARG, GVT_ERR_INDEX, GVT_ERR_KIND, GVT_ERR_HIP, GVT_ERR_NOMEM.
 */
int gvt_plan_create(gvt_plan_t *plan, const int *kinds, int nkinds, int64_t d_rows,
                    int64_t d_cols, int64_t t_rows, int64_t t_cols, const int32_t *out_a,
                    const int32_t *out_b, int64_t n_out, const int32_t *in_c,
                    const int32_t *in_e, int64_t n_in, int flags, void *stream);

/* gvt_plan_destroy — synchronises the plan's last stream and frees its
 * device memory.  NULL is accepted. */
int gvt_plan_destroy(gvt_plan_t plan);

/*
 * gvt_plan_execute — U_k = R(a,b) K_{kinds[k]} R(c,e)^T V for every kind of
 * the plan (Corollary 1: each kind is a sum of Kronecker terms, each term one
 * generalized vec trick, Theorem 1).
 *
 * D (ldd) and T (ldt) must have the shapes given at plan creation (T may be
 * NULL for homogeneous kinds).  V: n_in x nrhs, column stride ldv.  U: the
 * plan's nkinds output blocks stacked, block k at U + k*nrhs*ldu, each
 * n_out x nrhs with column stride ldu.  Asynchronous on `stream`.
 * Right-hand sides run in blocks of 8, 4, 2, 1, capped per precision by
 * tuned limits (FP64 2, FP32 4; environment GVT_MAX_RHS_BLOCK[_F64|_F32],
 * read at plan creation); blocks of 1-2 and of 4-8 use stage-2 tiles of their
 * own.  The plan holds those for one RHS (gvt_plan_create); the first
 * product with a block of the other kind builds that set (device or host
 * work, and allocation), so that first call must not be captured into a
 * graph (GVT_ERR_ARG if it is).
 * Errors: GVT_ERR_ARG, GVT_ERR_UNSUPPORTED (a split-bf16 precision for a plan
 * whose two-factor terms cannot run as dense tiles, or that has none),
 * GVT_ERR_HIP, GVT_ERR_NOMEM.
 */
int gvt_plan_execute(gvt_plan_t plan, int prec, const void *D, int64_t ldd, const void *T,
                     int64_t ldt, const void *V, int64_t nrhs, int64_t ldv, void *U,
                     int64_t ldu, void *stream);

/*
 * gvt_matvec — one generalized vec trick product (Theorem 1):
 *   U = R(a, b) (M (x) N) R(c, e)^T V
 * M: m_rows x m_cols (rows: output drugs, cols: input drugs), N: n_rows x
 * n_cols.  Plans internally and synchronises `stream` before returning.
 * When the input and output pairs are each the complete grid in natural
 * order (pair (d, t) at index d*cols + t, Section 4 Example), the product is
 * the dense contraction Umat = M Vmat N^T and runs on matrix cores.
 * Errors as gvt_plan_create / gvt_plan_execute.
 */
int gvt_matvec(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm,
               const void *N, int64_t n_rows, int64_t n_cols, int64_t ldn,
               const int32_t *out_a, const int32_t *out_b, int64_t n_out, const int32_t *in_c,
               const int32_t *in_e, int64_t n_in, const void *V, int64_t nrhs, int64_t ldv,
               void *U, int64_t ldu, void *stream);

/*
 * gvt_pairwise_matvec — U_k = R(a,b) K_{kinds[k]}(D, T) R(c,e)^T V for
 * nkinds kinds in one planned, fused pass (Corollary 1; shared stage-1
 * scatters and one-factor products across kinds).  Output blocks as in
 * gvt_plan_execute.  `flags` as in gvt_plan_create.  Plans internally and
 * synchronises `stream` before returning.
 */
int gvt_pairwise_matvec(int prec, const int *kinds, int nkinds, const void *D, int64_t d_rows,
                        int64_t d_cols, int64_t ldd, const void *T, int64_t t_rows,
                        int64_t t_cols, int64_t ldt, const int32_t *out_a, const int32_t *out_b,
                        int64_t n_out, const int32_t *in_c, const int32_t *in_e, int64_t n_in,
                        const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu,
                        int flags, void *stream);

/*
 * gvt_dense_matvec — the complete-data case of the Kronecker product.  With
 * every pair of the grid present in natural order (pair (d, t) at index
 * d*cols + t, the ordering of the Section 4 Example), R(.,.) are identities
 * and (M (x) N) vec(Vmat) = vec(M Vmat N^T) (row-major vec).
 * M: m_rows x m_cols (ldm), N: n_rows x n_cols (ldn), Vmat: m_cols x n_cols
 * (ldv), Umat: m_rows x n_rows (ldu), all row-major.  Two matrix-core GEMMs,
 * W = M Vmat and Umat = W N^T; W is stream-ordered library workspace.
 * prec: GVT_F64 (FP64 MFMA), GVT_F32 (FP32 MFMA) or GVT_BF16X3 (float
 * storage; each operand split x = hi + lo into bf16 with round-to-nearest-
 * even, products hi*hi' + hi*lo' + lo*hi' on bf16 MFMA with FP32
 * accumulation; W is split again for the second GEMM).  Asynchronous.
 */
int gvt_dense_matvec(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm,
                     const void *N, int64_t n_rows, int64_t n_cols, int64_t ldn, const void *V,
                     int64_t ldv, void *U, int64_t ldu, void *stream);

/*
 * gvt_dense_matvec_checked — gvt_dense_matvec with the error of the result
 * measured and bounded (the complete-data product of Section 3's vec-trick
 * identity, as gvt_dense_matvec).  After the product it recomputes up to 16
 * evenly spaced rows of Umat in FP64 from the same stored operands and
 * estimates the norm-wise relative error ||U_S - U_S,ref|| / ||U_S,ref||
 * over those rows.  While the estimate exceeds max_relerr / 2 the product is
 * redone in the next more accurate form (GVT_BF16X3 -> GVT_BF16X6 ->
 * GVT_F32; inputs stay float); GVT_F64 and GVT_F32 are only measured.  The
 * split-bf16 forms keep ~16 (bf16x3) or ~24 (bf16x6) significant bits per
 * operand, so their error relative to |Umat| grows with cancellation in the
 * sums, which the inputs decide.  max_relerr = 0 measures without escalating.
 * *relerr_out (host) receives the estimate for the returned result,
 * *prec_out (host) the precision that produced it.  Synchronises `stream`.
 * Returns GVT_OK, GVT_TOL_NOT_MET when the last estimate still exceeds
 * max_relerr (results written), or the errors of gvt_dense_matvec.
 */
int gvt_dense_matvec_checked(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm,
                             const void *N, int64_t n_rows, int64_t n_cols, int64_t ldn,
                             const void *V, int64_t ldv, void *U, int64_t ldu, double max_relerr,
                             double *relerr_out, int *prec_out, void *stream);

/*
 * gvt_dense_matvec_noalloc — gvt_dense_matvec for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and precisions
 * as gvt_dense_matvec; the intermediate W (or the split bf16 pieces) lives in
 * a static per-device workspace of 64 MiB (GVT_DENSE_NOALLOC_BYTES) that
 * each device using the library holds until the process ends.  The call
 * makes no hipMalloc/hipFree and no allocating library call.  Products whose
 * workspace exceeds the limit return GVT_ERR_ARG with the sizes in
 * gvt_last_error(): W needs m_rows x n_cols elements (8 bytes for GVT_F64,
 * 4 for GVT_F32); the split forms need 2 (GVT_BF16X3) or 3 (GVT_BF16X6)
 * bf16 copies of M, N, Vmat and W with k padded to 64 (32).  Every call on a
 * device uses the same workspace: calls that overlap on one device (two
 * streams, two threads) race and must be serialised by the caller.
 * Asynchronous on `stream`.
 */
#define GVT_DENSE_NOALLOC_BYTES ((int64_t)64 << 20)
int gvt_dense_matvec_noalloc(int prec, const void *M, int64_t m_rows, int64_t m_cols, int64_t ldm,
                             const void *N, int64_t n_rows, int64_t n_cols, int64_t ldn,
                             const void *V, int64_t ldv, void *U, int64_t ldu, void *stream);

/*
 * gvt_base_kernel — a base kernel matrix from object features (Section 5:
 * linear kernels <x, y> and Gaussian kernels exp(-gamma ||x - y||^2) on
 * feature or similarity-row vectors, the drug and target kernels D and T of
 * the pairwise kernels).
 * kind: GVT_BASE_LINEAR or GVT_BASE_GAUSSIAN.  prec: GVT_F64 (double X, Y, K;
 * FP64 matrix cores) or GVT_F32 (float).  X: nx x dim (row stride ldx >= dim),
 * Y: ny x dim (ldy) or NULL for Y = X (then ny must equal nx and K is exactly
 * symmetric with, for the Gaussian, exactly 1 on the diagonal).  K: nx x ny,
 * row stride ldk >= ny, K[i*ldk + j] = k(X_i, Y_j).  The Gaussian uses
 * ||x||^2 + ||y||^2 - 2<x, y> clamped at 0.  Stream-ordered scratch for the
 * row norms; asynchronous on `stream`.  Errors: GVT_ERR_ARG, GVT_ERR_HIP.
 */
int gvt_base_kernel(int kind, int prec, const void *X, int64_t nx, int64_t ldx, const void *Y,
                    int64_t ny, int64_t ldy, int64_t dim, double gamma, void *K, int64_t ldk,
                    void *stream);

/*
 * gvt_tanimoto_kernel — the Tanimoto kernel of binary feature vectors
 * (Section 5, Heterodimer data): bits set in both over bits set in either,
 * 1 for two all-zero vectors.  X: nx rows of packed bits, ldx >= (nbits + 63)
 * / 64 uint64 words per row; bit b of a row is bit b % 64 of word b / 64;
 * bits at and past nbits are ignored.  Y: ny rows (ldy) or NULL for Y = X
 * (ny must equal nx).  K: nx x ny, double (GVT_F64) or float (GVT_F32, the
 * double ratio rounded once), row stride ldk >= ny.  Counts are exact, so K
 * is reproducible bit for bit.  Asynchronous on `stream`.
 * Errors: GVT_ERR_ARG, GVT_ERR_HIP.
 */
int gvt_tanimoto_kernel(int prec, const uint64_t *X, int64_t nx, int64_t ldx, const uint64_t *Y,
                        int64_t ny, int64_t ldy, int64_t nbits, void *K, int64_t ldk, void *stream);

/*
 * gvt_krr_cg — kernel ridge regression, Section 3 eq. (1):
 *   (R K R^T + lambda_l I) a_l = y   for l < nlam (one shared operator,
 *   nlam right-hand sides advanced together as one batched product)
 * by conjugate gradients with FP64 vectors, inner products and step lengths
 * (the paper solves the same SPD system with MINRES and early stopping).
 *
 * kind: any GVT_* kind.  D (d x d, ldd) and T (t x t, ldt) are double,
 * square and symmetric (training kernels; T ignored for homogeneous kinds).
 * c, e: the n training pairs (device).  y: n labels (device, double).
 * lambdas[nlam] (host) > 0.  A: n x nlam solutions (device, double, column
 * stride lda >= n).  A0: optional initial guess with the same layout
 * (stride lda0), NULL = zero.  matvec_prec: GVT_F64 or GVT_F32 (products in
 * FP32, everything else FP64).  With FP32 products a system whose recurrence
 * residual meets `tol` is certified by its true residual from an FP64
 * product; if that fails, the solve continues with FP64 products from the
 * true residual.  A system still above `tol` after max_iter iterations is
 * certified the same way and, if it fails, gets at most max_iter / 10 more
 * iterations with FP64 products (the residual replaced by the true one, the
 * search continuing along its last direction), so that FP32 products lose no
 * system that FP64 products converge; iters_out counts those too.  check_every: iterations between host
 * convergence checks (>= 1); on a non-null stream each such block of
 * iterations after the first is captured once into a HIP graph and replayed,
 * on the null stream it is launched kernel by kernel (bitwise the same
 * results either way).  iters_out[nlam] and relres_out[nlam] (host)
 * receive the iteration counts and the TRUE relative residuals
 * ||y - (K + lambda I) a|| / ||y|| computed with an FP64 product.
 * Synchronises `stream`.  Returns GVT_OK when every system met `tol`,
 * GVT_NOT_CONVERGED when some reached max_iter, GVT_ERR_BREAKDOWN on
 * p.w <= 0 or a non-finite value, other errors as above.
 */
int gvt_krr_cg(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
               int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
               const double *lambdas, int nlam, double *A, int64_t lda, const double *A0,
               int64_t lda0, int max_iter, double tol, int matvec_prec, int check_every,
               int64_t *iters_out, double *relres_out, void *stream);

/*
 * One ridge problem of a batch (all pointers DEVICE, double, as in
 * gvt_krr_cg): base kernels D (d x d, ldd) and T (t x t, ldt; ignored for
 * homogeneous kinds), the n training pairs c, e, labels y[n], solutions A
 * (n x nlam, column stride lda >= n) and an optional initial guess A0 (same
 * layout, stride lda0; NULL = zero).
 */
typedef struct gvt_krr_problem {
  const double *D;
  int64_t d, ldd;
  const double *T;
  int64_t t, ldt;
  const int32_t *c, *e;
  int64_t n;
  const double *y;
  double *A;
  int64_t lda;
  const double *A0;
  int64_t lda0;
} gvt_krr_problem;

/*
 * gvt_krr_cg_batched — many independent kernel ridge problems (Section 3
 * eq. (1), each with its own base kernels, pairs and labels), every one
 * solved for the same grid lambdas[nlam] (host), all advanced together:
 * one set of CG vectors holds the nprob x nlam systems, the products of all
 * problems run as grouped launches (one launch per stage of the generalized
 * vec trick covers every problem), finished problems drop out of the
 * launches, and blocks of check_every iterations replay from one HIP graph.
 * kind, max_iter, tol, matvec_prec and check_every as in gvt_krr_cg; with
 * FP32 products, a problem one of whose systems fails its FP64 certification
 * (or reaches max_iter and gets the FP64 finish) runs FP64 products from then
 * on, the others keep FP32 products.
 * problems[nprob] (host array of descriptors).  iters_out and relres_out
 * (host, nprob x nlam, problem-major: [p * nlam + l]) receive iteration
 * counts and true relative residuals (FP64 products).  Synchronises
 * `stream`.  Returns GVT_OK when every system met tol, GVT_NOT_CONVERGED
 * when some hit max_iter, GVT_ERR_BREAKDOWN on breakdown, and the errors of
 * gvt_krr_cg, with the problem's index in the message.
 */
int gvt_krr_cg_batched(int kind, const gvt_krr_problem *problems, int nprob, const double *lambdas,
                       int nlam, int max_iter, double tol, int matvec_prec, int check_every,
                       int64_t *iters_out, double *relres_out, void *stream);

/*
 * A validation sample for early stopping (all pointers DEVICE): the pairs
 * (a[i], b[i]), i < n, index the rows of the training base kernels (as output
 * pairs of a product with the training pairs as inputs); labels[n] (double)
 * are binary, > 0.5 meaning positive.  patience > 0 stops a system after that
 * many iterations without a better validation AUC; 0 never stops early.
 */
typedef struct gvt_validation {
  const int32_t *a, *b;
  int64_t n;
  const double *labels;
  int64_t patience;
} gvt_validation;

/*
 * gvt_krr_minres — kernel ridge regression, Section 3 eq. (1),
 * (R K R^T + lambda_l I) a_l = y for l < nlam, by the minimal residual method
 * from a = 0, optionally with early stopping on a validation sample (the
 * paper's training procedure, Sections 3 and 6).
 *
 * All lambdas share one Lanczos basis of K (the Krylov spaces of K + lambda I
 * from y do not depend on lambda), so an iteration costs one product with one
 * right-hand side (plus one with the validation pairs as outputs) for the
 * whole grid.  Vectors and scalars are FP64; matvec_prec GVT_F64 or GVT_F32
 * selects the products' arithmetic.  lambdas[nlam] (host) >= 0.
 * Arguments D, T, c, e, n, y as in gvt_krr_cg.
 *
 * Without a validation sample (val NULL or val->n == 0) a system stops when
 * its MINRES residual estimate |phibar_k| / ||y|| < tol (tol 0: never) or
 * after max_iter iterations, and A (n x nlam, column stride lda, device)
 * receives the last iterate.  With one, after every iteration the
 * predictions on the validation pairs give an AUC per system (pairs of
 * positives and negatives ordered correctly, ties one half); A receives the
 * iterate of the best AUC (strictly above every earlier one, from a_0 = 0
 * with AUC 1/2), and a system also stops after val->patience iterations
 * without improvement.
 * Host outputs: iters_out[nlam] iterations run, relres_out[nlam] true
 * relative residual ||y - (K + lambda I) a|| / ||y|| of the returned A (FP64
 * product), best_iter_out[nlam] the iteration of the returned A and
 * best_auc_out[nlam] its AUC (NaN without validation) (both may be NULL),
 * auc_hist[max_iter * nlam] (may be NULL) the AUC after iteration k+1 at
 * [k * nlam + l], NaN past a system's last iteration.  check_every:
 * iterations between host looks at the states.  Synchronises `stream`.
 * Returns GVT_OK when every system met tol or stopped early,
 * GVT_NOT_CONVERGED when some ran to max_iter, GVT_ERR_BREAKDOWN on a
 * non-finite value or a zero Givens norm, other errors as gvt_krr_cg.
 */
int gvt_krr_minres(int kind, const double *D, int64_t d, int64_t ldd, const double *T, int64_t t,
                   int64_t ldt, const int32_t *c, const int32_t *e, int64_t n, const double *y,
                   const double *lambdas, int nlam, double *A, int64_t lda, int max_iter, double tol,
                   int matvec_prec, const gvt_validation *val, int check_every, int64_t *iters_out,
                   double *relres_out, int64_t *best_iter_out, double *best_auc_out,
                   double *auc_hist, void *stream);

/*
 * gvt_erm_objective — the regularized risk of Section 3 in dual coefficients
 * and its (sub)gradient, for the losses GVT_LOSS_*:
 *   J(a) = L(K a, y) + (lambda / 2) a^T K a,   grad J = K (g + lambda a),
 * g = dL/dp at p = K a (the hinge loss: the subgradient -y [y p < 1]).  K is
 * the training kernel matrix of `kind` on the pairs (c, e) (D, T, c, e, n, y
 * as in gvt_krr_cg; classification losses take y in {-1, +1}).  a: n
 * coefficients (device, double).  grad: n (device, double) or NULL.
 * *obj_out (host) receives J(a).  Two products (one without grad).
 * Synchronises `stream`.  Errors: GVT_ERR_ARG, GVT_ERR_BREAKDOWN (non-finite
 * J), GVT_ERR_HIP, GVT_ERR_NOMEM.
 */
int gvt_erm_objective(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T,
                      int64_t t, int64_t ldt, const int32_t *c, const int32_t *e, int64_t n,
                      const double *y, const double *a, double lambda, double *grad, double *obj_out,
                      void *stream);

/*
 * gvt_erm_newton — minimises J (gvt_erm_objective) from a = 0 by truncated
 * Newton, the optimiser Section 3 names for losses other than the squared
 * one (kernel logistic regression, L2-SVM).  Each step solves
 * K (D K + lambda I) delta = -grad J by conjugate gradients with Hessian
 * products K (d * (K v) + lambda v), D = diag(d), d = d^2L/dp^2, stopped after
 * max_cg iterations or once the CG residual is below
 * min(1/2, sqrt(||grad|| / ||grad_0||)) ||grad||; then backtracks t = 1, 1/2,
 * ... (at most 30 halvings) until J(a + t delta) <= J(a) + 1e-4 t grad.delta.
 * Stops when ||grad J|| <= tol ||grad J(0)|| or after max_newton steps.
 * loss: GVT_LOSS_SQUARED, _LOGISTIC or _SQHINGE (the hinge: GVT_ERR_UNSUPPORTED).
 * lambda >= 0.  A: n coefficients out (device, double).  matvec_prec: GVT_F64
 * or GVT_F32 products (vectors and scalars FP64).  Host outputs (may be NULL):
 * Newton steps, total CG iterations, J and ||grad J|| at A, ||grad J(0)||.
 * Synchronises `stream`.  Returns GVT_OK when the gradient test was met,
 * GVT_NOT_CONVERGED after max_newton steps, GVT_ERR_BREAKDOWN on a
 * non-finite value.
 */
int gvt_erm_newton(int kind, int loss, const double *D, int64_t d, int64_t ldd, const double *T,
                   int64_t t, int64_t ldt, const int32_t *c, const int32_t *e, int64_t n,
                   const double *y, double lambda, double *A, int max_newton, int max_cg, double tol,
                   int matvec_prec, int *steps_out, int *cg_iters_out, double *obj_out,
                   double *gnorm_out, double *gnorm0_out, void *stream);

/*
 * gvt_plan_profile — diagnostic: runs gvt_plan_execute `reps` times
 * (synchronising `stream` after each) with HIP events recorded at the stage
 * boundaries of the generalized vec trick, and writes the mean milliseconds
 * of each stage group to stage_ms[4] (host): [0] input gather + segment sums
 * + one-factor GEMVs, [1] stage 1 (scatters into S), [2] stage 2 (gather-dot
 * of every two-factor term), [3] match terms, gathers and the per-kind
 * combination.  Stage 2's launches run 8 times back to back within their
 * events and [2] is the mean per product, free of the events' own overhead
 * (every stage-2 kernel overwrites its outputs, so U is the product).
 * nrhs <= 8.  Gather path only (GVT_ERR_UNSUPPORTED for a complete-data
 * plan).
 */
int gvt_plan_profile(gvt_plan_t plan, int prec, const void *D, int64_t ldd, const void *T,
                     int64_t ldt, const void *V, int64_t nrhs, int64_t ldv, void *U, int64_t ldu,
                     int reps, double *stage_ms, void *stream);

/*
 * gvt_plan_info — diagnostic: info[11] (host) receives the Theorem 1 FMA count
 * of the plan's term program per right-hand side, whether it is a
 * complete-data plan, the numbers of distinct terms and stage-1 buffers, the
 * first buffer's row and key counts (rows: those stage 1 computes, which may
 * close small gaps in the rows the terms read) and key index (2 = drug, 3 =
 * target, -1 = none), and the unique counts of a, b, c, e (Table 1).
 */
int gvt_plan_info(gvt_plan_t plan, double *info);

/*
 * gvt_plan_uses_tiles — diagnostic: 1 when products of the plan in precision
 * prec run as dense tiles (a Kronecker term computed as M Vmat N^T on matrix
 * cores, Vmat the zero grid with the input vector scattered into it, the
 * outputs gathered from the result): for a single Kronecker term the whole
 * product; for several kinds or terms every two-factor term (Corollary 1's
 * terms of the form R(D (x) T)R^T keyed by the input pair (c, e); terms with
 * equal base matrices share one dense product, each gathering its own output
 * order), with the one-factor and match terms and the per-kind sums on the
 * gather path, which is possible when no two-factor term is keyed by (c, c)
 * or (e, e) (MLPK has such terms).  Taken always with GVT_FLAG_DENSE_TILES or
 * environment GVT_DENSE_TILES=1 at plan creation and for the split-bf16
 * precisions; never with GVT_FLAG_NO_DENSE_TILES or GVT_DENSE_TILES=0;
 * otherwise when the tuned cost model estimates the dense products faster
 * than the gather path.  0 when the gather path runs, GVT_ERR_ARG for a null
 * plan.
 */
int gvt_plan_uses_tiles(gvt_plan_t plan, int prec);

/*
 * gvt_empty_cache — releases the memory the library keeps for reuse.  Device
 * blocks that plans, products and solves give back are kept in a per-device
 * cache (at most 4 GiB per device, reused by later requests of up to twice
 * their size) instead of being freed, and plan uploads go through one pinned
 * host staging buffer.  This frees every cached block on every device and the
 * staging buffer; blocks held by live plans or running calls are not touched,
 * and later calls allocate again.  *freed_bytes (host, may be NULL) receives
 * the device bytes freed.  For callers that share the GPU with another
 * allocator (a framework's own cache) or want memory back between phases.
 * Thread-safe; returns GVT_OK, or GVT_ERR_HIP if selecting a device fails.
 */
int gvt_empty_cache(int64_t *freed_bytes);

/* Message describing the calling thread's most recent error ("" if none). */
const char *gvt_last_error(void);

/* Library version: major*10000 + minor*100 + patch. */
int gvt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GVT_H */
