/*
 * Plain FP64 CPU oracle for pairwise-kernel matrix-vector products and the
 * kernel-ridge-regression solve that uses them.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library and must never sit on the
 * product path.
 *
 * What it computes (Viljanen, Airola, Pahikkala, "Generalized vec trick for
 * fast learning of pairwise kernel models"):
 *
 *   u[i] = sum_{j=0}^{n-1} k((a_i, b_i), (c_j, e_j)) * v[j]
 *
 * i.e. row i of the two-sample kernel matrix R(a,b) K R(c,e)^T times v
 * (Section 3, the kernel matrix entries K_ij = k(x_i, x_j) and the prediction
 * product with a second sample; Section 4 "Efficient computation of pairwise
 * kernels", approach 1: the standard matrix-vector product).  k is the
 * pairwise kernel FUNCTION of Table 4b, evaluated by look-ups into the base
 * kernel matrices D (drug kernel) and T (target kernel).  The Corollary 1
 * sum-of-Kronecker decomposition is deliberately not used here, so agreement
 * with a GVT implementation also checks that decomposition.
 *
 * Readings of the paper used here:
 *  - Anti-symmetric: the Table 4b function k(d,db)k(d',db') - k(d,db')k(d',db)
 *    (its feature map in Table 4a agrees; the operator printed in Corollary 1
 *    has the opposite overall sign).
 *  - Symmetric: the Table 4b function with no factor 1/2.
 *  - Cartesian: delta(t = tb) compares object identities; a row index and a
 *    column index of a base matrix denote the same object iff they are equal.
 *  - Homogeneous kinds (symmetric, anti-symmetric, ranking, MLPK) use only D:
 *    output pairs index its rows, input pairs index its columns.
 *
 * Summation: for each output row the sum over j runs sequentially in
 * ascending j starting from 0.0; products are formed left to right as the
 * table writes them.  Built with -O2 -ffp-contract=off (no FMA contraction),
 * so the result is exactly specified and independent of the thread count
 * (OpenMP splits output rows statically).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Kind codes of this oracle (private to the oracle). */
enum {
    OK_KRONECKER = 0,
    OK_LINEAR = 1,
    OK_POLY2D = 2,
    OK_CARTESIAN = 3,
    OK_SYMMETRIC = 4,
    OK_ANTISYMMETRIC = 5,
    OK_RANKING = 6,
    OK_MLPK = 7
};

typedef struct {
    const double *D;
    int64_t ldd;
    const double *T;
    int64_t ldt;
} bases_t;

#define DV(i, j) (B->D[(int64_t)(i) * B->ldd + (int64_t)(j)])
#define TV(i, j) (B->T[(int64_t)(i) * B->ldt + (int64_t)(j)])

/* Table 4b: the pairwise kernel function k((a,b),(c,e)).
 * (a,b) = (d, t) or (d, d') is the output-side pair, (c,e) = (db, tb) or
 * (db, db') is the input-side pair. */
static double pair_kernel(int kind, const bases_t *B, int32_t a, int32_t b,
                          int32_t c, int32_t e)
{
    switch (kind) {
    case OK_KRONECKER: /* k_D(d,db) k_T(t,tb) */
        return DV(a, c) * TV(b, e);
    case OK_LINEAR: /* k_D(d,db) + k_T(t,tb) */
        return DV(a, c) + TV(b, e);
    case OK_POLY2D: { /* (k_D(d,db) + k_T(t,tb))^2 */
        double s = DV(a, c) + TV(b, e);
        return s * s;
    }
    case OK_CARTESIAN: { /* k_D(d,db) delta(t=tb) + delta(d=db) k_T(t,tb) */
        double x = 0.0;
        if (b == e) x = x + DV(a, c);
        if (a == c) x = x + TV(b, e);
        return x;
    }
    case OK_SYMMETRIC: /* k(d,db)k(d',db') + k(d,db')k(d',db) */
        return DV(a, c) * DV(b, e) + DV(a, e) * DV(b, c);
    case OK_ANTISYMMETRIC: /* k(d,db)k(d',db') - k(d,db')k(d',db) */
        return DV(a, c) * DV(b, e) - DV(a, e) * DV(b, c);
    case OK_RANKING: /* k(d,db) - k(d,db') - k(d',db) + k(d',db') */
        return DV(a, c) - DV(a, e) - DV(b, c) + DV(b, e);
    case OK_MLPK: { /* (k(d,db) - k(d,db') - k(d',db) + k(d',db'))^2 */
        double r = DV(a, c) - DV(a, e) - DV(b, c) + DV(b, e);
        return r * r;
    }
    default:
        return NAN;
    }
}

static int kind_valid(int kind) { return kind >= OK_KRONECKER && kind <= OK_MLPK; }
static int kind_homogeneous(int kind)
{
    return kind == OK_SYMMETRIC || kind == OK_ANTISYMMETRIC || kind == OK_RANKING ||
           kind == OK_MLPK;
}

/*
 * u[r][s] (u + s*ldu + r) = sum_j k(out_sel[r], in_j) * v[j + s*ldv]
 *
 * rows:     optional list of output-pair indices to evaluate (row-sampled
 *           mode); NULL means all nout output pairs, u then has nout rows.
 * v, u:     column-major, nrhs columns, leading dimensions ldv >= nin,
 *           ldu >= number of evaluated rows.
 * Returns 0 on success, -1 on a bad argument or out-of-range index.
 */
int oracle_pairwise_matvec(int kind, const double *D, int64_t d_rows, int64_t d_cols,
                           int64_t ldd, const double *T, int64_t t_rows, int64_t t_cols,
                           int64_t ldt, const int32_t *a, const int32_t *b, int64_t nout,
                           const int64_t *rows, int64_t nrows, const int32_t *c,
                           const int32_t *e, int64_t nin, const double *v, int64_t nrhs,
                           int64_t ldv, double *u, int64_t ldu, int nthreads)
{
    if (!kind_valid(kind) || nrhs < 1 || nin < 0 || nout < 0) return -1;
    if (kind_homogeneous(kind)) {
        T = D;
        t_rows = d_rows;
        t_cols = d_cols;
        ldt = ldd;
    }
    if (!D || !T) return -1;
    int64_t nev = rows ? nrows : nout;
    if (ldv < nin || ldu < nev) return -1;
    /* index validation */
    for (int64_t j = 0; j < nin; ++j) {
        int64_t cmax = d_cols, emax = kind_homogeneous(kind) ? d_cols : t_cols;
        if (c[j] < 0 || c[j] >= cmax || e[j] < 0 || e[j] >= emax) return -1;
    }
    for (int64_t r = 0; r < nev; ++r) {
        int64_t i = rows ? rows[r] : r;
        if (i < 0 || i >= nout) return -1;
        int64_t bmax = kind_homogeneous(kind) ? d_rows : t_rows;
        if (a[i] < 0 || a[i] >= d_rows || b[i] < 0 || b[i] >= bmax) return -1;
    }
    bases_t B = {D, ldd, T, ldt};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)nrhs);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < nev; ++r) {
            int64_t i = rows ? rows[r] : r;
            for (int64_t s = 0; s < nrhs; ++s) acc[s] = 0.0;
            for (int64_t j = 0; j < nin; ++j) {
                double kv = pair_kernel(kind, &B, a[i], b[i], c[j], e[j]);
                for (int64_t s = 0; s < nrhs; ++s) acc[s] = acc[s] + kv * v[j + s * ldv];
            }
            for (int64_t s = 0; s < nrhs; ++s) u[r + s * ldu] = acc[s];
        }
        free(acc);
    }
    return 0;
}

/* Kernel matrix entries (for tiny explicit checks): K[i*nin + j] = k(out_i, in_j). */
int oracle_kernel_matrix(int kind, const double *D, int64_t d_rows, int64_t d_cols,
                         int64_t ldd, const double *T, int64_t t_rows, int64_t t_cols,
                         int64_t ldt, const int32_t *a, const int32_t *b, int64_t nout,
                         const int32_t *c, const int32_t *e, int64_t nin, double *K)
{
    (void)t_rows;
    (void)t_cols;
    (void)d_rows;
    (void)d_cols;
    if (!kind_valid(kind)) return -1;
    if (kind_homogeneous(kind)) {
        T = D;
        ldt = ldd;
    }
    bases_t B = {D, ldd, T, ldt};
    for (int64_t i = 0; i < nout; ++i)
        for (int64_t j = 0; j < nin; ++j)
            K[i * nin + j] = pair_kernel(kind, &B, a[i], b[i], c[j], e[j]);
    return 0;
}

static double dot_seq(const double *x, const double *y, int64_t n)
{
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s = s + x[k] * y[k];
    return s;
}

/*
 * Kernel ridge regression, Section 3 eq. (1): solve (K + lambda I) a = y with
 * K = R (pairwise operator) R^T over the training pairs, by textbook
 * conjugate gradients (Hestenes-Stiefel) in FP64.  The paper uses MINRES with
 * early stopping; K + lambda I is symmetric positive definite for lambda > 0,
 * so both iterate towards the same solution.
 *
 *   a0 = 0, r0 = y, p0 = r0, rho0 = r0.r0
 *   repeat: w = K p + lambda p; alpha = rho / (p.w); a += alpha p;
 *           r -= alpha w; rho' = r.r; stop if sqrt(rho')/||y|| < tol;
 *           p = r + (rho'/rho) p
 *
 * One solve per lambda (nlam of them, each column of A).  On return
 * iters[l] = iterations taken, relres_rec[l] = recurrence residual and
 * relres_true[l] = ||y - (K + lambda I) a|| / ||y|| from one more matvec.
 * Returns 0, or -1 on bad arguments, -2 on breakdown (p.w <= 0 or NaN).
 */
int oracle_krr_cg(int kind, const double *D, int64_t d_rows, int64_t d_cols, int64_t ldd,
                  const double *T, int64_t t_rows, int64_t t_cols, int64_t ldt,
                  const int32_t *c, const int32_t *e, int64_t n, const double *y,
                  const double *lambdas, int64_t nlam, int64_t max_iter, double tol,
                  double *A, int64_t lda, int64_t *iters, double *relres_rec,
                  double *relres_true, int nthreads)
{
    if (n <= 0 || nlam <= 0 || lda < n) return -1;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    int status = 0;
    double ynorm = sqrt(dot_seq(y, y, n));
    for (int64_t l = 0; l < nlam && status == 0; ++l) {
        double lam = lambdas[l];
        double *a = A + l * lda;
        for (int64_t k = 0; k < n; ++k) {
            a[k] = 0.0;
            r[k] = y[k];
            p[k] = y[k];
        }
        double rho = dot_seq(r, r, n);
        int64_t it = 0;
        double rel = sqrt(rho) / ynorm;
        while (it < max_iter && !(rel < tol)) {
            if (oracle_pairwise_matvec(kind, D, d_rows, d_cols, ldd, T, t_rows, t_cols, ldt, c,
                                       e, n, NULL, 0, c, e, n, p, 1, n, w, n, nthreads) != 0) {
                status = -1;
                break;
            }
            for (int64_t k = 0; k < n; ++k) w[k] = w[k] + lam * p[k];
            double pw = dot_seq(p, w, n);
            if (!(pw > 0.0)) {
                status = -2;
                break;
            }
            double alpha = rho / pw;
            for (int64_t k = 0; k < n; ++k) a[k] = a[k] + alpha * p[k];
            for (int64_t k = 0; k < n; ++k) r[k] = r[k] - alpha * w[k];
            double rho_new = dot_seq(r, r, n);
            ++it;
            rel = sqrt(rho_new) / ynorm;
            if (rel < tol) break;
            double beta = rho_new / rho;
            for (int64_t k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
            rho = rho_new;
        }
        iters[l] = it;
        relres_rec[l] = rel;
        /* true residual from one more matvec */
        if (status == 0) {
            oracle_pairwise_matvec(kind, D, d_rows, d_cols, ldd, T, t_rows, t_cols, ldt, c, e, n,
                                   NULL, 0, c, e, n, a, 1, n, w, n, nthreads);
            double s = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                double d = y[k] - (w[k] + lam * a[k]);
                s = s + d * d;
            }
            relres_true[l] = sqrt(s) / ynorm;
        }
    }
    free(r);
    free(p);
    free(w);
    return status;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Base kernels from object features (Section 5: the drug and target kernels
 * the pairwise kernels are built from).
 *
 *   linear    k(x, y) = <x, y>                      (Metz data: similarity rows)
 *   gaussian  k(x, y) = exp(-gamma ||x - y||^2)     (Metz data, squared norm)
 *
 * X is nx x dim (row stride ldx), Y is ny x dim (ldy); K[i*ldk + j] = k(X_i, Y_j).
 * Sums run over ascending feature index from 0.0; the Gaussian sums squared
 * differences directly (no norm expansion).  Returns 0, or -1 on bad arguments.
 */
int oracle_base_kernel(int kind, const double *X, int64_t nx, int64_t ldx, const double *Y,
                       int64_t ny, int64_t ldy, int64_t dim, double gamma, double *K, int64_t ldk)
{
    if ((kind != 0 && kind != 1) || nx < 0 || ny < 0 || dim < 0 || ldx < dim || ldy < dim ||
        ldk < ny)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nx; ++i) {
        for (int64_t j = 0; j < ny; ++j) {
            double s = 0.0;
            for (int64_t k = 0; k < dim; ++k) {
                if (kind == 0) {
                    s = s + X[i * ldx + k] * Y[j * ldy + k];
                } else {
                    double d = X[i * ldx + k] - Y[j * ldy + k];
                    s = s + d * d;
                }
            }
            K[i * ldk + j] = kind == 0 ? s : exp(-gamma * s);
        }
    }
    return 0;
}

/*
 * Tanimoto kernel on binary vectors (Section 5, Heterodimer data): the number
 * of positions set in both vectors over the number set in either,
 * sum_i min(v_i, w_i) / sum_i max(v_i, w_i).  Two all-zero vectors give 1
 * (a vector is identical to itself; reading of 0/0).
 *
 * Rows are packed bit vectors of nbits bits: bit b of row i is bit (b % 64) of
 * 64-bit word X[i*ldx + b/64].  Bits at and past nbits in the last word are
 * ignored.  Counts are taken bit by bit; the ratio is formed in double.
 */
int oracle_tanimoto(const uint64_t *X, int64_t nx, int64_t ldx, const uint64_t *Y, int64_t ny,
                    int64_t ldy, int64_t nbits, double *K, int64_t ldk)
{
    const int64_t words = (nbits + 63) / 64;
    if (nx < 0 || ny < 0 || nbits < 0 || ldx < words || ldy < words || ldk < ny) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nx; ++i) {
        for (int64_t j = 0; j < ny; ++j) {
            int64_t both = 0, either = 0;
            for (int64_t b = 0; b < nbits; ++b) {
                int v = (int)((X[i * ldx + b / 64] >> (b % 64)) & 1u);
                int w = (int)((Y[j * ldy + b / 64] >> (b % 64)) & 1u);
                both += v & w;
                either += v | w;
            }
            K[i * ldk + j] = either == 0 ? 1.0 : (double)both / (double)either;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Area under the ROC curve of predictions p against binary labels (label > 0.5
 * is a positive): the fraction of (positive, negative) pairs the predictions
 * order correctly, ties counting one half.  Plain double loop over all
 * pairs.  One class empty: 0.5 (no pair to order; reading). */
double oracle_auc(const double *p, const double *label, int64_t n)
{
    double good = 0.0;
    int64_t np = 0, nn = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] > 0.5) ++np;
        else ++nn;
    }
    if (np == 0 || nn == 0) return 0.5;
    for (int64_t i = 0; i < n; ++i) {
        if (!(label[i] > 0.5)) continue;
        for (int64_t j = 0; j < n; ++j) {
            if (label[j] > 0.5) continue;
            if (p[i] > p[j]) good = good + 1.0;
            else if (p[i] == p[j]) good = good + 0.5;
        }
    }
    return good / ((double)np * (double)nn);
}

/*
 * Kernel ridge regression (Section 3 eq. (1), (K + lambda I) a = y) by the
 * minimal residual method with early stopping on a validation sample
 * (Section 3; Section 6, early stopping ridge regression).
 *
 * MINRES: Lanczos on A = K + lambda I from r0 = y (a0 = 0),
 *   beta_1 v_1 = y;  q = A v_k - beta_k v_{k-1};  alpha_k = v_k.q;
 *   q -= alpha_k v_k;  beta_{k+1} = ||q||;  v_{k+1} = q / beta_{k+1},
 * and the QR factorisation of the tridiagonal Lanczos matrix by Givens
 * rotations, one new rotation per step:
 *   eps_k = s_{k-2} beta_k,  dt = c_{k-2} beta_k,
 *   delta_k = c_{k-1} dt + s_{k-1} alpha_k,  gbar = c_{k-1} alpha_k - s_{k-1} dt,
 *   gamma_k = sqrt(gbar^2 + beta_{k+1}^2),  c_k = gbar / gamma_k,  s_k = beta_{k+1} / gamma_k,
 *   tau_k = c_k phibar_{k-1},  phibar_k = -s_k phibar_{k-1}   (|phibar_k| = ||y - A a_k||),
 *   d_k = (v_k - delta_k d_{k-1} - eps_k d_{k-2}) / gamma_k,  a_k = a_{k-1} + tau_k d_k.
 * Stops when |phibar_k| / ||y|| < tol or after max_iter steps.
 *
 * Early stopping (optional, va != NULL): after every step the predictions on
 * the validation pairs (va, vb), p = R(va, vb) K R(c, e)^T a_k, give an AUC
 * against the binary labels yval; the best AUC (strictly larger than every
 * earlier one, starting from a_0 = 0) and its step are kept, Abest receives
 * a at that step, and the solve stops once `patience` steps have passed
 * without a better AUC (patience <= 0: no early stop).  auc_hist[k*nlam + l]
 * (may be NULL) receives the AUC after step k+1, NaN past the last step.
 *
 * Outputs per lambda: A (final iterate), iters, relres_est = |phibar|/||y||,
 * relres_true = ||y - (K + lambda I) a|| / ||y|| (one more product),
 * best_iter, best_auc.  Returns 0, -1 on bad arguments, -2 on a breakdown
 * (a non-finite value or gamma_k = 0).
 */
int oracle_krr_minres(int kind, const double *D, int64_t d_rows, int64_t d_cols, int64_t ldd,
                      const double *T, int64_t t_rows, int64_t t_cols, int64_t ldt,
                      const int32_t *c, const int32_t *e, int64_t n, const double *y,
                      const double *lambdas, int64_t nlam, int64_t max_iter, double tol,
                      const int32_t *va, const int32_t *vb, int64_t nval, const double *yval,
                      int64_t patience, double *A, int64_t lda, double *Abest, int64_t *iters,
                      double *relres_est, double *relres_true, double *auc_hist,
                      int64_t *best_iter, double *best_auc, int nthreads)
{
    if (n <= 0 || nlam <= 0 || lda < n || max_iter < 0) return -1;
    if (va && (!vb || !yval || nval <= 0)) return -1;
    double *vprev = (double *)malloc(sizeof(double) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *d1 = (double *)malloc(sizeof(double) * (size_t)n); /* d_{k-1} */
    double *d2 = (double *)malloc(sizeof(double) * (size_t)n); /* d_{k-2} */
    double *pv = va ? (double *)malloc(sizeof(double) * (size_t)nval) : NULL;
    int status = 0;
    const double ynorm = sqrt(dot_seq(y, y, n));
    for (int64_t l = 0; l < nlam && status == 0; ++l) {
        const double lam = lambdas[l];
        double *a = A + l * lda;
        double *ab = Abest ? Abest + l * lda : NULL;
        for (int64_t k = 0; k < n; ++k) {
            a[k] = 0.0;
            vprev[k] = 0.0;
            d1[k] = 0.0;
            d2[k] = 0.0;
            if (ab) ab[k] = 0.0;
        }
        for (int64_t k = 0; k < max_iter && auc_hist; ++k) auc_hist[k * nlam + l] = NAN;
        double beta = ynorm; /* beta_k */
        for (int64_t k = 0; k < n; ++k) v[k] = beta > 0.0 ? y[k] / beta : 0.0;
        double c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0; /* rotations k-1 and k-2 */
        double phibar = beta;
        double best = 0.5;
        if (va) { /* a_0 = 0: every prediction ties */
            for (int64_t i = 0; i < nval; ++i) pv[i] = 0.0;
            best = oracle_auc(pv, yval, nval);
        }
        int64_t kbest = 0, it = 0;
        while (it < max_iter && !(fabs(phibar) / (ynorm > 0.0 ? ynorm : 1.0) < tol)) {
            /* q = A v_k - beta_k v_{k-1} */
            if (oracle_pairwise_matvec(kind, D, d_rows, d_cols, ldd, T, t_rows, t_cols, ldt, c,
                                       e, n, NULL, 0, c, e, n, v, 1, n, q, n, nthreads) != 0) {
                status = -1;
                break;
            }
            for (int64_t k = 0; k < n; ++k) q[k] = q[k] + lam * v[k] - beta * vprev[k];
            const double alpha = dot_seq(v, q, n);
            for (int64_t k = 0; k < n; ++k) q[k] = q[k] - alpha * v[k];
            const double beta_next = sqrt(dot_seq(q, q, n));
            /* QR update of the new tridiagonal column */
            const double eps = s2 * beta, dt = c2 * beta;
            const double delta = c1 * dt + s1 * alpha;
            const double gbar = c1 * alpha - s1 * dt;
            const double gamma = sqrt(gbar * gbar + beta_next * beta_next);
            if (!(gamma > 0.0) || !isfinite(gamma)) {
                status = -2;
                break;
            }
            const double cs = gbar / gamma, sn = beta_next / gamma;
            const double tau = cs * phibar;
            phibar = -sn * phibar;
            /* d_k and the new iterate; rotate the history */
            for (int64_t k = 0; k < n; ++k) {
                const double dk = (v[k] - delta * d1[k] - eps * d2[k]) / gamma;
                d2[k] = d1[k];
                d1[k] = dk;
                a[k] = a[k] + tau * dk;
            }
            c2 = c1; s2 = s1; c1 = cs; s1 = sn;
            for (int64_t k = 0; k < n; ++k) {
                vprev[k] = v[k];
                v[k] = beta_next > 0.0 ? q[k] / beta_next : 0.0;
            }
            beta = beta_next;
            ++it;
            if (va) {
                oracle_pairwise_matvec(kind, D, d_rows, d_cols, ldd, T, t_rows, t_cols, ldt, va, vb,
                                       nval, NULL, 0, c, e, n, a, 1, n, pv, nval, nthreads);
                const double auc = oracle_auc(pv, yval, nval);
                if (auc_hist) auc_hist[(it - 1) * nlam + l] = auc;
                if (auc > best) {
                    best = auc;
                    kbest = it;
                    if (ab)
                        for (int64_t k = 0; k < n; ++k) ab[k] = a[k];
                }
                if (patience > 0 && it - kbest >= patience) break;
            }
        }
        iters[l] = it;
        relres_est[l] = fabs(phibar) / (ynorm > 0.0 ? ynorm : 1.0);
        if (best_iter) best_iter[l] = kbest;
        if (best_auc) best_auc[l] = best;
        if (status == 0) {
            oracle_pairwise_matvec(kind, D, d_rows, d_cols, ldd, T, t_rows, t_cols, ldt, c, e, n,
                                   NULL, 0, c, e, n, a, 1, n, q, n, nthreads);
            double s = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                const double dd = y[k] - (q[k] + lam * a[k]);
                s = s + dd * dd;
            }
            relres_true[l] = sqrt(s) / (ynorm > 0.0 ? ynorm : 1.0);
        }
    }
    free(vprev);
    free(v);
    free(q);
    free(d1);
    free(d2);
    free(pv);
    return status;
}
