/*
 * Plain FP64 CPU oracle for block-Jacobi preconditioned CG and Lanczos
 * condition-number estimation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product path never does.  It shares no code, header or table with the GPU
 * library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, all
 * sums sequential left to right, single thread).  This is the build every
 * parity check uses.
 *
 * Timing build (-fopenmp, used only to time the oracle on all host cores):
 * the loops marked "omp" below run in parallel.  Row products, element-wise
 * vector updates and block solves give the same values as the sequential
 * build; a dot product becomes fixed contiguous per-thread chunks (static
 * split of [0, n) by thread number), each summed left to right, then the
 * chunk sums added in thread order: deterministic for a given thread count,
 * but rounded differently from the sequential sum.
 *
 * What it follows (paper: "Optimised Hybrid Classical-Quantum Algorithm ...",
 * arXiv 2410.02408):
 *   - Section 3.1: A is sparse, Hermitian (here: real symmetric) positive
 *     definite; kappa(A) = ||A|| ||A^-1||, read as the 2-norm ratio
 *     lambda_max / lambda_min.
 *   - Section 3.2: A and b are split into contiguous diagonal blocks of size
 *     n_b; the partition code of Section 4.2 slices in steps of n_b, so the
 *     last block is shorter when n_b does not divide N.
 *   - Section 3.3: each block gets its own preconditioner M_i and the system
 *     becomes M_i A_i.  The paper's M_i is the inverse of diag(A_i) (its CUDA
 *     kernel in Section 4.3 stores 1/A[i][i]); this library generalises it to
 *     the inverse of the whole diagonal block A_ii, so that block size 1
 *     reproduces the paper's point Jacobi exactly.
 *   - Section 3.6: x is the concatenation of the block solutions; for a
 *     block-diagonal A one application of M^-1 is that aggregate.
 *   - Section 3.7: accuracy is ||A x - b|| / ||b|| (2-norm).
 * The paper has no iterative solver and no estimator; the algorithms below
 * are textbook:
 *   - PCG: Hestenes-Stiefel conjugate gradient with a symmetric
 *     preconditioner (Saad, Iterative Methods for Sparse Linear Systems,
 *     2nd ed., Algorithm 9.1), recursive-residual stop, then a true-residual
 *     check with residual replacement.
 *   - Lanczos in the M inner product (Golub & Van Loan, Matrix
 *     Computations, 4th ed., Sec. 10.1 / 11.3 for the preconditioned form)
 *     with classical Gram-Schmidt applied twice for full
 *     reorthogonalisation.
 *   - Extreme eigenvalues of the Lanczos tridiagonal by Sturm-count
 *     bisection (Barth, Martin & Wilkinson, Numer. Math. 9, 1967).
 *   - Block factorisation: Cholesky-Banachiewicz (row by row, no pivoting);
 *     M^-1 is applied by forward then backward substitution with L.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTSPD (-2)
#define ORC_ENOCONV (-3)
#define ORC_EBREAKDOWN (-4)
#define ORC_ENONFINITE (-5)

/* ------------------------------------------------------------------ */
/* CSR basics                                                          */
/* ------------------------------------------------------------------ */

/* Structural validation: row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz,
 * 0 <= col < n, all values finite. */
int orc_csr_validate(int n, const int *row_ptr, const int *col, const double *val)
{
    if (n < 0) return ORC_EINVAL;
    if (n == 0) return ORC_OK;
    if (row_ptr[0] != 0) return ORC_EINVAL;
    for (int i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return ORC_EINVAL;
    for (int k = 0; k < row_ptr[n]; ++k) {
        if (col[k] < 0 || col[k] >= n) return ORC_EINVAL;
        if (!isfinite(val[k])) return ORC_ENONFINITE;
    }
    return ORC_OK;
}

/* y = A x, each row summed in storage order. */
void orc_spmv(int n, const int *row_ptr, const int *col, const double *val,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

double orc_dot(int n, const double *a, const double *b)
{
#ifdef _OPENMP
    /* timing build only: per-thread chunks, chunk sums in thread order */
    double part[256];
    int nt = omp_get_max_threads();
    if (nt > 256) nt = 256;
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num(), used = omp_get_num_threads();
        long lo = (long)n * t / used, hi = (long)n * (t + 1) / used;
        double s = 0.0;
        for (long i = lo; i < hi; ++i) s += a[i] * b[i];
        part[t] = s;
#pragma omp single
        nt = used;
    }
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += part[t];
    return s;
#else
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
#endif
}

/* Threads of the timing build (no effect on the sequential build); returns
 * the number the parallel loops will use. */
int orc_set_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
    return omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Block partition (Section 3.2 and the slicing of Section 4.2)         */
/* ------------------------------------------------------------------ */

/* Contiguous blocks of nb rows, the last one ragged: block t covers rows
 * [t*nb, min((t+1)*nb, n)).  Writes offsets[0..k]; returns k (or -1). */
int orc_uniform_offsets(int n, int nb, int *offsets)
{
    if (nb <= 0 || n < 0) return -1;
    int k = 0;
    offsets[0] = 0;
    for (int s = 0; s < n; s += nb) {
        int e = s + nb < n ? s + nb : n;
        offsets[++k] = e;
    }
    return k;
}

/* Dense copy of the diagonal block rows/cols [s, e): the sum of every stored
 * entry (i, j) with both i and j inside the block; entries outside the block
 * are ignored, missing ones are zero.  tile is (e-s)^2, row-major. */
void orc_extract_block(const int *row_ptr, const int *col, const double *val,
                       int s, int e, double *tile)
{
    int m = e - s;
    memset(tile, 0, sizeof(double) * (size_t)m * (size_t)m);
    for (int i = s; i < e; ++i)
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] >= s && col[k] < e)
                tile[(size_t)(i - s) * m + (col[k] - s)] += val[k];
}

/* Cholesky-Banachiewicz on an m x m row-major SPD tile, in place: on return
 * the lower triangle holds L (A = L L^T) and the strict upper triangle is
 * zero.  Returns ORC_OK, or ORC_ENOTSPD if a pivot argument is <= 0 or not
 * finite. */
int orc_cholesky(int m, double *a)
{
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = a[(size_t)i * m + j];
            for (int k = 0; k < j; ++k)
                s -= a[(size_t)i * m + k] * a[(size_t)j * m + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return ORC_ENOTSPD;
                a[(size_t)i * m + i] = sqrt(s);
            } else {
                a[(size_t)i * m + j] = s / a[(size_t)j * m + j];
            }
        }
        for (int j = i + 1; j < m; ++j) a[(size_t)i * m + j] = 0.0;
    }
    return ORC_OK;
}

/* Solve (L L^T) z = r for one block: forward L y = r, then backward
 * L^T z = y.  z may alias r. */
void orc_chol_solve(int m, const double *L, const double *r, double *z)
{
    for (int i = 0; i < m; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * m + k] * z[k];
        z[i] = s / L[(size_t)i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < m; ++k) s -= L[(size_t)k * m + i] * z[k];
        z[i] = s / L[(size_t)i * m + i];
    }
}

/* The block-Jacobi preconditioner: one dense Cholesky factor per block. */
typedef struct {
    int n, nblocks;
    int *offsets;       /* [nblocks+1] */
    size_t *tile_at;    /* [nblocks] start of block t's factor in L */
    double *L;          /* sum_t m_t^2 doubles */
} orc_precond;

void orc_precond_free(orc_precond *P)
{
    if (!P) return;
    free(P->offsets);
    free(P->tile_at);
    free(P->L);
    free(P);
}

/* Build M = blockdiag(A_11, ..., A_kk) for the given offsets and factor every
 * block.  On failure returns NULL and sets *status (ORC_ENOTSPD with
 * *failed_block = first failing block, or ORC_EINVAL). */
orc_precond *orc_precondition(int n, const int *row_ptr, const int *col, const double *val,
                              int nblocks, const int *offsets, int *status, int *failed_block)
{
    *status = ORC_OK;
    *failed_block = -1;
    if (n < 0 || nblocks < 0 || offsets[0] != 0 || offsets[nblocks] != n) {
        *status = ORC_EINVAL;
        return NULL;
    }
    for (int t = 0; t < nblocks; ++t)
        if (offsets[t + 1] <= offsets[t]) {
            *status = ORC_EINVAL;
            return NULL;
        }
    orc_precond *P = (orc_precond *)calloc(1, sizeof(orc_precond));
    P->n = n;
    P->nblocks = nblocks;
    P->offsets = (int *)malloc(sizeof(int) * (size_t)(nblocks + 1));
    P->tile_at = (size_t *)malloc(sizeof(size_t) * (size_t)(nblocks > 0 ? nblocks : 1));
    memcpy(P->offsets, offsets, sizeof(int) * (size_t)(nblocks + 1));
    size_t total = 0;
    for (int t = 0; t < nblocks; ++t) {
        size_t m = (size_t)(offsets[t + 1] - offsets[t]);
        P->tile_at[t] = total;
        total += m * m;
    }
    P->L = (double *)malloc(sizeof(double) * (total > 0 ? total : 1));
    for (int t = 0; t < nblocks; ++t) {
        int s = offsets[t], e = offsets[t + 1];
        double *tile = P->L + P->tile_at[t];
        orc_extract_block(row_ptr, col, val, s, e, tile);
        if (orc_cholesky(e - s, tile) != ORC_OK) {
            *status = ORC_ENOTSPD;
            *failed_block = t;
            orc_precond_free(P);
            return NULL;
        }
    }
    return P;
}

/* z = M^-1 r, block by block. */
void orc_apply(const orc_precond *P, const double *r, double *z)
{
#pragma omp parallel for schedule(static)
    for (int t = 0; t < P->nblocks; ++t) {
        int s = P->offsets[t], e = P->offsets[t + 1];
        orc_chol_solve(e - s, P->L + P->tile_at[t], r + s, z + s);
    }
}

/* Copy of block t's Cholesky factor (m x m row-major) for tests. */
int orc_precond_block(const orc_precond *P, int t, double *out)
{
    if (t < 0 || t >= P->nblocks) return ORC_EINVAL;
    int m = P->offsets[t + 1] - P->offsets[t];
    memcpy(out, P->L + P->tile_at[t], sizeof(double) * (size_t)m * (size_t)m);
    return m;
}

static void apply_or_copy(const orc_precond *P, int n, const double *r, double *z)
{
    if (P) orc_apply(P, r, z);
    else memcpy(z, r, sizeof(double) * (size_t)n);
}

static int all_finite(int n, const double *v)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Preconditioned conjugate gradient                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int status, iterations, replacements;
    double rel_res_recursive, rel_res_true;
} orc_pcg_info;

/* Solve A x = b with PCG (Saad Alg. 9.1), M = P (NULL: plain CG).
 *   x: in = x0 when x0_given, out = solution (last iterate on failure).
 *   Stop when ||r||_2 <= tol ||b||_2 on the recursive residual; then check
 *   the true residual ||b - A x|| / ||b|| (Section 3.7); if it is above tol,
 *   replace r by the true residual, restart the direction and continue (at
 *   most max_replacements times).  max_iter bounds the total number of
 *   iterations; a replacement is made only while iterations remain (at
 *   k = max_iter the solve ends with ENOCONV instead, the replacement count
 *   unchanged).  history (optional, >= max_iter+1 entries) receives the
 *   recursive relative residual after every iteration (index 0 = start). */
int orc_pcg(int n, const int *row_ptr, const int *col, const double *val,
            const orc_precond *P, const double *b, double *x, double tol, int max_iter,
            int x0_given, int max_replacements, orc_pcg_info *info, double *history)
{
    memset(info, 0, sizeof(*info));
    if (!all_finite(n, b) || (x0_given && !all_finite(n, x))) {
        info->status = ORC_ENONFINITE;
        return info->status;
    }
    if (!x0_given)
        for (int i = 0; i < n; ++i) x[i] = 0.0;
    double bnorm = sqrt(orc_dot(n, b, b));
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        info->status = ORC_OK;
        return ORC_OK;
    }
    size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(bytes), *z = (double *)malloc(bytes);
    double *p = (double *)malloc(bytes), *q = (double *)malloc(bytes);
    int k = 0, status = ORC_OK;
    double relres = 0.0;

    for (;;) {
        /* (re)start: r = b - A x, z = M^-1 r, p = z */
        orc_spmv(n, row_ptr, col, val, x, q);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
        double rr = orc_dot(n, r, r);
        if (!isfinite(rr)) { status = ORC_ENONFINITE; break; }
        relres = sqrt(rr) / bnorm;
        if (history && k == 0) history[0] = relres;
        if (relres > tol) {
            apply_or_copy(P, n, r, z);
            double rho = orc_dot(n, r, z);
            if (!(rho > 0.0)) { status = isfinite(rho) ? ORC_EBREAKDOWN : ORC_ENONFINITE; break; }
            memcpy(p, z, bytes);
            for (;;) {
                if (k >= max_iter) { status = ORC_ENOCONV; break; }
                orc_spmv(n, row_ptr, col, val, p, q);
                double sigma = orc_dot(n, p, q);
                if (!(sigma > 0.0)) { status = isfinite(sigma) ? ORC_EBREAKDOWN : ORC_ENONFINITE; break; }
                double alpha = rho / sigma;
#pragma omp parallel for schedule(static)
                for (int i = 0; i < n; ++i) x[i] += alpha * p[i];
#pragma omp parallel for schedule(static)
                for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];
                ++k;  /* iterations = completed updates of x */
                rr = orc_dot(n, r, r);
                if (!isfinite(rr)) { status = ORC_ENONFINITE; break; }
                relres = sqrt(rr) / bnorm;
                if (history) history[k] = relres;
                if (relres <= tol) break;
                apply_or_copy(P, n, r, z);
                double rho_new = orc_dot(n, r, z);
                if (!(rho_new > 0.0)) { status = isfinite(rho_new) ? ORC_EBREAKDOWN : ORC_ENONFINITE; break; }
                double beta = rho_new / rho;
#pragma omp parallel for schedule(static)
                for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
                rho = rho_new;
            }
            if (status != ORC_OK) break;
        }
        /* true-residual check (Section 3.7) */
        orc_spmv(n, row_ptr, col, val, x, q);
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
        double tres = sqrt(orc_dot(n, q, q)) / bnorm;
        info->rel_res_true = tres;
        if (tres <= tol) break;
        if (info->replacements >= max_replacements || k >= max_iter) { status = ORC_ENOCONV; break; }
        info->replacements++;
    }
    if (status != ORC_OK) {
        orc_spmv(n, row_ptr, col, val, x, q);
        for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
        info->rel_res_true = sqrt(orc_dot(n, q, q)) / bnorm;
    }
    info->status = status;
    info->iterations = k;
    info->rel_res_recursive = relres;
    free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Lanczos in the M inner product, full CGS2 reorthogonalisation        */
/* ------------------------------------------------------------------ */

/* m-step Lanczos on M^-1 A (M = P; NULL -> A itself) from start vector v0.
 * Basis v_j is M-orthonormal, u_j = M v_j is kept alongside so that M is
 * never applied forward.  Outputs alpha[0..s-1], beta[0..s-2] of the s x s
 * tridiagonal T (s = *steps_done) and, if beta_last is non-NULL, the final
 * off-diagonal residual.  Stops early (success) when the new beta falls below
 * 1e-12 times the largest |alpha| or beta seen so far. */
int orc_lanczos(int n, const int *row_ptr, const int *col, const double *val,
                const orc_precond *P, const double *v0, int m,
                double *alpha, double *beta, int *steps_done)
{
    *steps_done = 0;
    if (m <= 0 || n <= 0) return ORC_EINVAL;
    if (!all_finite(n, v0)) return ORC_ENONFINITE;
    size_t bytes = sizeof(double) * (size_t)n;
    double *U = (double *)malloc(bytes * (size_t)(m + 1));
    double *V = (double *)malloc(bytes * (size_t)(m + 1));
    double *r = (double *)malloc(bytes), *z = (double *)malloc(bytes);
    double *c = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    int status = ORC_OK;

    memcpy(r, v0, bytes);
    apply_or_copy(P, n, r, z);
    double b0 = orc_dot(n, r, z);
    if (!(b0 > 0.0)) {
        status = isfinite(b0) ? ORC_EBREAKDOWN : ORC_ENONFINITE;
        goto done;
    }
    b0 = sqrt(b0);
    for (int i = 0; i < n; ++i) { U[i] = r[i] / b0; V[i] = z[i] / b0; }

    double scale = 0.0, beta_prev = 0.0;
    for (int j = 0; j < m; ++j) {
        double *uj = U + (size_t)j * n, *vj = V + (size_t)j * n;
        orc_spmv(n, row_ptr, col, val, vj, r);            /* w = A v_j */
        double a = orc_dot(n, vj, r);
        alpha[j] = a;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) r[i] -= a * uj[i];
        if (j > 0) {
            double *up = U + (size_t)(j - 1) * n;
#pragma omp parallel for schedule(static)
            for (int i = 0; i < n; ++i) r[i] -= beta_prev * up[i];
        }
        for (int pass = 0; pass < 2; ++pass) {              /* CGS2 */
            for (int l = 0; l <= j; ++l) c[l] = orc_dot(n, V + (size_t)l * n, r);
            for (int l = 0; l <= j; ++l) {
                double *ul = U + (size_t)l * n;
#pragma omp parallel for schedule(static)
                for (int i = 0; i < n; ++i) r[i] -= c[l] * ul[i];
            }
        }
        apply_or_copy(P, n, r, z);
        double bb = orc_dot(n, r, z);
        if (!isfinite(bb) || !isfinite(a)) { status = ORC_ENONFINITE; *steps_done = j + 1; goto done; }
        double bj = sqrt(bb > 0.0 ? bb : 0.0);
        if (fabs(a) > scale) scale = fabs(a);
        *steps_done = j + 1;
        if (j + 1 == m || bj <= 1e-12 * scale) break;
        if (bj > scale) scale = bj;
        beta[j] = bj;
        double *un = U + (size_t)(j + 1) * n, *vn = V + (size_t)(j + 1) * n;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) { un[i] = r[i] / bj; vn[i] = z[i] / bj; }
        beta_prev = bj;
    }
done:
    free(U); free(V); free(r); free(z); free(c);
    return status;
}

/* ------------------------------------------------------------------ */
/* Extreme eigenvalues of a symmetric tridiagonal (Sturm bisection)     */
/* ------------------------------------------------------------------ */

static double orc_pivmin(int s, const double *beta)
{
    double mx = 1.0;
    for (int i = 0; i + 1 < s; ++i)
        if (beta[i] * beta[i] > mx) mx = beta[i] * beta[i];
    return 2.2250738585072014e-308 * mx;
}

/* Number of eigenvalues of T (diag alpha[0..s-1], off beta[0..s-2]) that are
 * strictly less than x: the count of negative pivots of the LDL^T
 * factorisation of T - x I, d_0 = alpha_0 - x,
 * d_i = alpha_i - x - beta_{i-1}^2 / d_{i-1}; tiny pivots are pushed to
 * -pivmin. */
int orc_sturm_count(int s, const double *alpha, const double *beta, double x)
{
    double pivmin = orc_pivmin(s, beta);
    int cnt = 0;
    double d = alpha[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0.0) ++cnt;
    for (int i = 1; i < s; ++i) {
        d = alpha[i] - x - beta[i - 1] * beta[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

/* Smallest and largest eigenvalue of T by bisection on the Sturm count,
 * starting from the (slightly widened) Gershgorin interval and stopping when
 * the bracket is below 2 eps max(|lo|, |hi|) (or after 200 halvings). */
int orc_tridiag_extremes(int s, const double *alpha, const double *beta,
                         double *theta_min, double *theta_max)
{
    if (s <= 0) return ORC_EINVAL;
    double glo = alpha[0], ghi = alpha[0];
    for (int i = 0; i < s; ++i) {
        double rad = 0.0;
        if (i > 0) rad += fabs(beta[i - 1]);
        if (i + 1 < s) rad += fabs(beta[i]);
        if (alpha[i] - rad < glo) glo = alpha[i] - rad;
        if (alpha[i] + rad > ghi) ghi = alpha[i] + rad;
    }
    double pivmin = orc_pivmin(s, beta);
    double widen = 4.0 * 2.220446049250313e-16 * (fabs(glo) + fabs(ghi) + (ghi - glo)) * s + 2.0 * pivmin;
    glo -= widen;
    ghi += widen;
    for (int which = 0; which < 2; ++which) {
        /* which = 0: the first eigenvalue (count reaches 1);
         * which = 1: the last one (count reaches s). */
        int target = which == 0 ? 1 : s;
        double lo = glo, hi = ghi;
        for (int it = 0; it < 200; ++it) {
            double tolw = 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi));
            if (hi - lo <= tolw || hi - lo <= pivmin) break;
            double mid = 0.5 * (lo + hi);
            if (orc_sturm_count(s, alpha, beta, mid) >= target) hi = mid;
            else lo = mid;
        }
        if (which == 0) *theta_min = 0.5 * (lo + hi);
        else *theta_max = 0.5 * (lo + hi);
    }
    return ORC_OK;
}

/* kappa estimate: Lanczos followed by the tridiagonal extremes. */
int orc_kappa(int n, const int *row_ptr, const int *col, const double *val,
              const orc_precond *P, const double *v0, int m, double *alpha, double *beta,
              int *steps_done, double *theta_min, double *theta_max, double *kappa)
{
    int st = orc_lanczos(n, row_ptr, col, val, P, v0, m, alpha, beta, steps_done);
    if (st != ORC_OK) return st;
    orc_tridiag_extremes(*steps_done, alpha, beta, theta_min, theta_max);
    *kappa = *theta_max / *theta_min;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Adjoint gradients of a PCG solve                                     */
/* ------------------------------------------------------------------ */

/* For x = A^-1 b and a loss with dL/dx = g, the adjoint lambda = A^-1 g
 * (A symmetric) gives dL/db = lambda and dL/dA_ij = -lambda_i x_j for every
 * stored entry (i, j).  grad[k] receives that value for stored entry k. */
void orc_value_grad(int n, const int *row_ptr, const int *col,
                    const double *lambda, const double *x, double *grad)
{
    for (int i = 0; i < n; ++i)
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            grad[k] = -lambda[i] * x[col[k]];
}

/* Chain rule to per-edge conductivities of A = sum_e c_e (e_i - e_j)(e_i -
 * e_j)^T + sum_b c_b e_i e_i^T: dL/dc_e = -(lambda_i - lambda_j)(x_i - x_j)
 * for an interior edge and -lambda_i x_i for a boundary face. */
void orc_edge_grad(int n_edges, const int *ei, const int *ej, int n_bdry, const int *bi,
                   const double *lambda, const double *x, double *grad)
{
    for (int e = 0; e < n_edges; ++e)
        grad[e] = -(lambda[ei[e]] - lambda[ej[e]]) * (x[ei[e]] - x[ej[e]]);
    for (int e = 0; e < n_bdry; ++e)
        grad[n_edges + e] = -lambda[bi[e]] * x[bi[e]];
}
