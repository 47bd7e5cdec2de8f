/*
 * FP64 CPU oracle for the EbV LU path.  TEST INFRASTRUCTURE ONLY: it is called
 * by the test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark, never by the GPU product path, and it shares no code with it.
 *
 * What it computes (Hashemi, Lahooti, Shirani, "Equal bi-Vectorized (EbV)
 * method to high performance on GPU", arXiv:1907.05767):
 *
 *   AX = B  <=>  L(UX) = B: solve LY = B by forward substitution, then UX = Y
 *   by backward substitution (Eq. 1; the paper's "UX = B" is read as UX = Y).
 *
 *   The factors are the Doolittle ones: L unit lower triangular, U upper
 *   triangular carrying the pivots, stored in place of A (Eq. 3 read with the
 *   unit diagonal on L).  For strictly diagonally dominant A (Eq. 2) every
 *   leading principal minor is nonzero, so this factorization exists, is
 *   unique, and needs no pivoting.
 *
 *   Elimination step r (Eq. 6-a, 6-c): the multipliers of column r are the
 *   sub-diagonal entries divided by the pivot A_rr, and the active submatrix
 *   receives the rank-1 update  A <- A - l_r u_r^T  where u_r is row r right of
 *   (and including) the diagonal.  The paper writes the multipliers with a
 *   minus sign (the Gauss-transform convention); the stored L here holds the
 *   positive multipliers and the update subtracts, which is the same factor.
 *   The U row is left unscaled (Doolittle), so det(A) = prod U_ii.
 *
 *   The EbV equalization (Eq. 7 and the following paragraph) only decides
 *   which thread computes which part of each step; it does not change the
 *   result, so the oracle performs the steps in plain loop order.
 *
 * Layout: row-major, a_ij at A[i*lda + j].  Band storage is row-wise:
 * a_ij at AB[i*ldab + (j - i + kl)] for |band| entries.
 *
 * Precision: double throughout, except oracle_refine_mixed, which follows the
 * mixed-precision recipe (float factor and correction solves, double residual
 * and update) in plain C float/double arithmetic.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no FMA contraction, so every
 * product and sum is rounded separately, in loop order).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#define EBV_ORACLE_VERSION 1

int oracle_version(void) { return EBV_ORACLE_VERSION; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- dense --- */

/* Doolittle LU in place (Eq. 6-a, 6-c).  Returns 0, or k+1 when the pivot of
 * step k is exactly zero (the factor stops there, entries beyond are left as
 * they were after step k-1). */
int oracle_lu_factor(int64_t n, double *A, int64_t lda)
{
    for (int64_t k = 0; k < n; ++k) {
        const double p = A[k * lda + k];
        if (p == 0.0)
            return (int)(k + 1);
        /* Eq. 6-a: multipliers of column k */
        for (int64_t i = k + 1; i < n; ++i)
            A[i * lda + k] = A[i * lda + k] / p;
        /* Eq. 6-c: rank-1 update of the active submatrix */
#pragma omp parallel for schedule(static) if (n - k > 256)
        for (int64_t i = k + 1; i < n; ++i) {
            const double l = A[i * lda + k];
            double *ri = A + i * lda;
            const double *rk = A + k * lda;
            for (int64_t j = k + 1; j < n; ++j)
                ri[j] = ri[j] - l * rk[j];
        }
    }
    return 0;
}

/* Forward substitution L Y = B (unit diagonal), in place in B (n x nrhs). */
void oracle_forward(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                    double *B, int64_t ldb)
{
#pragma omp parallel for schedule(static) if (nrhs > 1)
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t i = 0; i < n; ++i) {
            double s = B[i * ldb + c];
            for (int64_t j = 0; j < i; ++j)
                s = s - LU[i * lda + j] * B[j * ldb + c];
            B[i * ldb + c] = s;
        }
    }
}

/* Backward substitution U X = Y, in place in B. */
void oracle_backward(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                     double *B, int64_t ldb)
{
#pragma omp parallel for schedule(static) if (nrhs > 1)
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = B[i * ldb + c];
            for (int64_t j = i + 1; j < n; ++j)
                s = s - LU[i * lda + j] * B[j * ldb + c];
            B[i * ldb + c] = s / LU[i * lda + i];
        }
    }
}

/* Eq. 1: forward then backward substitution. */
void oracle_lu_solve(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                     double *B, int64_t ldb)
{
    oracle_forward(n, nrhs, LU, lda, B, ldb);
    oracle_backward(n, nrhs, LU, lda, B, ldb);
}

/* ----------------------------------------------------------------- band --- */

/* Band Doolittle LU in row-wise band storage.  Without pivoting the factors of
 * a band matrix keep its band (L has kl sub-diagonals, U has ku super-
 * diagonals), so the dense steps restricted to the band give the same result. */
#define BAND(AB, ldab, kl, i, j) (AB)[(i) * (ldab) + ((j) - (i) + (kl))]

int oracle_lu_factor_band(int64_t n, int64_t kl, int64_t ku, double *AB, int64_t ldab)
{
    for (int64_t k = 0; k < n; ++k) {
        const double p = BAND(AB, ldab, kl, k, k);
        if (p == 0.0)
            return (int)(k + 1);
        const int64_t ilast = (k + kl < n - 1) ? k + kl : n - 1;
        const int64_t jlast = (k + ku < n - 1) ? k + ku : n - 1;
        for (int64_t i = k + 1; i <= ilast; ++i)
            BAND(AB, ldab, kl, i, k) = BAND(AB, ldab, kl, i, k) / p;
        for (int64_t i = k + 1; i <= ilast; ++i) {
            const double l = BAND(AB, ldab, kl, i, k);
            for (int64_t j = k + 1; j <= jlast; ++j)
                BAND(AB, ldab, kl, i, j) = BAND(AB, ldab, kl, i, j) - l * BAND(AB, ldab, kl, k, j);
        }
    }
    return 0;
}

void oracle_lu_solve_band(int64_t n, int64_t kl, int64_t ku, int64_t nrhs,
                          const double *AB, int64_t ldab, double *B, int64_t ldb)
{
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t i = 0; i < n; ++i) {
            double s = B[i * ldb + c];
            const int64_t j0 = (i - kl > 0) ? i - kl : 0;
            for (int64_t j = j0; j < i; ++j)
                s = s - BAND(AB, ldab, kl, i, j) * B[j * ldb + c];
            B[i * ldb + c] = s;
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = B[i * ldb + c];
            const int64_t j1 = (i + ku < n - 1) ? i + ku : n - 1;
            for (int64_t j = i + 1; j <= j1; ++j)
                s = s - BAND(AB, ldab, kl, i, j) * B[j * ldb + c];
            B[i * ldb + c] = s / BAND(AB, ldab, kl, i, i);
        }
    }
}

/* -------------------------------------------------------------- skyline --- */

/* Skyline (profile) storage: the strictly lower part by rows, row i holding
 * a_ij for f[i] <= j < i at AL[rp[i] + j - f[i]]; the upper part with the
 * diagonal by columns, column j holding a_ij for g[j] <= i <= j at
 * AU[cp[j] + i - g[j]].  Without pivoting the factors keep this envelope:
 * the update of step k reaches a_ij only when a_ik and a_kj are inside it
 * (k >= f[i], k >= g[j]), and then j > k >= f[i] and i > k >= g[j]. */
#define SKY_L(i, j) AL[rp[i] + (j) - f[i]]
#define SKY_U(i, j) AU[cp[j] + (i) - g[j]]

/* Doolittle LU restricted to the envelope (Eq. 6-a, 6-c): the same steps in
 * the same order as the dense factor, skipping the products with an entry
 * outside the envelope (zero). */
int oracle_lu_factor_skyline(int64_t n, const int32_t *f, const int64_t *rp, double *AL,
                             const int32_t *g, const int64_t *cp, double *AU)
{
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int ret = 0;
    if (!rows || !cols) {
        free(rows);
        free(cols);
        return -1;
    }
    for (int64_t k = 0; k < n; ++k) {
        const double p = SKY_U(k, k);
        if (p == 0.0) {
            ret = (int)(k + 1);
            break;
        }
        /* rows and columns whose envelope reaches step k, in index order */
        int64_t nr = 0, nc = 0;
        for (int64_t i = k + 1; i < n; ++i)
            if (f[i] <= k)
                rows[nr++] = i;
        for (int64_t j = k + 1; j < n; ++j)
            if (g[j] <= k)
                cols[nc++] = j;
        /* Eq. 6-a: multipliers of column k */
        for (int64_t a = 0; a < nr; ++a)
            SKY_L(rows[a], k) = SKY_L(rows[a], k) / p;
        /* Eq. 6-c: rank-1 update of the envelope */
#pragma omp parallel for schedule(static) if (nr > 64)
        for (int64_t a = 0; a < nr; ++a) {
            const int64_t i = rows[a];
            const double l = SKY_L(i, k);
            for (int64_t b = 0; b < nc; ++b) {
                const int64_t j = cols[b];
                const double u = SKY_U(k, j);
                if (j < i)
                    SKY_L(i, j) = SKY_L(i, j) - l * u;
                else
                    SKY_U(i, j) = SKY_U(i, j) - l * u;
            }
        }
    }
    free(rows);
    free(cols);
    return ret;
}

/* Eq. 1 on the skyline factors: L Y = B by rows (ascending j), then U X = Y
 * by rows (ascending j over the columns whose envelope reaches row i), in
 * place in B (n x nrhs): the dense substitutions' order, zero terms skipped. */
void oracle_lu_solve_skyline(int64_t n, int64_t nrhs, const int32_t *f, const int64_t *rp, const double *AL,
                             const int32_t *g, const int64_t *cp, const double *AU, double *B, int64_t ldb)
{
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t i = 0; i < n; ++i) {
            double s = B[i * ldb + c];
            for (int64_t j = f[i]; j < i; ++j)
                s = s - SKY_L(i, j) * B[j * ldb + c];
            B[i * ldb + c] = s;
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = B[i * ldb + c];
            for (int64_t j = i + 1; j < n; ++j)
                if (g[j] <= i)
                    s = s - SKY_U(i, j) * B[j * ldb + c];
            B[i * ldb + c] = s / SKY_U(i, i);
        }
    }
}
#undef SKY_L
#undef SKY_U

/* -------------------------------------------------------------- adjoint --- */

/* Reverse-mode derivative of X = A^{-1} B given the factors LU = A and the
 * solution X.  With Xbar = dLoss/dX:
 *     Bbar = A^{-T} Xbar       (U^T Z = Xbar forward, then L^T Bbar = Z backward)
 *     Abar = -Bbar X^T
 * Bbar overwrites Xbar in place.  Abar (n x n) is written when non-NULL. */
void oracle_lu_solve_adjoint(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                             const double *X, int64_t ldx, double *Bbar, int64_t ldb,
                             double *Abar, int64_t ldabar)
{
    for (int64_t c = 0; c < nrhs; ++c) {
        /* U^T z = xbar: (U^T)_{ij} = U_ji, lower triangular, non-unit */
        for (int64_t i = 0; i < n; ++i) {
            double s = Bbar[i * ldb + c];
            for (int64_t j = 0; j < i; ++j)
                s = s - LU[j * lda + i] * Bbar[j * ldb + c];
            Bbar[i * ldb + c] = s / LU[i * lda + i];
        }
        /* L^T bbar = z: (L^T)_{ij} = L_ji, upper triangular, unit diagonal */
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = Bbar[i * ldb + c];
            for (int64_t j = i + 1; j < n; ++j)
                s = s - LU[j * lda + i] * Bbar[j * ldb + c];
            Bbar[i * ldb + c] = s;
        }
    }
    if (Abar) {
#pragma omp parallel for schedule(static) if (n > 256)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double s = 0.0;
                for (int64_t c = 0; c < nrhs; ++c)
                    s = s + Bbar[i * ldb + c] * X[j * ldx + c];
                Abar[i * ldabar + j] = -s;
            }
    }
}

/* -------------------------------------------------------------- batched --- */

/* Independent systems packed back to back: system s has size n[s], its matrix
 * (row-major, lda = n[s]) at A + offA[s] and its n[s] x nrhs right-hand side at
 * B + offB[s].  Factor + solve each; info[s] as oracle_lu_factor. */
void oracle_lu_factor_solve_batched(int64_t count, const int32_t *n, const int64_t *offA,
                                    double *A, const int64_t *offB, double *B,
                                    int64_t nrhs, int32_t *info)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < count; ++s) {
        const int64_t m = n[s];
        int st = oracle_lu_factor(m, A + offA[s], m);
        info[s] = st;
        if (st == 0 && B)
            oracle_lu_solve(m, nrhs, A + offA[s], m, B + offB[s], nrhs);
    }
}

/* ------------------------------------------------------- mixed precision --- */

/* Mixed-precision solve (iterative refinement): the factor and the correction
 * solves run in float on the float-rounded matrix; the residual R = B - A X,
 * the update X += D and the stopping test run in double.  Stops when, for
 * every column c, max_i |r_ic| / max_i |b_ic| <= tol, or after max_iter
 * corrections.  iters[c] and relres[c] report per column.  Returns 0 when
 * converged, 1 when not, -k for a zero float pivot at step k-1.
 * Scratch: caller-free; the routine allocates with malloc. */
int oracle_refine_mixed(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double *X, int64_t ldx,
                        int max_iter, double tol, int32_t *iters, double *relres)
{
    float *F = (float *)malloc(sizeof(float) * (size_t)(n * n + 1));
    float *r32 = (float *)malloc(sizeof(float) * (size_t)(n + 1));
    double *r = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    int status = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            F[i * n + j] = (float)A[i * lda + j];
    /* float Doolittle LU */
    for (int64_t k = 0; k < n && status == 0; ++k) {
        const float p = F[k * n + k];
        if (p == 0.0f) {
            status = -(int)(k + 1);
            break;
        }
        for (int64_t i = k + 1; i < n; ++i)
            F[i * n + k] = F[i * n + k] / p;
        for (int64_t i = k + 1; i < n; ++i) {
            const float l = F[i * n + k];
            for (int64_t j = k + 1; j < n; ++j)
                F[i * n + j] = F[i * n + j] - l * F[k * n + j];
        }
    }
    int notconv = 0;
    for (int64_t c = 0; c < nrhs && status == 0; ++c) {
        double bmax = 0.0;
        for (int64_t i = 0; i < n; ++i)
            bmax = fmax(bmax, fabs(B[i * ldb + c]));
        /* x0 = solve32(b) */
        for (int64_t i = 0; i < n; ++i)
            r32[i] = (float)B[i * ldb + c];
        for (int it = 0;; ++it) {
            /* float forward / backward substitution on r32 */
            for (int64_t i = 0; i < n; ++i) {
                float s = r32[i];
                for (int64_t j = 0; j < i; ++j)
                    s = s - F[i * n + j] * r32[j];
                r32[i] = s;
            }
            for (int64_t i = n - 1; i >= 0; --i) {
                float s = r32[i];
                for (int64_t j = i + 1; j < n; ++j)
                    s = s - F[i * n + j] * r32[j];
                r32[i] = s / F[i * n + i];
            }
            for (int64_t i = 0; i < n; ++i)
                X[i * ldx + c] = (it == 0) ? (double)r32[i] : X[i * ldx + c] + (double)r32[i];
            /* double residual */
            double rmax = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double s = B[i * ldb + c];
                for (int64_t j = 0; j < n; ++j)
                    s = s - A[i * lda + j] * X[j * ldx + c];
                r[i] = s;
                rmax = fmax(rmax, fabs(s));
            }
            const double rel = (bmax > 0.0) ? rmax / bmax : rmax;
            relres[c] = rel;
            iters[c] = it;
            if (rel <= tol)
                break;
            if (it >= max_iter) {
                notconv = 1;
                break;
            }
            for (int64_t i = 0; i < n; ++i)
                r32[i] = (float)r[i];
        }
    }
    free(F);
    free(r32);
    free(r);
    return (status != 0) ? status : notconv;
}
