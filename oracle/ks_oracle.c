/*
 * ks_oracle.c -- plain, sequential, FP64 reference smoother.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code,
 * header, helper or constant with the GPU library; the two meet only in the
 * seeded inputs.
 *
 * What it computes (Section II-A, eqs. (global-nonlinear-ls) and
 * (nonlinear-generalized-least-squares) with linear F_i, G_i; Section IV):
 *
 *     u_hat   = argmin_u || U (A u - b) ||_2^2,   U^T U = cov(e)^{-1}
 *     Sigma_i = [ (R^T R)^{-1} ]_{ii}             for a thin QR  U A = Q R
 *
 * How:
 *
 *   1. Whitening (Section II-A): V_i^T V_i = K_i^{-1}, W_i^T W_i = C_i^{-1}
 *      with V = L_K^{-1}, W = L_C^{-1} from Cholesky factors K = L_K L_K^T;
 *      diagonal covariances scale rows by 1/sqrt(variance).  The whitened
 *      blocks are B_i = V F_i, D_i = V H_i, c~_i = V c_i, G^_i = W G_i,
 *      o~_i = W o_i (Section III; the paper writes C_i for W G_i).
 *   2. States: the sequential Paige-Saunders ordering of Section II-B.  Over
 *      block columns i = 0..k in natural order, the rows carried in from the
 *      previous column and the whitened observation rows of step i are
 *      triangularized (Householder); then that triangle is stacked over the
 *      whitened evolution rows of step i+1 and column i of the stack is
 *      triangularized.  The first n rows are block row i of R; the rest touch
 *      column i+1 only and are carried on.  Block back-substitution over
 *      the bidiagonal R gives u_hat.
 *   3. Covariances (the quantities of Section IV), by the backward
 *      recursion of the Rauch-Tung-Striebel smoother in square-root
 *      information form over the blocks of R: Sigma_k = R_kk^{-1} R_kk^{-T},
 *      and for i < k the smoother gain M_i = -R_ii^{-1} R_{i,i+1} gives
 *          S_{i,i+1} = M_i Sigma_{i+1},
 *          Sigma_i   = R_ii^{-1} R_ii^{-T} + M_i Sigma_{i+1} M_i^T.
 *      Because R is bidiagonal in the natural order, this is also what the
 *      selected inversion of Section IV reduces to when every column's only
 *      later neighbour is the next one.  Sigma_i is returned symmetrized.
 *   kso_smooth_rts forms the covariances instead without R, by the RTS
 *   recursion in information form written from the model matrices.  The
 *   normal matrix J = A^T cov(e)^{-1} A is block tridiagonal:
 *          J_ii    = H_i^T K_i^{-1} H_i [i >= 1] + F_{i+1}^T K_{i+1}^{-1} F_{i+1} [i < k]
 *                    + G_i^T C_i^{-1} G_i,
 *          J_i,i+1 = -F_{i+1}^T K_{i+1}^{-1} H_{i+1}.
 *   Filter: Lam_0 = J_00, Lam_i = J_ii - N_i^T Lam_{i-1}^{-1} N_i with
 *   N_i = F_i^T K_i^{-1} H_i; Lam_i is the information about u_i from
 *   observations 0..i and evolution steps 1..i+1, so no prior on u_0 is needed
 *   (Section VI).  Smoother: Sigma_k = Lam_k^{-1}, M_i = Lam_i^{-1} N_{i+1},
 *   S_{i,i+1} = M_i Sigma_{i+1}, Sigma_i = Lam_i^{-1} + M_i Sigma_{i+1} M_i^T.
 *   With H = I and Lam_i = P_{i|i}^{-1} + F^T K^{-1} F this is the textbook RTS
 *   smoother (M_i = P_{i|i} F^T P_{i+1|i}^{-1}), also where P_{i|i} does not
 *   exist yet.  It shares no step with the square-root form, so the tests
 *   check the two against each other; it forms J, so its error grows with
 *   cond(J) (the square-root form's with cond(U A) only), which is why the
 *   square-root form is the reference.
 *
 * Householder convention (Golub & Van Loan, Alg. 5.1.1): for x = A[p:,p],
 * beta = -sign(alpha) ||x|| with sign(+0) = +1, tau = (beta - alpha)/beta,
 * v = x / (alpha - beta) with v_0 = 1; a column whose sub-diagonal part is
 * already zero gets tau = 0 (identity).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ks_oracle.h"

/* ---- small dense kernels (row-major) ----------------------------------- */

/* In-place Cholesky A = L L^T of a d x d SPD matrix (lower triangle used).
 * Returns 0, or -1 when a pivot is not positive. */
static int chol_lower(double *a, int d)
{
    for (int j = 0; j < d; ++j) {
        double s = a[j * d + j];
        for (int p = 0; p < j; ++p)
            s -= a[j * d + p] * a[j * d + p];
        if (!(s > 0.0) || !isfinite(s))
            return -1;
        double l = sqrt(s);
        a[j * d + j] = l;
        for (int i = j + 1; i < d; ++i) {
            double t = a[i * d + j];
            for (int p = 0; p < j; ++p)
                t -= a[i * d + p] * a[j * d + p];
            a[i * d + j] = t / l;
        }
    }
    return 0;
}

/* X (d rows, w columns, leading dim ldx) <- L^{-1} X, L lower triangular. */
static void forward_subst(const double *L, int d, double *X, int w, int ldx)
{
    for (int r = 0; r < d; ++r) {
        for (int s = 0; s < r; ++s) {
            double l = L[r * d + s];
            for (int c = 0; c < w; ++c)
                X[r * ldx + c] -= l * X[s * ldx + c];
        }
        double inv = 1.0 / L[r * d + r];
        for (int c = 0; c < w; ++c)
            X[r * ldx + c] *= inv;
    }
}

/* Whiten d rows of X (w columns) by the covariance cov (dense d x d or diagonal
 * d).  work must hold d*d doubles.  Returns 0 or KSO_E_NOT_SPD. */
static int whiten_rows(double *X, int d, int w, int ldx, const double *cov,
                       int diag, double *work)
{
    if (d == 0)
        return 0;
    if (diag) {
        for (int r = 0; r < d; ++r) {
            if (!(cov[r] > 0.0) || !isfinite(cov[r]))
                return KSO_E_NOT_SPD;
            double s = 1.0 / sqrt(cov[r]);
            for (int c = 0; c < w; ++c)
                X[r * ldx + c] *= s;
        }
        return 0;
    }
    memcpy(work, cov, sizeof(double) * (size_t)d * d);
    if (chol_lower(work, d))
        return KSO_E_NOT_SPD;
    forward_subst(work, d, X, w, ldx);
    return 0;
}

/* Householder QR of the leading npiv columns of A (rows x cols, row-major);
 * reflectors are applied to all cols columns and the annihilated entries are
 * set to zero. */
static void householder_qr(double *A, int rows, int cols, int npiv)
{
    for (int p = 0; p < npiv && p < rows; ++p) {
        double alpha = A[p * cols + p];
        double xn2 = 0.0;
        for (int r = p + 1; r < rows; ++r)
            xn2 += A[r * cols + p] * A[r * cols + p];
        if (xn2 == 0.0)
            continue;
        double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        double tau = (beta - alpha) / beta;
        double scal = 1.0 / (alpha - beta);
        for (int r = p + 1; r < rows; ++r)
            A[r * cols + p] *= scal;
        for (int j = p + 1; j < cols; ++j) {
            double w = A[p * cols + j];
            for (int r = p + 1; r < rows; ++r)
                w += A[r * cols + p] * A[r * cols + j];
            w *= tau;
            A[p * cols + j] -= w;
            for (int r = p + 1; r < rows; ++r)
                A[r * cols + j] -= w * A[r * cols + p];
        }
        A[p * cols + p] = beta;
        for (int r = p + 1; r < rows; ++r)
            A[r * cols + p] = 0.0;
    }
}

/* x <- R^{-1} x for upper-triangular R (n x n) and nrhs columns of X (ldx). */
static void back_subst(const double *R, int n, double *X, int nrhs, int ldx)
{
    for (int r = n - 1; r >= 0; --r) {
        for (int s = r + 1; s < n; ++s) {
            double v = R[r * n + s];
            for (int c = 0; c < nrhs; ++c)
                X[r * ldx + c] -= v * X[s * ldx + c];
        }
        double inv = 1.0 / R[r * n + r];
        for (int c = 0; c < nrhs; ++c)
            X[r * ldx + c] *= inv;
    }
}

static int diag_ok(const double *R, int n)
{
    for (int p = 0; p < n; ++p) {
        double d = R[p * n + p];
        if (d == 0.0 || !isfinite(d))
            return 0;
    }
    return 1;
}

/* U A has numerically full column rank when no diagonal entry of R is below
 * 64 eps times the largest one (a rank-deficient problem leaves rounding-level
 * diagonal entries, not exact zeros, once earlier rows have been rotated). */
static int rank_ok(const double *Rd, int64_t k, int n)
{
    double dmax = 0.0;
    for (int64_t i = 0; i <= k; ++i)
        for (int p = 0; p < n; ++p) {
            double d = fabs(Rd[(size_t)i * n * n + p * n + p]);
            dmax = d > dmax ? d : dmax;
        }
    const double tol = 64.0 * 2.220446049250313e-16 * dmax;
    for (int64_t i = 0; i <= k; ++i)
        for (int p = 0; p < n; ++p)
            if (!(fabs(Rd[(size_t)i * n * n + p * n + p]) > tol))
                return 0;
    return 1;
}

/* inv = A^{-1} for a d x d SPD matrix A, through its Cholesky factor
 * (inv = L^{-T} L^{-1}).  work holds d*d doubles.  Returns 0, or -1 when A is
 * not positive definite. */
static int spd_inverse(const double *A, int d, double *inv, double *work)
{
    memcpy(work, A, sizeof(double) * (size_t)d * d);
    if (chol_lower(work, d))
        return -1;
    memset(inv, 0, sizeof(double) * (size_t)d * d);
    for (int r = 0; r < d; ++r)
        inv[r * d + r] = 1.0;
    forward_subst(work, d, inv, d, d); /* inv = L^{-1} */
    for (int r = 0; r < d; ++r)
        for (int s = 0; s < d; ++s) {
            double acc = 0.0;
            for (int q = 0; q < d; ++q)
                acc += inv[q * d + r] * inv[q * d + s];
            work[r * d + s] = acc;
        }
    memcpy(inv, work, sizeof(double) * (size_t)d * d);
    return 0;
}

/* out (cx x cy) = X^T A Y, X: rx x cx, A: rx x rx, Y: rx x cy (row-major). */
static void xt_a_y(const double *X, int rx, int cx, const double *A,
                   const double *Y, int cy, double *out)
{
    for (int a = 0; a < cx; ++a)
        for (int b = 0; b < cy; ++b) {
            double acc = 0.0;
            for (int r = 0; r < rx; ++r)
                for (int q = 0; q < rx; ++q)
                    acc += X[r * cx + a] * A[r * rx + q] * Y[q * cy + b];
            out[a * cy + b] = acc;
        }
}

/* The inverse of a covariance given dense (d x d) or as d variances. */
static int cov_inverse(const double *cov, int d, int diag, double *inv,
                       double *work)
{
    if (!diag)
        return spd_inverse(cov, d, inv, work) ? KSO_E_NOT_SPD : 0;
    memset(inv, 0, sizeof(double) * (size_t)d * d);
    for (int r = 0; r < d; ++r) {
        if (!(cov[r] > 0.0) || !isfinite(cov[r]))
            return KSO_E_NOT_SPD;
        inv[r * d + r] = 1.0 / cov[r];
    }
    return 0;
}

/* Covariance blocks by the information-form RTS recursion from the model
 * matrices (kso_smooth_rts in the header).  Sigma_i -> cov_out (optional), S_{i,i+1} -> lag1_out (optional). */
static int rts_covariances(int64_t k, int n, int m, int K_diag, int C_diag,
                           const double *H, const double *F, const double *K,
                           const double *G, const double *C, double *cov_out,
                           double *lag1_out)
{
    const size_t nn = (size_t)n * n;
    const int dmax = n > m ? n : m;
    int status = KSO_OK;
    double *Linv = malloc(sizeof(double) * nn * (size_t)(k + 1)); /* Lam_i^{-1} */
    double *Mg = malloc(sizeof(double) * nn * (size_t)(k > 0 ? k : 1)); /* M_i */
    double *Nprev = malloc(sizeof(double) * nn); /* N_i of the step into column i */
    double *Nnext = malloc(sizeof(double) * nn);
    double *Lam = malloc(sizeof(double) * nn);
    double *tmp = malloc(sizeof(double) * nn);
    double *Sig = malloc(sizeof(double) * nn);
    double *Snew = malloc(sizeof(double) * nn);
    double *Cov = malloc(sizeof(double) * (size_t)dmax * dmax);
    double *work = malloc(sizeof(double) * (size_t)dmax * dmax);
    double *Ident = malloc(sizeof(double) * nn);
    if (!Linv || !Mg || !Nprev || !Nnext || !Lam || !tmp || !Sig || !Snew || !Cov ||
        !work || !Ident) {
        status = KSO_E_NOMEM;
        goto done;
    }
    memset(Ident, 0, sizeof(double) * nn);
    for (int r = 0; r < n; ++r)
        Ident[r * n + r] = 1.0;

    /* filter */
    for (int64_t i = 0; i <= k; ++i) {
        memset(Lam, 0, sizeof(double) * nn);
        if (m > 0) { /* G_i^T C_i^{-1} G_i */
            const double *Ci = C_diag ? C + (size_t)i * m : C + (size_t)i * m * m;
            if ((status = cov_inverse(Ci, m, C_diag, Cov, work)))
                goto done;
            xt_a_y(G + (size_t)i * m * n, m, n, Cov, G + (size_t)i * m * n, n, tmp);
            for (size_t e = 0; e < nn; ++e)
                Lam[e] += tmp[e];
        }
        if (i >= 1) { /* step i (entry i-1): H_i^T K_i^{-1} H_i - N_i^T M_{i-1} */
            const double *Ki = K_diag ? K + (size_t)(i - 1) * n : K + (size_t)(i - 1) * nn;
            const double *Hi = H ? H + (size_t)(i - 1) * nn : Ident;
            if ((status = cov_inverse(Ki, n, K_diag, Cov, work)))
                goto done;
            xt_a_y(Hi, n, n, Cov, Hi, n, tmp);
            for (size_t e = 0; e < nn; ++e)
                Lam[e] += tmp[e];
            const double *Mp = Mg + (size_t)(i - 1) * nn;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    double acc = 0.0;
                    for (int q = 0; q < n; ++q)
                        acc += Nprev[q * n + a] * Mp[q * n + b];
                    Lam[a * n + b] -= acc;
                }
        }
        if (i < k) { /* step i+1 (entry i): F_{i+1}^T K^{-1} F_{i+1}, N_{i+1} */
            const double *Kn = K_diag ? K + (size_t)i * n : K + (size_t)i * nn;
            const double *Fn = F + (size_t)i * nn;
            const double *Hn = H ? H + (size_t)i * nn : Ident;
            if ((status = cov_inverse(Kn, n, K_diag, Cov, work)))
                goto done;
            xt_a_y(Fn, n, n, Cov, Fn, n, tmp);
            for (size_t e = 0; e < nn; ++e)
                Lam[e] += tmp[e];
            xt_a_y(Fn, n, n, Cov, Hn, n, Nnext);
        }
        for (int a = 0; a < n; ++a) /* symmetric by construction up to rounding */
            for (int b = 0; b < a; ++b)
                Lam[a * n + b] = Lam[b * n + a] = 0.5 * (Lam[a * n + b] + Lam[b * n + a]);
        double *Li = Linv + (size_t)i * nn;
        if (spd_inverse(Lam, n, Li, work)) {
            status = KSO_E_RANK;
            goto done;
        }
        if (i < k) { /* M_i = Lam_i^{-1} N_{i+1} */
            double *Mi = Mg + (size_t)i * nn;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) {
                    double acc = 0.0;
                    for (int q = 0; q < n; ++q)
                        acc += Li[a * n + q] * Nnext[q * n + b];
                    Mi[a * n + b] = acc;
                }
            memcpy(Nprev, Nnext, sizeof(double) * nn);
        }
    }

    /* smoother */
    memcpy(Sig, Linv + (size_t)k * nn, sizeof(double) * nn);
    if (cov_out)
        memcpy(cov_out + (size_t)k * nn, Sig, sizeof(double) * nn);
    for (int64_t i = k - 1; i >= 0; --i) {
        const double *Mi = Mg + (size_t)i * nn;
        for (int a = 0; a < n; ++a) /* tmp = S_{i,i+1} = M_i Sigma_{i+1} */
            for (int b = 0; b < n; ++b) {
                double acc = 0.0;
                for (int q = 0; q < n; ++q)
                    acc += Mi[a * n + q] * Sig[q * n + b];
                tmp[a * n + b] = acc;
            }
        if (lag1_out)
            memcpy(lag1_out + (size_t)i * nn, tmp, sizeof(double) * nn);
        const double *Li = Linv + (size_t)i * nn;
        for (int a = 0; a < n; ++a) /* Sigma_i = Lam_i^{-1} + S_{i,i+1} M_i^T */
            for (int b = 0; b < n; ++b) {
                double acc = 0.0;
                for (int q = 0; q < n; ++q)
                    acc += tmp[a * n + q] * Mi[b * n + q];
                Snew[a * n + b] = Li[a * n + b] + acc;
            }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < a; ++b)
                Snew[a * n + b] = Snew[b * n + a] = 0.5 * (Snew[a * n + b] + Snew[b * n + a]);
        if (cov_out)
            memcpy(cov_out + (size_t)i * nn, Snew, sizeof(double) * nn);
        memcpy(Sig, Snew, sizeof(double) * nn);
    }

done:
    free(Linv); free(Mg); free(Nprev); free(Nnext); free(Lam); free(tmp);
    free(Sig); free(Snew); free(Cov); free(work); free(Ident);
    return status;
}

/* ---- the smoother ------------------------------------------------------- */

static int smooth_impl(int64_t k, int n, int m, int K_diag, int C_diag,
                       const double *H, const double *F, const double *c,
                       const double *K, const double *G, const double *o,
                       const double *C, double *u_out, double *cov_out,
                       double *lag1_out, double *resid2_out, int cov_by_rts)
{
    if (k < 0 || n < 1 || m < 0 || !u_out)
        return KSO_E_ARG;
    if (k > 0 && (!F || !c || !K))
        return KSO_E_ARG;
    if (m > 0 && (!G || !o || !C))
        return KSO_E_ARG;

    const size_t nn = (size_t)n * n;
    const int w1 = n + 1, w2 = 2 * n + 1;
    const int dmax = n > m ? n : m;
    int status = KSO_OK;

    double *Rd = malloc(sizeof(double) * nn * (size_t)(k + 1));       /* R_ii      */
    double *Rs = malloc(sizeof(double) * nn * (size_t)(k > 0 ? k : 1)); /* R_{i,i+1} */
    double *rho = malloc(sizeof(double) * (size_t)n * (size_t)(k + 1));
    double *S1 = malloc(sizeof(double) * (size_t)(n + m) * w1);
    double *S2 = malloc(sizeof(double) * (size_t)(2 * n) * w2);
    double *P = malloc(sizeof(double) * (size_t)n * w1);
    double *work = malloc(sizeof(double) * (size_t)dmax * dmax);
    double *T = malloc(sizeof(double) * nn);
    double *Ri = malloc(sizeof(double) * nn);
    double *Snext = malloc(sizeof(double) * nn);
    double *Sij = malloc(sizeof(double) * nn);
    double *Sjj = malloc(sizeof(double) * nn);
    if (!Rd || !Rs || !rho || !S1 || !S2 || !P || !work || !T || !Ri || !Snext ||
        !Sij || !Sjj) {
        status = KSO_E_NOMEM;
        goto done;
    }

    double resid2 = 0.0;
    int p = 0; /* rows carried in P */
    for (int64_t i = 0; i <= k; ++i) {
        /* S1 = [P_i ; G^_i | o~_i] */
        int rows1 = p + m;
        memcpy(S1, P, sizeof(double) * (size_t)p * w1);
        for (int r = 0; r < m; ++r) {
            memcpy(S1 + (size_t)(p + r) * w1, G + ((size_t)i * m + r) * n, sizeof(double) * n);
            S1[(size_t)(p + r) * w1 + n] = o[(size_t)i * m + r];
        }
        const double *Ci = C_diag ? C + (size_t)i * m : C + (size_t)i * m * m;
        if (m && (status = whiten_rows(S1 + (size_t)p * w1, m, w1, w1, Ci, C_diag, work)))
            goto done;
        householder_qr(S1, rows1, w1, n);
        int rt = rows1 < n ? rows1 : n;
        for (int r = rt; r < rows1; ++r)
            resid2 += S1[r * w1 + n] * S1[r * w1 + n];

        if (i < k) {
            /* S2 = [R~_i, 0, rho~_i ; -B_{i+1}, D_{i+1}, c~_{i+1}] */
            int rows2 = rt + n;
            for (int r = 0; r < rt; ++r) {
                double *row = S2 + (size_t)r * w2;
                memcpy(row, S1 + (size_t)r * w1, sizeof(double) * n);
                memset(row + n, 0, sizeof(double) * n);
                row[2 * n] = S1[r * w1 + n];
            }
            const double *Fi = F + (size_t)i * nn; /* entry i is step i+1 */
            for (int r = 0; r < n; ++r) {
                double *row = S2 + (size_t)(rt + r) * w2;
                for (int s = 0; s < n; ++s) {
                    row[s] = -Fi[r * n + s];
                    row[n + s] = H ? H[(size_t)i * nn + r * n + s] : (r == s ? 1.0 : 0.0);
                }
                row[2 * n] = c[(size_t)i * n + r];
            }
            const double *Ki = K_diag ? K + (size_t)i * n : K + (size_t)i * nn;
            if ((status = whiten_rows(S2 + (size_t)rt * w2, n, w2, w2, Ki, K_diag, work)))
                goto done;
            householder_qr(S2, rows2, w2, n);
            for (int r = 0; r < n; ++r) {
                memcpy(Rd + (size_t)i * nn + r * n, S2 + (size_t)r * w2, sizeof(double) * n);
                memcpy(Rs + (size_t)i * nn + r * n, S2 + (size_t)r * w2 + n, sizeof(double) * n);
                rho[(size_t)i * n + r] = S2[r * w2 + 2 * n];
            }
            /* the remaining rows touch column i+1 only: they are P_{i+1} */
            for (int r = 0; r < rt; ++r)
                memcpy(P + (size_t)r * w1, S2 + (size_t)(n + r) * w2 + n, sizeof(double) * w1);
            p = rt;
        } else {
            if (rt < n) {
                status = KSO_E_RANK;
                goto done;
            }
            for (int r = 0; r < n; ++r) {
                memcpy(Rd + (size_t)i * nn + r * n, S1 + (size_t)r * w1, sizeof(double) * n);
                rho[(size_t)i * n + r] = S1[r * w1 + n];
            }
        }
        if (!diag_ok(Rd + (size_t)i * nn, n)) {
            status = KSO_E_RANK;
            goto done;
        }
    }
    if (!rank_ok(Rd, k, n)) {
        status = KSO_E_RANK;
        goto done;
    }
    if (resid2_out)
        *resid2_out = resid2;

    /* back-substitution */
    for (int64_t i = k; i >= 0; --i) {
        double *y = u_out + (size_t)i * n;
        memcpy(y, rho + (size_t)i * n, sizeof(double) * n);
        if (i < k) {
            const double *Rsi = Rs + (size_t)i * nn;
            const double *yn = u_out + (size_t)(i + 1) * n;
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s)
                    y[r] -= Rsi[r * n + s] * yn[s];
        }
        back_subst(Rd + (size_t)i * nn, n, y, 1, 1);
    }

    if (!cov_out && !lag1_out)
        goto done;
    if (cov_by_rts) {
        status = rts_covariances(k, n, m, K_diag, C_diag, H, F, K, G, C, cov_out, lag1_out);
        goto done;
    }

    /* square-root RTS recursion over the blocks of R */
    for (int64_t j = k; j >= 0; --j) {
        const double *Rjj = Rd + (size_t)j * nn;
        /* Ri = R_jj^{-1} R_jj^{-T}: invert R_jj then form the Gram product */
        memset(T, 0, sizeof(double) * nn);
        for (int r = 0; r < n; ++r)
            T[r * n + r] = 1.0;
        back_subst(Rjj, n, T, n, n); /* T = R_jj^{-1} */
        for (int r = 0; r < n; ++r)
            for (int s = 0; s < n; ++s) {
                double acc = 0.0;
                for (int q = 0; q < n; ++q)
                    acc += T[r * n + q] * T[s * n + q];
                Ri[r * n + s] = acc;
            }
        if (j == k) {
            memcpy(Sjj, Ri, sizeof(double) * nn);
        } else {
            /* T = R_jj^{-1} R_{j,j+1} */
            memcpy(T, Rs + (size_t)j * nn, sizeof(double) * nn);
            back_subst(Rjj, n, T, n, n);
            /* S_{j,I} = -T S_{I,I} */
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    double acc = 0.0;
                    for (int q = 0; q < n; ++q)
                        acc += T[r * n + q] * Snext[q * n + s];
                    Sij[r * n + s] = -acc;
                }
            /* S_jj = R_jj^{-1} R_jj^{-T} - S_{j,I} T^T */
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    double acc = 0.0;
                    for (int q = 0; q < n; ++q)
                        acc += Sij[r * n + q] * T[s * n + q];
                    Sjj[r * n + s] = Ri[r * n + s] - acc;
                }
            if (lag1_out)
                memcpy(lag1_out + (size_t)j * nn, Sij, sizeof(double) * nn);
        }
        for (int r = 0; r < n; ++r)
            for (int s = 0; s < r; ++s) {
                double a = 0.5 * (Sjj[r * n + s] + Sjj[s * n + r]);
                Sjj[r * n + s] = Sjj[s * n + r] = a;
            }
        if (cov_out)
            memcpy(cov_out + (size_t)j * nn, Sjj, sizeof(double) * nn);
        memcpy(Snext, Sjj, sizeof(double) * nn);
    }

done:
    free(Rd); free(Rs); free(rho); free(S1); free(S2); free(P); free(work);
    free(T); free(Ri); free(Snext); free(Sij); free(Sjj);
    return status;
}

int kso_smooth(int64_t k, int n, int m, int K_diag, int C_diag,
               const double *H, const double *F, const double *c,
               const double *K, const double *G, const double *o,
               const double *C, double *u_out, double *cov_out,
               double *lag1_out, double *resid2_out)
{
    return smooth_impl(k, n, m, K_diag, C_diag, H, F, c, K, G, o, C, u_out,
                       cov_out, lag1_out, resid2_out, 0);
}

int kso_smooth_rts(int64_t k, int n, int m, int K_diag, int C_diag,
                   const double *H, const double *F, const double *c,
                   const double *K, const double *G, const double *o,
                   const double *C, double *u_out, double *cov_out,
                   double *lag1_out, double *resid2_out)
{
    return smooth_impl(k, n, m, K_diag, C_diag, H, F, c, K, G, o, C, u_out,
                       cov_out, lag1_out, resid2_out, 1);
}
