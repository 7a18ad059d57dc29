/*
 * ks_oracle.h -- plain sequential FP64 reference smoother (TEST INFRASTRUCTURE).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
 * it.  Host pointers, row-major, step-major, in the layout below.
 *
 *   H, F   [k][n][n]   entry t is evolution step t+1; H may be NULL (identity)
 *   c      [k][n]
 *   K      [k][n][n] dense, or [k][n] variances when K_diag != 0
 *   G      [k+1][m][n]
 *   o      [k+1][m]
 *   C      [k+1][m][m] dense, or [k+1][m] variances when C_diag != 0
 *
 * Outputs: u_out [k+1][n] (required); cov_out [k+1][n][n] = Sigma_i (optional);
 * lag1_out [k][n][n] = cov(u_i, u_{i+1}) = S_{i,i+1} (optional);
 * resid2_out = squared norm of the whitened least-squares residual (optional).
 *
 * kso_smooth forms the covariance outputs by the RTS recursion in
 * square-root information form over the QR factor R; kso_smooth_rts forms
 * them by the RTS recursion in information form from the model matrices
 * (a cross-check; less accurate when A^T cov(e)^{-1} A is ill conditioned).
 * The states are the same.
 */
#ifndef KS_ORACLE_H
#define KS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KSO_OK = 0,
    KSO_E_ARG = -1,      /* bad dimension or a required NULL pointer      */
    KSO_E_NOT_SPD = -3,  /* a covariance is not symmetric positive definite */
    KSO_E_RANK = -4,     /* U A lacks full column rank                    */
    KSO_E_NOMEM = -9     /* host allocation failed                        */
};

int kso_smooth(int64_t k, int n, int m, int K_diag, int C_diag,
               const double *H, const double *F, const double *c,
               const double *K, const double *G, const double *o,
               const double *C, double *u_out, double *cov_out,
               double *lag1_out, double *resid2_out);
int kso_smooth_rts(int64_t k, int n, int m, int K_diag, int C_diag,
                   const double *H, const double *F, const double *c,
                   const double *K, const double *G, const double *o,
                   const double *C, double *u_out, double *cov_out,
                   double *lag1_out, double *resid2_out);

#ifdef __cplusplus
}
#endif
#endif
