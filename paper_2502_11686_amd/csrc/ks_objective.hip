// ks_objective.hip -- value of the generalized least-squares objective
// || U (A u - b) ||^2 of Section II-A at a given u.
//
// Step i contributes the whitened squared norm of its evolution residual
// H_i u_i - F_i u_{i-1} - c_i (i >= 1, covariance K_i) and of its observation
// residual G_i u_i - o_i (covariance C_i): r^T V^{-1} r = ||L^{-1} r||^2 with
// V = L L^T.  A Gauss-Newton or Levenberg-Marquardt driver (Section II-B)
// compares this value before and after a step; at u = 0 it is ||U b||^2, the
// objective at the current iterate once b holds the nonlinear residuals.
#include "ks_internal.h"
#include "ks_objective.h"

namespace ks {

namespace {

constexpr int kObjThreads = 64;  // one wavefront per time step, one lane per residual row

// ||L^{-1} e||^2 for the residual e (lane r holds e_r, r < d) and covariance V
// (dense d x d row-major, or d variances).  A dense V is factored in LDS by a
// right-looking Cholesky whose column steps also carry out the forward
// substitution L y = e.  Returns the same value in every lane; sets bad when a
// pivot or variance is not positive.
__device__ double whitened_sq(double e, const double *V, bool diag, int d, double *Ls, double *ys,
                              bool &bad) {
    const int r = threadIdx.x;
    if (diag) {
        double y2 = 0.0;
        if (r < d) {
            const double v = V[r];
            if (!(v > 0.0)) bad = true;
            y2 = e * e / v;
        }
        for (int off = 32; off >= 1; off >>= 1) y2 += __shfl_xor(y2, off, kObjThreads);
        return y2;
    }
    for (int idx = r; idx < d * d; idx += kObjThreads) Ls[idx] = V[idx];
    if (r < d) ys[r] = e;
    __syncthreads();
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        const double piv = Ls[j * d + j];
        if (!(piv > 0.0)) bad = true;
        const double s = sqrt(piv);
        const double yj = ys[j] / s;
        acc += yj * yj;
        const bool below = r > j && r < d;
        const double lrj = below ? Ls[r * d + j] / s : 0.0;
        __syncthreads();
        if (below) Ls[r * d + j] = lrj;
        __syncthreads();
        if (below) {
            for (int q = j + 1; q <= r; ++q) Ls[r * d + q] -= lrj * Ls[q * d + j];
            ys[r] -= lrj * yj;
        }
        __syncthreads();
    }
    return acc;
}

__global__ __launch_bounds__(kObjThreads) void k_objective(ObjArgs a) {
    extern __shared__ double sh[];
    const int n = a.n, m = a.m;
    const int dm = n > m ? n : m;
    double *Ls = sh, *ys = sh + dm * dm;
    const int r = threadIdx.x;
    bool bad = false;
    double part = 0.0;
    for (int64_t i = blockIdx.x; i <= a.k; i += gridDim.x) {
        double term = 0.0;
        if (i >= 1) {
            const int64_t t = i - 1;  // evolution entry of step i
            double e = 0.0;
            if (r < n) {
                if (a.u) {
                    const double *ui = a.u + i * n, *up = a.u + t * n;
                    const double *Fr = a.F + (t * n + r) * n;
                    double hu = 0.0, fu = 0.0;
                    if (a.H) {
                        const double *Hr = a.H + (t * n + r) * n;
                        for (int q = 0; q < n; ++q) hu = fma(Hr[q], ui[q], hu);
                    } else {
                        hu = ui[r];
                    }
                    for (int q = 0; q < n; ++q) fu = fma(Fr[q], up[q], fu);
                    e = hu - fu;
                }
                e -= a.c[t * n + r];
            }
            term += whitened_sq(e, a.K + t * (a.K_diag ? n : (int64_t)n * n), a.K_diag, n, Ls, ys, bad);
        }
        if (m > 0) {
            double e = 0.0;
            if (r < m) {
                if (a.u) {
                    const double *Gr = a.G + (i * m + r) * n, *ui = a.u + i * n;
                    for (int q = 0; q < n; ++q) e = fma(Gr[q], ui[q], e);
                }
                e -= a.o[i * m + r];
            }
            term += whitened_sq(e, a.C + i * (a.C_diag ? m : (int64_t)m * m), a.C_diag, m, Ls, ys, bad);
        }
        if (r == 0 && a.terms) a.terms[i] = term;
        part += term;
        __syncthreads();  // the next step reuses Ls and ys
    }
    if (r == 0) a.partial[blockIdx.x] = part;
    if (bad) atomicOr(a.flags, FLAG_NOT_SPD);
}

// Fixed-order sum of the per-block partials (the total does not depend on timing).
__global__ __launch_bounds__(256) void k_objective_sum(double *partial, int count) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < count; b += 256) acc += partial[b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[count] = s[0];
}

}  // namespace

int objective_blocks(int64_t k) { return (int)(k + 1 < kObjBlocks ? k + 1 : kObjBlocks); }

void launch_objective(const ObjArgs &a, hipStream_t s) {
    const int blocks = objective_blocks(a.k);
    const int dm = a.n > a.m ? a.n : a.m;
    const size_t lds = sizeof(double) * (size_t)(dm * dm + dm);
    hipLaunchKernelGGL(k_objective, dim3(blocks), dim3(kObjThreads), lds, s, a);
    hipLaunchKernelGGL(k_objective_sum, dim3(1), dim3(256), 0, s, a.partial, blocks);
}

}  // namespace ks
