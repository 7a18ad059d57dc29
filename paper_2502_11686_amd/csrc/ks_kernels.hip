// ks_kernels.hip -- gfx950 kernels of the odd-even Kalman smoother.
//
// Forward (Section III): one launch per level l.  The level-l system has N_l
// block columns; column j carries an observation-like block (O_j | w_j) and,
// for j >= 1, an evolution-like block (E-_j, E+_j | eta_j) encoding
// E-_j u_{j-1} + E+_j u_j ~ eta_j.  At level 0 these are the whitened inputs
// O = W G, E- = -V F, E+ = V H, eta = V c (Section III, whitening of
// Section II-A).  One "unit" owns the even column j = 2t and its right
// neighbour j+1 and performs, in registers,
//   step 1: QR of [O_j ; E-_{j+1}] applied to [0 ; E+_{j+1}] and the rhs
//           (the paper's QR of [C_i ; -B_{i+1}] producing R~_j, fill X_j, D~_{j+1})
//   step 3: QR of [D~_{j+1} ; O_{j+1}] -> observation block of reduced column t
//   step 2: QR of [E+_j ; R~_j] applied to [E-_j, 0 ; 0, X_j] and the rhs
//           (the paper's QR of [D_i ; R~_i]) -> the permanent block row of R
//           (R_jj, R_j,j+1, rho_j, R_j,j-1) and the reduced evolution block
//           (Z_j, X~_j | zeta_j) of reduced column t.
// When N_l is odd the last (even) column has no right neighbour: the last unit
// also eliminates it, and its Z rows, which touch only column N_l - 2, are
// stacked into that unit's step-3 QR.  A level with one column is the base
// case: QR of its observation block.
//
// Backward: one launch per level, L down to 0.  For each block row of level l
// (original column i, neighbours a = i - 2^l and b = i + 2^l) the kernel forms
// T = R_ii^{-1} [R_ia R_ib], y_i = R_ii^{-1} rho_i - T [y_a ; y_b]
// (Section III-A) and, for Algorithm 2, S_iI = -T S_II and
// S_ii = R_ii^{-1} R_ii^{-T} - S_iI T^T (returned symmetrized).
//
// Mapping to CDNA4: a unit is a group of G lanes (G = 16/32/64 >= 3n+1) inside
// one 64-wide wavefront.  Lane g of the group owns one column of every stack:
//   g in [0, n)      columns of u_j        ("cur")
//   g in [n, 2n)     columns of u_{j+1}    ("right")
//   g == 2n          the right-hand side   ("rhs")
//   g in (2n, 3n]    columns of u_{j-1}    ("left")
// so a Householder reflector needs no reduction: the pivot lane forms it from
// its own column and broadcasts it with ds_bpermute, and every lane updates
// its own column.  Stacks live in VGPRs with every row index a compile-time
// constant.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ks_internal.h"

namespace ks {

enum Role { CUR = 0, RIGHT = 1, RHS = 2, LEFT = 3, IDLE = 4 };

template <int N>
struct Geo {
    static constexpr int COLS = 3 * N + 1;
    static constexpr int G = COLS <= 16 ? 16 : (COLS <= 32 ? 32 : 64);
    static constexpr int UPB = kBlock / G;          // units per workgroup
    static constexpr int RREC = N * (3 * N + 1);    // R-row record
    static constexpr int OREC = N * (N + 1);        // observation block [O | w]
    static constexpr int EREC = N * (2 * N + 1);    // evolution block [E- | E+ | eta]
    static constexpr int SREC = OREC + EREC;        // reduced-system column
    static_assert(COLS <= 64, "state dimension too large for the wavefront family");
};

template <int N>
struct LaneRole {
    int gl, role, rc;
    __device__ explicit LaneRole(int g) : gl(g) {
        if (g < N) { role = CUR; rc = g; }
        else if (g < 2 * N) { role = RIGHT; rc = g - N; }
        else if (g == 2 * N) { role = RHS; rc = 0; }
        else if (g <= 3 * N) { role = LEFT; rc = g - 2 * N - 1; }
        else { role = IDLE; rc = 0; }
    }
};

template <int G>
__device__ __forceinline__ double gbcast(double v, int src) {
    return __shfl(v, src, G);
}

// Householder QR of the first NP columns of a column-distributed stack of H
// rows.  The pivot column p lives on group lane PL0 + p.  Reflector
// P = I - c x' x'^T with x' = (alpha - beta, x_{p+1}, ..., x_{H-1}),
// beta = -sign(alpha) ||x_{p:}||, c = 1 / (beta (beta - alpha)); a column whose
// sub-diagonal part is zero gets the identity.
template <int G, int H, int NP, int PL0>
__device__ __forceinline__ void hqr(double (&x)[H], int gl) {
    constexpr int P = NP < H ? NP : H;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const double alpha = x[p];
        double xn2 = 0.0;
#pragma unroll
        for (int r = p + 1; r < H; ++r) xn2 = fma(x[r], x[r], xn2);
        const bool nz = xn2 != 0.0;
        const double beta = -copysign(sqrt(fma(alpha, alpha, xn2)), alpha);
        const double v0 = alpha - beta;
        const double cc = nz ? 1.0 / (beta * (beta - alpha)) : 0.0;
        const double cb = gbcast<G>(cc, PL0 + p);
        const double v0b = gbcast<G>(v0, PL0 + p);
        double v[H];
#pragma unroll
        for (int r = p + 1; r < H; ++r) v[r] = gbcast<G>(x[r], PL0 + p);
        double w = v0b * x[p];
#pragma unroll
        for (int r = p + 1; r < H; ++r) w = fma(v[r], x[r], w);
        w *= cb;
        const bool piv = gl == PL0 + p;
        x[p] = piv ? (nz ? beta : alpha) : fma(-w, v0b, x[p]);
#pragma unroll
        for (int r = p + 1; r < H; ++r) x[r] = piv ? 0.0 : fma(-w, v[r], x[r]);
    }
}

// Whitening by a dense SPD covariance (Section II-A): rows roff..roff+D-1 of
// every lane's column are replaced by L^{-1} times themselves, where
// Cov = L L^T.  Lane q < D holds column q of Cov in cv; the Cholesky
// factorization runs right-looking over the lanes (each lane keeps its column
// of the symmetric Schur complement, so L(q,p) = cv_q[p] / L(p,p) is local) and
// is fused with the forward substitution, one broadcast column per pivot.
template <int G, int H, int D>
__device__ __forceinline__ void whiten_dense(double (&x)[H], int roff, double (&cv)[D], int gl,
                                             bool &bad) {
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const double piv = cv[p];
        if (gl == p && !(piv > 0.0 && isfinite(piv))) bad = true;
        const double il = 1.0 / sqrt(piv);
        const double ilb = gbcast<G>(il, p);
        double lb[D];
#pragma unroll
        for (int r = p + 1; r < D; ++r) lb[r] = gbcast<G>(cv[r] * il, p);
        const double f = cv[p] * ilb;
#pragma unroll
        for (int r = p + 1; r < D; ++r) cv[r] = fma(-lb[r], f, cv[r]);
        const double xp = x[roff + p] * ilb;
        x[roff + p] = xp;
#pragma unroll
        for (int r = p + 1; r < D; ++r) x[roff + r] = fma(-lb[r], xp, x[roff + r]);
    }
}

// Whitening by a diagonal covariance: row r scaled by 1/sqrt(var_r).  Rows
// r >= dv (padding) are left as they are.
template <int H, int D>
__device__ __forceinline__ void whiten_diag(double (&x)[H], int roff, const double *var, int dv,
                                            bool valid, int gl, bool &bad) {
#pragma unroll
    for (int r = 0; r < D; ++r) {
        const double v = (valid && r < dv) ? var[r] : 1.0;
        if (gl == 0 && !(v > 0.0 && isfinite(v))) bad = true;
        x[roff + r] *= 1.0 / sqrt(v);
    }
}

// ---------------------------------------------------------------- loaders

// observation block of a reduced system column: rows [O | w]
template <int N, int H>
__device__ __forceinline__ void load_obs_sys(double (&x)[H], int roff, const double *obs,
                                             const LaneRole<N> &L, int own, bool valid) {
    const int col = (L.role == own) ? L.rc : (L.role == RHS ? N : -1);
    const bool ld = valid && col >= 0;
#pragma unroll
    for (int r = 0; r < N; ++r) x[roff + r] = ld ? obs[r * (N + 1) + col] : 0.0;
}

// evolution block of a reduced system column: rows [E- | E+ | eta]
template <int N, int H>
__device__ __forceinline__ void load_evol_sys(double (&x)[H], int roff, const double *ev,
                                              const LaneRole<N> &L, int role_m, int role_p,
                                              bool valid) {
    const int col = L.role == role_m ? L.rc
                  : L.role == role_p ? N + L.rc
                  : L.role == RHS    ? 2 * N : -1;
    const bool ld = valid && col >= 0;
#pragma unroll
    for (int r = 0; r < N; ++r) x[roff + r] = ld ? ev[r * (2 * N + 1) + col] : 0.0;
}

// raw observation step j: W_j [G_j | o_j], m rows padded with zero rows to MM
template <int N, int MM, int G, int H>
__device__ __forceinline__ void load_obs_raw(double (&x)[H], int roff, int64_t j,
                                             const LaneRole<N> &L, int own, const FwdArgs &a,
                                             bool valid, bool &bad) {
    const int m = a.m;
    const int col = (L.role == own) ? L.rc : (L.role == RHS ? N : -1);
    const bool ld = valid && col >= 0;
    const double *Gj = a.G + j * (int64_t)m * N;
    const double *oj = a.o + j * (int64_t)m;
#pragma unroll
    for (int r = 0; r < MM; ++r)
        x[roff + r] = (ld && r < m) ? (col < N ? Gj[r * N + col] : oj[r]) : 0.0;
    if (a.C_diag) {
        whiten_diag<H, MM>(x, roff, a.C + j * (int64_t)m, m, valid, L.gl, bad);
    } else {
        const double *Cj = a.C + j * (int64_t)m * m;
        double cv[MM];
#pragma unroll
        for (int r = 0; r < MM; ++r)
            cv[r] = (valid && L.gl < m && r < m) ? Cj[r * m + L.gl] : (r == L.gl ? 1.0 : 0.0);
        whiten_dense<G, H, MM>(x, roff, cv, L.gl, bad);
    }
}

// raw evolution step i (1..k): V_i [-F_i | H_i | c_i]; zero block when !valid
template <int N, int G, int H>
__device__ __forceinline__ void load_evol_raw(double (&x)[H], int roff, int64_t i,
                                              const LaneRole<N> &L, int role_m, int role_p,
                                              const FwdArgs &a, bool valid, bool &bad) {
    const int64_t t = i - 1;  // ABI entry of step i
    const double *F = a.F + t * N * N;
    const double *Hm = a.H ? a.H + t * N * N : nullptr;
    const double *c = a.c + t * N;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double v = 0.0;
        if (valid) {
            if (L.role == role_m) v = -F[r * N + L.rc];
            else if (L.role == role_p) v = Hm ? Hm[r * N + L.rc] : (r == L.rc ? 1.0 : 0.0);
            else if (L.role == RHS) v = c[r];
        }
        x[roff + r] = v;
    }
    if (a.K_diag) {
        whiten_diag<H, N>(x, roff, a.K + t * N, N, valid, L.gl, bad);
    } else {
        const double *Kt = a.K + t * N * N;
        double cv[N];
#pragma unroll
        for (int r = 0; r < N; ++r)
            cv[r] = (valid && L.gl < N) ? Kt[r * N + L.gl] : (r == L.gl ? 1.0 : 0.0);
        whiten_dense<G, H, N>(x, roff, cv, L.gl, bad);
    }
}

// ------------------------------------------------------ shared epilogues

template <int N, int H>
__device__ __forceinline__ void diag_stats(const double (&x)[H], const LaneRole<N> &L, bool valid,
                                           double &dmin, double &dmax, bool &nonfinite) {
    if (!valid || L.role != CUR) return;
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r)
        if (L.rc == r) d = fabs(x[r]);
    if (!isfinite(d)) nonfinite = true;
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
}

// block-wide min/max of |R_pp| into slots[2*blockIdx], error bits into flags
__device__ __forceinline__ void block_epilogue(double dmin, double dmax, bool bad,
                                               bool nonfinite, double *slots,
                                               unsigned *flags) {
    __shared__ double red[2][kBlock / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        dmin = fmin(dmin, __shfl_xor(dmin, off));
        dmax = fmax(dmax, __shfl_xor(dmax, off));
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = dmin;
        red[1][wave] = dmax;
    }
    if (bad) atomicOr(flags, FLAG_NOT_SPD);
    if (nonfinite) atomicOr(flags, FLAG_NONFINITE);
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[0][0], b = red[1][0];
        for (int w = 1; w < kBlock / 64; ++w) {
            a = fmin(a, red[0][w]);
            b = fmax(b, red[1][w]);
        }
        slots[2 * blockIdx.x] = a;
        slots[2 * blockIdx.x + 1] = b;
    }
}

// R-row record: n rows of [R_jj | R_j,right | rho | R_j,left] = lanes 0..3n
template <int N, int H>
__device__ __forceinline__ void store_rrow(double *rec, const double (&x)[H], int gl, bool valid) {
    if (!valid || gl > 3 * N) return;
#pragma unroll
    for (int r = 0; r < N; ++r) rec[r * (3 * N + 1) + gl] = x[r];
}

// ------------------------------------------------------------- forward level

template <int N, int MM, bool RAW>
__global__ __launch_bounds__(kBlock) void k_forward(FwdArgs a) {
    using GE = Geo<N>;
    constexpr int G = GE::G;
    constexpr int RO = RAW ? MM : N;           // rows of an observation block
    constexpr int HA = RO + N, HB = 2 * RO, HC = 2 * N;
    constexpr int PB = HB < N ? HB : N;        // rows of the step-3 triangle
    const int gl = threadIdx.x % G;
    const int64_t t = (int64_t)blockIdx.x * GE::UPB + threadIdx.x / G;
    const bool valid = t < a.units;
    const LaneRole<N> L(gl);
    const int64_t j = 2 * t;
    const bool fold = valid && (a.Nl & 1) && t == a.units - 1;
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;

    // step 1: [O_j | 0 | w_j ; E-_{j+1} | E+_{j+1} | eta_{j+1}], pivots on cur lanes
    double A[HA];
    if constexpr (RAW) {
        load_obs_raw<N, MM, G>(A, 0, j, L, CUR, a, valid, bad);
        load_evol_raw<N, G>(A, RO, j + 1, L, CUR, RIGHT, a, valid, bad);
    } else {
        const double *rec = a.sys_in + j * GE::SREC;
        load_obs_sys<N>(A, 0, rec, L, CUR, valid);
        load_evol_sys<N>(A, RO, rec + GE::SREC + GE::OREC, L, CUR, RIGHT, valid);
    }
    hqr<G, HA, N, 0>(A, gl);

    // step 3: [D~_{j+1} | gamma ; O_{j+1} | w_{j+1}], pivots on right lanes
    double B[HB];
#pragma unroll
    for (int r = 0; r < RO; ++r) B[r] = A[N + r];
    if constexpr (RAW) {
        load_obs_raw<N, MM, G>(B, RO, j + 1, L, RIGHT, a, valid, bad);
    } else {
        load_obs_sys<N>(B, RO, a.sys_in + (j + 1) * GE::SREC, L, RIGHT, valid);
    }
    hqr<G, HB, N, N>(B, gl);
    double Onew[N];
#pragma unroll
    for (int r = 0; r < N; ++r) Onew[r] = r < PB ? B[r] : 0.0;

    // step 2: [E+_j | 0 | eta_j | E-_j ; R~_j | X_j | rho~_j | 0], pivots on cur lanes
    double Cs[HC];
    if constexpr (RAW) {
        load_evol_raw<N, G>(Cs, 0, j, L, LEFT, CUR, a, valid && j >= 1, bad);
    } else {
        load_evol_sys<N>(Cs, 0, a.sys_in + j * GE::SREC + GE::OREC, L, LEFT, CUR, valid && j >= 1);
    }
#pragma unroll
    for (int r = 0; r < N; ++r) Cs[N + r] = A[r];
    hqr<G, HC, N, 0>(Cs, gl);
    store_rrow<N>(a.rrows + t * GE::RREC, Cs, gl, valid);
    diag_stats<N>(Cs, L, valid, dmin, dmax, nonfinite);
    // reduced column t, evolution block (Z_j | X~_j | zeta_j) from the bottom of step 2
    if (valid) {
        const int ec = L.role == LEFT ? L.rc
                     : L.role == RIGHT ? N + L.rc
                     : L.role == RHS ? 2 * N : -1;
        if (ec >= 0) {
            double *rec = a.sys_out + t * GE::SREC + GE::OREC;
#pragma unroll
            for (int r = 0; r < N; ++r) rec[r * (2 * N + 1) + ec] = Cs[N + r];
        }
    }

    if (fold) {
        // the last column jl = N_l - 1 (even, no right neighbour)
        const int64_t jl = a.Nl - 1;
        double A2[RO];
        if constexpr (RAW) {
            load_obs_raw<N, MM, G>(A2, 0, jl, L, CUR, a, true, bad);
        } else {
            load_obs_sys<N>(A2, 0, a.sys_in + jl * GE::SREC, L, CUR, true);
        }
        hqr<G, RO, N, 0>(A2, gl);
        double C2[HC];
        if constexpr (RAW) {
            load_evol_raw<N, G>(C2, 0, jl, L, LEFT, CUR, a, true, bad);
        } else {
            load_evol_sys<N>(C2, 0, a.sys_in + jl * GE::SREC + GE::OREC, L, LEFT, CUR, true);
        }
#pragma unroll
        for (int r = 0; r < N; ++r) C2[N + r] = r < RO ? A2[r] : 0.0;
        hqr<G, HC, N, 0>(C2, gl);
        store_rrow<N>(a.rrows + (t + 1) * GE::RREC, C2, gl, true);
        diag_stats<N>(C2, L, true, dmin, dmax, nonfinite);
        // Z rows (left lanes) move onto the right lanes; rhs keeps zeta
        const int src = (L.role == RIGHT) ? gl + N + 1 : gl;
        double B2[2 * N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const double z = __shfl(C2[N + r], src, G);
            B2[r] = Onew[r];
            B2[N + r] = (L.role == RIGHT || L.role == RHS) ? z : 0.0;
        }
        hqr<G, 2 * N, N, N>(B2, gl);
#pragma unroll
        for (int r = 0; r < N; ++r) Onew[r] = B2[r];
    }

    // reduced column t, observation block from step 3 (with the fold, if any)
    if (valid) {
        const int oc = L.role == RIGHT ? L.rc : (L.role == RHS ? N : -1);
        if (oc >= 0) {
            double *rec = a.sys_out + t * GE::SREC;
#pragma unroll
            for (int r = 0; r < N; ++r) rec[r * (N + 1) + oc] = Onew[r];
        }
    }
    block_epilogue(dmin, dmax, bad, nonfinite, a.slots, a.flags);
}

// base case: a level with a single column; R = triangular factor of its
// observation block (Section III, recursion end; Algorithm 2, one column)
template <int N, int MM, bool RAW>
__global__ __launch_bounds__(kBlock) void k_base(FwdArgs a) {
    using GE = Geo<N>;
    constexpr int G = GE::G;
    constexpr int RO = RAW ? MM : N;
    const int gl = threadIdx.x % G;
    const bool valid = threadIdx.x < G;
    const LaneRole<N> L(gl);
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    double A[RO];
    if constexpr (RAW) {
        load_obs_raw<N, MM, G>(A, 0, 0, L, CUR, a, valid, bad);
    } else {
        load_obs_sys<N>(A, 0, a.sys_in, L, CUR, valid);
    }
    hqr<G, RO, N, 0>(A, gl);
    double R[N];
#pragma unroll
    for (int r = 0; r < N; ++r) R[r] = (r < RO && (L.role == CUR || L.role == RHS)) ? A[r] : 0.0;
    store_rrow<N>(a.rrows, R, gl, valid);
    diag_stats<N>(R, L, valid, dmin, dmax, nonfinite);
    block_epilogue(dmin, dmax, bad, nonfinite, a.slots, a.flags);
}

// ------------------------------------------------------------ backward level

__device__ __forceinline__ int64_t rec_of(int64_t x, const int64_t *rec_off) {
    const int l = __builtin_ctzll((unsigned long long)(x + 1));
    return rec_off[l] + ((x + 1) >> (l + 1));
}

template <int N, bool DO_Y, bool DO_COV>
struct BwdSmem {
    static constexpr int RR = N * (3 * N + 1);
    static constexpr int YI = 2 * N;
    static constexpr int SI = DO_COV ? 4 * N * N : 0;
    static constexpr int TT = N * (2 * N + 1);
    static constexpr int RI = DO_COV ? N * N : 0;
    static constexpr int PP = DO_COV ? 2 * N * N : 0;
    static constexpr int SS = DO_COV ? N * N : 0;
    static constexpr int PER = RR + YI + SI + TT + RI + PP + SS;
};

template <int N, bool DO_Y, bool DO_COV>
__global__ __launch_bounds__(kBlock) void k_backward(BwdArgs a) {
    using GE = Geo<N>;
    using SM = BwdSmem<N, DO_Y, DO_COV>;
    constexpr int G = GE::G;
    constexpr int W = 3 * N + 1;      // R-row width
    constexpr int TW = 2 * N + 1;     // T columns: [T+ | z | T-]
    __shared__ double smem[GE::UPB * SM::PER];
    const int gl = threadIdx.x % G;
    const int ui = threadIdx.x / G;
    const int64_t t = (int64_t)blockIdx.x * GE::UPB + ui;
    const bool valid = t < a.units;
    const int l = a.level;
    const int64_t i = ((2 * t + 1) << l) - 1;
    const int64_t aa = i - ((int64_t)1 << l), bb = i + ((int64_t)1 << l);
    const bool va = valid && aa >= 0, vb = valid && bb <= a.k;

    double *Rr = smem + ui * SM::PER;
    double *yI = Rr + SM::RR;
    double *SII = yI + SM::YI;
    double *TT = SII + SM::SI;
    double *RI = TT + SM::TT;
    double *PP = RI + SM::RI;
    double *SS = PP + SM::PP;

    // stage the record and the neighbour data
    const double *rec = a.rrows_all + (a.rec_off[l] + t) * GE::RREC;
    for (int e = gl; e < SM::RR; e += G) Rr[e] = valid ? rec[e] : (e % (W + 1) == 0 ? 1.0 : 0.0);
    if constexpr (DO_Y) {
        for (int e = gl; e < 2 * N; e += G) {
            const bool left = e < N;
            const int64_t src = left ? aa : bb;
            yI[e] = (left ? va : vb) ? a.u_in[src * N + (left ? e : e - N)] : 0.0;
        }
    }
    if constexpr (DO_COV) {
        // S_II = [S_aa S_ab ; S_ab^T S_bb] (row-major 2n x 2n)
        const double *sab = nullptr;
        bool trans = false;
        if (va && vb) {
            const int la = __builtin_ctzll((unsigned long long)(aa + 1));
            if (la == l + 1) {
                sab = a.spm + (rec_of(aa, a.rec_off) - a.spm_first) * 2 * N * N + N * N;  // S_a,b
            } else {
                sab = a.spm + (rec_of(bb, a.rec_off) - a.spm_first) * 2 * N * N;          // S_b,a
                trans = true;
            }
        }
        for (int e = gl; e < 4 * N * N; e += G) {
            const int r = e / (2 * N), c = e % (2 * N);
            double v = 0.0;
            if (r < N && c < N) {
                if (va) v = a.cov[aa * N * N + r * N + c];
            } else if (r >= N && c >= N) {
                if (vb) v = a.cov[bb * N * N + (r - N) * N + (c - N)];
            } else if (sab) {
                const int rr = r < N ? r : c, cc = r < N ? c - N : r - N;  // S_ab(rr, cc)
                v = trans ? sab[cc * N + rr] : sab[rr * N + cc];
            }
            SII[e] = v;
        }
    }
    __syncthreads();

    // triangular solves with R_ii: lanes < n -> columns of R_ii^{-1},
    // lanes n..3n -> T+ columns, z = R_ii^{-1} rho, T- columns
    if (gl < W && (DO_COV || gl >= N)) {
        double x[N];
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] = gl < N ? (r == gl ? 1.0 : 0.0) : Rr[r * W + gl];
#pragma unroll
        for (int r = N - 1; r >= 0; --r) {
            double acc = x[r];
#pragma unroll
            for (int s = r + 1; s < N; ++s) acc = fma(-Rr[r * W + s], x[s], acc);
            x[r] = acc / Rr[r * W + r];
        }
        if (gl < N) {
#pragma unroll
            for (int r = 0; r < N; ++r) RI[r * N + gl] = x[r];
        } else {
#pragma unroll
            for (int r = 0; r < N; ++r) TT[r * TW + (gl - N)] = x[r];
        }
    }
    __syncthreads();

    // T_I(r, d) for I = (a, b): d < n -> T-, else T+
    auto TI = [&](int r, int d) -> double {
        return d < N ? TT[r * TW + N + 1 + d] : TT[r * TW + (d - N)];
    };

    if constexpr (DO_Y) {
        if (valid && gl < N) {
            double y = TT[gl * TW + N];
#pragma unroll
            for (int d = 0; d < 2 * N; ++d) y = fma(-TI(gl, d), yI[d], y);
            a.u_out[i * N + gl] = y;
        }
    }

    if constexpr (DO_COV) {
        // P = T_I S_II; S_iI = -P
        if (gl < 2 * N) {
            double p[N];
#pragma unroll
            for (int r = 0; r < N; ++r) p[r] = 0.0;
#pragma unroll
            for (int d = 0; d < 2 * N; ++d) {
                const double s = SII[d * 2 * N + gl];
#pragma unroll
                for (int r = 0; r < N; ++r) p[r] = fma(TI(r, d), s, p[r]);
            }
#pragma unroll
            for (int r = 0; r < N; ++r) PP[r * 2 * N + gl] = p[r];
            if (valid && a.store_s) {
                const int64_t ri = a.rec_off[l] + t - a.spm_first;
                double *dst = a.spm + ri * 2 * N * N + (gl < N ? 0 : N * N);
                const int c = gl < N ? gl : gl - N;
#pragma unroll
                for (int r = 0; r < N; ++r) dst[r * N + c] = -p[r];
            }
        }
        __syncthreads();
        // S_ii = R^{-1} R^{-T} + P T_I^T
        if (gl < N) {
            double s[N];
#pragma unroll
            for (int r = 0; r < N; ++r) s[r] = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const double rc = RI[gl * N + q];
#pragma unroll
                for (int r = 0; r < N; ++r) s[r] = fma(RI[r * N + q], rc, s[r]);
            }
#pragma unroll
            for (int d = 0; d < 2 * N; ++d) {
                const double tc = TI(gl, d);
#pragma unroll
                for (int r = 0; r < N; ++r) s[r] = fma(PP[r * 2 * N + d], tc, s[r]);
            }
#pragma unroll
            for (int r = 0; r < N; ++r) SS[r * N + gl] = s[r];
        }
        __syncthreads();
        if (valid && gl < N) {
#pragma unroll
            for (int r = 0; r < N; ++r)
                a.cov[i * N * N + r * N + gl] = 0.5 * (SS[r * N + gl] + SS[gl * N + r]);
        }
    }
}

// ----------------------------------------------------------------- status

__global__ void k_clear_flags(unsigned *flags) {
    if (threadIdx.x == 0) flags[0] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_status(const double *slots, int64_t nslots,
                                                   unsigned *flags) {
    __shared__ double red[2][kBlock];
    double lo = INFINITY, hi = 0.0;
    for (int64_t s = threadIdx.x; s < nslots; s += kBlock) {
        lo = fmin(lo, slots[2 * s]);
        hi = fmax(hi, slots[2 * s + 1]);
    }
    red[0][threadIdx.x] = lo;
    red[1][threadIdx.x] = hi;
    __syncthreads();
    for (int off = kBlock / 2; off >= 1; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + off]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double dmin = red[0][0], dmax = red[1][0];
        if (!(dmin > 64.0 * 2.220446049250313e-16 * dmax)) atomicOr(flags, FLAG_RANK);
    }
}

void launch_clear_flags(unsigned *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, flags);
}

void launch_status(const double *slots, int64_t nslots, unsigned *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_status, dim3(1), dim3(kBlock), 0, s, slots, nslots, flags);
}

// -------------------------------------------------------------- dispatch

template <int N, int MM, bool RAW>
static void launch_fwd_t(const FwdArgs &a, hipStream_t s) {
    const int64_t blocks = (a.units + Geo<N>::UPB - 1) / Geo<N>::UPB;
    hipLaunchKernelGGL((k_forward<N, MM, RAW>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
}

template <int N, int MM, bool RAW>
static void launch_base_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_base<N, MM, RAW>), dim3(1), dim3(kBlock), 0, s, a);
}

template <int N, bool Y, bool COV>
static void launch_bwd_t(const BwdArgs &a, hipStream_t s) {
    const int64_t blocks = (a.units + Geo<N>::UPB - 1) / Geo<N>::UPB;
    hipLaunchKernelGGL((k_backward<N, Y, COV>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
}

template <int N, int MM>
static constexpr KernelSet make_set() {
    return KernelSet{N,
                     MM,
                     &launch_fwd_t<N, MM, true>,
                     &launch_fwd_t<N, MM, false>,
                     &launch_base_t<N, MM, true>,
                     &launch_base_t<N, MM, false>,
                     &launch_bwd_t<N, true, false>,
                     &launch_bwd_t<N, false, true>,
                     &launch_bwd_t<N, true, true>,
                     Geo<N>::UPB,
                     Geo<N>::UPB};
}

#define KS_SETS(N) make_set<N, (N + 1) / 2>(), make_set<N, N>(), make_set<N, 2 * N>()

static const KernelSet kSets[] = {
    KS_SETS(1), KS_SETS(2), KS_SETS(3), KS_SETS(4), KS_SETS(6), KS_SETS(8),
};

const KernelSet *find_kernels(int n, int m) {
    const KernelSet *best = nullptr;
    for (const KernelSet &s : kSets) {
        if (s.n != n || s.mm < (m > 0 ? m : 1)) continue;
        if (!best || s.mm < best->mm) best = &s;
    }
    return best;
}

}  // namespace ks
