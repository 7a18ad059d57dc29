#pragma once
// ks_device.h -- gfx950 kernels of the odd-even Kalman smoother (templates;
// instantiated per state dimension by the ks_inst_*.hip translation units).
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
//   step 3: QR of [O_{j+1} ; D~_{j+1}] -> observation block of reduced column t
//   step 2: QR of [E+_j ; R~_j] applied to [E-_j, 0 ; 0, X_j] and the rhs
//           (the paper's QR of [D_i ; R~_i]) -> the permanent block row of R
//           (R_jj, R_j,j+1, rho_j, R_j,j-1) and the reduced evolution block
//           (Z_j, X~_j | zeta_j) of reduced column t.
// Steps 2 and 3 are independent once step 1 is done.  When N_l is odd the last
// (even) column has no right neighbour: the last unit also eliminates it, and
// its Z rows, which touch only column N_l - 2, are stacked into that unit's
// step-3 QR.  A level with one column is the base case: QR of its observation
// block.
//
// Backward: one launch per level, L down to 0.  For each block row of level l
// (original column i, neighbours a = i - 2^l and b = i + 2^l) the kernel forms
// T = R_ii^{-1} [R_ia R_ib], y_i = R_ii^{-1} rho_i - T [y_a ; y_b]
// (Section III-A) and, for Algorithm 2, S_iI = -T S_II and
// S_ii = R_ii^{-1} R_ii^{-T} - S_iI T^T (returned symmetrized).
//
// Mapping to CDNA4: a unit is a group of G = 3n+1 consecutive lanes of one
// 64-wide wavefront (floor(64/G) units per wavefront).  Lane g of the group
// owns one column of every stack:
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

enum Role { CUR = 0, RIGHT = 1, RHS = 2, LEFT = 3, IDLE = 4, BRIGHT = 5, BRHS = 6 };

// Minimum wavefronts per SIMD the forward level kernels are compiled for: at
// n = 6 a unit's stacks need about 130 VGPRs unconstrained (three wavefronts
// per SIMD), at 128 a fourth fits (n = 8 would spill heavily).
constexpr int wf_min_waves(int n) { return n >= 4 && n <= 6 ? 4 : 1; }

template <int N>
struct Geo {
    static constexpr int G = 3 * N + 1;             // lanes per unit
    static constexpr int UPW = 64 / G;              // units per wavefront
    static constexpr int UPB = (kBlock / 64) * UPW; // units per workgroup
    static constexpr int RREC = N * (3 * N + 1);    // R-row record
    static constexpr int OREC = N * (N + 1);        // observation block [O | w]
    static constexpr int EREC = N * (2 * N + 1);    // evolution block [E- | E+ | eta]
    static constexpr int SREC = OREC + EREC;        // reduced-system column
    static_assert(G <= 64, "state dimension too large for the wavefront family");
};

// position of this thread: its unit within the workgroup and its lane in the unit
template <int N>
struct Grp {
    int gl;     // lane within the unit (G for lanes outside any unit)
    int gbase;  // wavefront lane of the unit's lane 0
    int ui;     // unit within the workgroup
    bool in;    // lane belongs to a unit
    __device__ Grp() {
        constexpr int G = Geo<N>::G;
        const int lane = threadIdx.x & 63;
        const int g = lane / G;
        in = g < Geo<N>::UPW;
        gl = in ? lane - g * G : G;
        gbase = in ? g * G : 0;
        ui = (threadIdx.x >> 6) * Geo<N>::UPW + (in ? g : 0);
    }
};

template <int N>
struct LaneRole {
    int role, rc;
    __device__ explicit LaneRole(int g) {
        if (g < N) { role = CUR; rc = g; }
        else if (g < 2 * N) { role = RIGHT; rc = g - N; }
        else if (g == 2 * N) { role = RHS; rc = 0; }
        else if (g <= 3 * N) { role = LEFT; rc = g - 2 * N - 1; }
        else { role = IDLE; rc = 0; }
    }
};

// value of v on wavefront lane src (ds_bpermute, two dwords)
__device__ __forceinline__ double bperm(double v, int src) {
    const int addr = src << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float bperm(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

template <class T>
struct Num;
template <>
struct Num<double> {
    static constexpr double eps = 2.220446049250313e-16;
};
template <>
struct Num<float> {
    static constexpr double eps = 1.1920928955078125e-07;
};

// 1/d and 1/sqrt(d) from the hardware estimates refined by Newton steps
// (two in FP64, one in FP32)
__device__ __forceinline__ float rcp_nr(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(r, fmaf(-d, r, 1.0f), r);
}

__device__ __forceinline__ float rsq_nr(float d) {
    const float r = __builtin_amdgcn_rsqf(d);
    return r * fmaf(-0.5f * d * r, r, 1.5f);
}

__device__ __forceinline__ double rcp_nr(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

__device__ __forceinline__ double rsq_nr(double d) {
    double r = __builtin_amdgcn_rsq(d);
    const double h = 0.5 * d;
    r = r * fma(-h * r, r, 1.5);
    r = r * fma(-h * r, r, 1.5);
    return r;
}

// Householder QR of the first NP columns of a column-distributed stack of H
// rows.  Pivot column p lives on unit lane pl0 + p.  Reflector
// P = I - c x' x'^T with x' = (alpha - beta, x_{p+1}, ..., x_{H-1}),
// beta = -sign(alpha) ||x_{p:}||, c = 1 / (beta (beta - alpha)); a column whose
// sub-diagonal part is zero gets the identity.  Every lane applies the
// reflector to its own column (the pivot lane too); the pivot diagonal is then
// set to beta and, at the end, the strictly lower parts of the pivot columns
// are set to zero.
// TT > 0: rows 0..TT-1 form an upper-triangular block in the pivot columns
// (row r is zero in pivot columns q < r).  Reflector p then has zeros in rows
// p+1..TT-1, and leaves them (and the triangle) as they are, so it is formed
// and applied over rows p and TT..H-1 only: the same reflector as the dense
// loop, with the known zeros skipped.
template <int H, int NP, class T, int TT = 0>
__device__ __forceinline__ void hqr(T (&x)[H], int gl, int gbase, int pl0) {
    constexpr int P = NP < H ? NP : H;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int src = gbase + pl0 + p;
        const int r0 = p + 1 > TT ? p + 1 : TT;  // first row below the pivot that may be nonzero
        const T alpha = x[p];
        T s0 = 0, s1 = 0, sc = 1, am = 1, as = alpha;
        if constexpr (sizeof(T) == 4) {
            // FP32: sum of squares of the column scaled by its largest entry
            // (no overflow or underflow for any representable column)
            am = fabs(alpha);
#pragma unroll
            for (int r = r0; r < H; ++r) am = fmax(am, fabs(x[r]));
            sc = am > T(0) ? rcp_nr(am) : T(0);
            as = alpha * sc;
#pragma unroll
            for (int r = r0; r < H; r += 2) s0 = fma(x[r] * sc, x[r] * sc, s0);
#pragma unroll
            for (int r = r0 + 1; r < H; r += 2) s1 = fma(x[r] * sc, x[r] * sc, s1);
        } else {
#pragma unroll
            for (int r = r0; r < H; r += 2) s0 = fma(x[r], x[r], s0);
#pragma unroll
            for (int r = r0 + 1; r < H; r += 2) s1 = fma(x[r], x[r], s1);
        }
        const T xn2 = s0 + s1;                       // scaled by sc^2 in FP32
        const T s = fma(as, as, xn2);
        const T nrs = sqrt(s);                       // ||x_{p:}|| * sc
        const bool nz = xn2 != T(0);
        const T beta = -copysign(nrs * am, alpha);
        const T cc = nz ? sc * sc * rcp_nr(fma(fabs(as), nrs, s)) : T(0);
        const T v0 = alpha - beta;
        const T dnew = nz ? beta : alpha;
        const T cb = bperm(cc, src);
        const T v0b = bperm(v0, src);
        T v[H];
#pragma unroll
        for (int r = r0; r < H; ++r) v[r] = bperm(x[r], src);
        T w0 = v0b * x[p], w1 = 0;
#pragma unroll
        for (int r = r0; r < H; r += 2) w0 = fma(v[r], x[r], w0);
#pragma unroll
        for (int r = r0 + 1; r < H; r += 2) w1 = fma(v[r], x[r], w1);
        const T w = (w0 + w1) * cb;
        x[p] = (gl == pl0 + p) ? dnew : fma(-w, v0b, x[p]);
#pragma unroll
        for (int r = r0; r < H; ++r) x[r] = fma(-w, v[r], x[r]);
    }
    const unsigned q = (unsigned)(gl - pl0);
#pragma unroll
    for (int r = 1; r < H; ++r)
        if (q < (unsigned)(r < P ? r : P)) x[r] = T(0);
}

// Whitening by a dense SPD covariance (Section II-A): rows roff..roff+D-1 of
// every lane's column are replaced by L^{-1} times themselves, where
// Cov = L L^T.  Unit lane cl0 + q (q < D) holds column q of Cov in cv (other
// lanes hold zeros); the Cholesky factorization runs right-looking over those
// lanes (each keeps its column of the symmetric Schur complement, so
// L(q,p) = cv_q[p] / L(p,p) is local) and is fused with the forward
// substitution, one broadcast column of L per pivot.
template <int H, int D, class T>
__device__ __forceinline__ void whiten_dense(T (&x)[H], int roff, T (&cv)[D], int gl,
                                             int gbase, int cl0, bool &bad) {
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const int src = gbase + cl0 + p;
        const T piv = cv[p];
        if (gl == cl0 + p && !(piv > T(0) && isfinite(piv))) bad = true;
        const T il = rsq_nr(piv);
        const T ilb = bperm(il, src);
        T lb[D];
#pragma unroll
        for (int r = p + 1; r < D; ++r) lb[r] = bperm(cv[r] * il, src);
        const T f = cv[p] * ilb;
#pragma unroll
        for (int r = p + 1; r < D; ++r) cv[r] = fma(-lb[r], f, cv[r]);
        const T xp = x[roff + p] * ilb;
        x[roff + p] = xp;
#pragma unroll
        for (int r = p + 1; r < D; ++r) x[roff + r] = fma(-lb[r], xp, x[roff + r]);
    }
}

// Whitening by a diagonal covariance: row r scaled by 1/sqrt(var_r).
template <int H, int D, class T>
__device__ __forceinline__ void whiten_diag(T (&x)[H], int roff, const T (&var)[D],
                                            int gl, bool &bad) {
#pragma unroll
    for (int r = 0; r < D; ++r) {
        const T v = var[r];
        if (gl == 0 && !(v > T(0) && isfinite(v))) bad = true;
        x[roff + r] *= rsq_nr(v);
    }
}

// ---------------------------------------------------------------- loaders

// observation block of a reduced-system column, rows [O | w], onto owner lanes
template <int N, int H, class LR, class T, class TIN>
__device__ __forceinline__ void load_obs_sys(T (&x)[H], int roff, const TIN *obs,
                                             const LR &L, int own, bool valid, int rhs = RHS) {
    const int col = (L.role == own) ? L.rc : (L.role == rhs ? N : -1);
    // one conditional region for all rows (a select per row would become a
    // branch per row)
    if (valid && col >= 0) {
#pragma unroll
        for (int r = 0; r < N; ++r) x[roff + r] = T(obs[r * (N + 1) + col]);
    } else {
#pragma unroll
        for (int r = 0; r < N; ++r) x[roff + r] = T(0);
    }
}

// evolution block of a reduced-system column, rows [E- | E+ | eta]
template <int N, int H, class LR, class T, class TIN>
__device__ __forceinline__ void load_evol_sys(T (&x)[H], int roff, const TIN *ev,
                                              const LR &L, int role_m, int role_p,
                                              bool valid) {
    const int col = L.role == role_m ? L.rc
                  : L.role == role_p ? N + L.rc
                  : L.role == RHS    ? 2 * N : -1;
    if (valid && col >= 0) {
#pragma unroll
        for (int r = 0; r < N; ++r) x[roff + r] = T(ev[r * (2 * N + 1) + col]);
    } else {
#pragma unroll
        for (int r = 0; r < N; ++r) x[roff + r] = T(0);
    }
}

// Raw observation step j, rows [G_j | o_j] (m rows, zero rows up to MM), and
// the covariance data for its whitening: cv = column (gl - cl0) of C_j on the
// lanes cl0 .. cl0+MM-1 (identity columns for padding rows), or the variances.
template <int N, int MM, int H, class LR, class T>
__device__ __forceinline__ void load_obs_raw(T (&x)[H], int roff, T (&cv)[MM],
                                             int64_t j, const LR &L, int gl, int own,
                                             int cl0, const FwdArgs &a, bool valid,
                                             int rhs = RHS) {
    const int m = a.m;
    const int col = (L.role == own) ? L.rc : (L.role == rhs ? N : -1);
    const bool ld = valid && col >= 0;
    j -= a.col0;
    const double *Gj = a.G + j * (int64_t)m * N;
    const double *oj = a.o + j * (int64_t)m;
    // one conditional region per lane for its loads (m is uniform); the
    // column of G or o is chosen by address
    if (ld) {
        const double *src = col < N ? Gj + col : oj;
        const int stride = col < N ? N : 1;
#pragma unroll
        for (int r = 0; r < MM; ++r) x[roff + r] = r < m ? T(src[r * stride]) : T(0);
    } else {
#pragma unroll
        for (int r = 0; r < MM; ++r) x[roff + r] = T(0);
    }
    if (a.C_diag) {
        const double *Cj = a.C + j * (int64_t)m;
        if (valid) {
#pragma unroll
            for (int r = 0; r < MM; ++r) cv[r] = r < m ? T(Cj[r]) : T(1);
        } else {
#pragma unroll
            for (int r = 0; r < MM; ++r) cv[r] = T(1);
        }
    } else {
        const double *Cj = a.C + j * (int64_t)m * m;
        const int q = gl - cl0;
        const bool mine = (unsigned)q < (unsigned)MM;
        if (mine && valid && q < m) {
#pragma unroll
            for (int r = 0; r < MM; ++r) cv[r] = r < m ? T(Cj[r * m + q]) : T(r == q ? 1 : 0);
        } else {
#pragma unroll
            for (int r = 0; r < MM; ++r) cv[r] = mine ? T(r == q ? 1 : 0) : T(0);
        }
    }
}

// Raw evolution step i (1..k), rows [-F_i | H_i | c_i] (zero block when
// !valid), with its covariance data as in load_obs_raw.
template <int N, int H, class LR, class T>
__device__ __forceinline__ void load_evol_raw(T (&x)[H], int roff, T (&cv)[N], int64_t i,
                                              const LR &L, int gl, int role_m,
                                              int role_p, int cl0, const FwdArgs &a, bool valid) {
    const int64_t t = i - 1 - a.ent0;  // ABI entry of step i (relative to the first one the pointers hold)
    const double *F = a.F + t * N * N;
    const double *Hm = a.H ? a.H + t * N * N : nullptr;
    const double *c = a.c + t * N;
    // the lane's source column (-F, H or c), chosen once; one conditional
    // region holds its loads
    const bool fm = valid && L.role == role_m;
    const bool fh = valid && L.role == role_p && Hm;
    const bool fc = valid && L.role == RHS;
    if (fm || fh || fc) {
        const double *src = fm ? F + L.rc : fh ? Hm + L.rc : c;
        const int stride = fc ? 1 : N;
        const double sgn = fm ? -1.0 : 1.0;
#pragma unroll
        for (int r = 0; r < N; ++r) x[roff + r] = T(sgn * src[r * stride]);
    } else {
        const bool ident = valid && L.role == role_p;  // H = identity
#pragma unroll
        for (int r = 0; r < N; ++r) x[roff + r] = T(ident && r == L.rc ? 1.0 : 0.0);
    }
    if (a.K_diag) {
        const double *Kt = a.K + t * N;
        if (valid) {
#pragma unroll
            for (int r = 0; r < N; ++r) cv[r] = T(Kt[r]);
        } else {
#pragma unroll
            for (int r = 0; r < N; ++r) cv[r] = T(1);
        }
    } else {
        const double *Kt = a.K + t * N * N;
        const int q = gl - cl0;
        const bool mine = (unsigned)q < (unsigned)N;
        if (mine && valid) {
#pragma unroll
            for (int r = 0; r < N; ++r) cv[r] = T(Kt[r * N + q]);
        } else {
#pragma unroll
            for (int r = 0; r < N; ++r) cv[r] = mine ? T(r == q ? 1 : 0) : T(0);
        }
    }
}

template <int H, int D, class T>
__device__ __forceinline__ void whiten(bool diag, T (&x)[H], int roff, T (&cv)[D],
                                       int gl, int gbase, int cl0, bool &bad) {
    if (diag)
        whiten_diag<H, D, T>(x, roff, cv, gl, bad);
    else
        whiten_dense<H, D, T>(x, roff, cv, gl, gbase, cl0, bad);
}

// ------------------------------------------------------ shared epilogues

template <int N, int H, class LR, class T>
__device__ __forceinline__ void diag_stats(const T (&x)[H], const LR &L, bool valid,
                                           double &dmin, double &dmax, bool &nonfinite) {
    if (!valid || L.role != CUR) return;
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r)
        if (L.rc == r) d = fabs(double(x[r]));
    if (!isfinite(d)) nonfinite = true;
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
}

// workgroup min/max of |R_pp| (result valid in thread 0), error bits into flags
template <int TB>
__device__ __forceinline__ void block_minmax(double &dmin, double &dmax, bool bad, bool nonfinite,
                                             unsigned *flags) {
    __shared__ double red[2][TB / 64];
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
#pragma unroll
        for (int w = 1; w < TB / 64; ++w) {
            red[0][0] = fmin(red[0][0], red[0][w]);
            red[1][0] = fmax(red[1][0], red[1][w]);
        }
        dmin = red[0][0];
        dmax = red[1][0];
    }
}

// R-row record: n rows of [R_jj | R_j,right | rho | R_j,left] = lanes 0..3n
template <int N, int H, class T>
__device__ __forceinline__ void store_rrow(T *rec, const T (&x)[H], int gl, bool valid) {
    if (!valid || gl > 3 * N) return;
#pragma unroll
    for (int r = 0; r < N; ++r) rec[r * (3 * N + 1) + gl] = x[r];
}

// Record idx of a segment whose records are `stride` doubles apart; records of
// FP32 levels hold floats in the first half of their slot.
template <class T>
__device__ __forceinline__ T *slot(double *base, int64_t idx, int stride) {
    return reinterpret_cast<T *>(base + idx * stride);
}
template <class T>
__device__ __forceinline__ const T *slot(const double *base, int64_t idx, int stride) {
    return reinterpret_cast<const T *>(base + idx * stride);
}

// ------------------------------------------------------------- forward level

// The last column jl = N_l - 1 of a level with N_l odd (even, no right
// neighbour), in two parts.  fold_col: its R row (record t+1, t the last
// unit) and its Z rows, which touch only column jl - 1, left in the bottom
// rows of C2 (Z on the left lanes, zeta on the rhs lane).  fold_merge: those
// rows stacked under the last unit's step-3 triangle Onew and
// re-triangularized.  Inputs are read through `in` (the level's arguments, or
// a view of them in LDS), results written through `a`.
template <int N, int MM, bool RAW, class T, class TIN>
__device__ __forceinline__ void fold_col(const FwdArgs &a, const FwdArgs &in, int64_t t, int gl, int gb,
                                         const LaneRole<N> &L, T (&C2)[2 * N], double &dmin, double &dmax,
                                         bool &bad, bool &nonfinite) {
    using GE = Geo<N>;
    constexpr int RO = RAW ? MM : N;
    constexpr int HC = 2 * N;
    const int64_t jl = a.Nl - 1;
    // C2 = [R~ (its observation block, triangular) ; E+ | E- | eta]
    T A2[RO];
    if constexpr (RAW) {
        T cvO[MM], cvE[N];
        load_obs_raw<N, MM>(A2, 0, cvO, jl, L, gl, CUR, 0, in, true);
        load_evol_raw<N>(C2, N, cvE, jl, L, gl, LEFT, CUR, 2 * N + 1, in, true);
        whiten<RO, MM>(a.C_diag, A2, 0, cvO, gl, gb, 0, bad);
        whiten<HC, N>(a.K_diag, C2, N, cvE, gl, gb, 2 * N + 1, bad);
        hqr<RO, N>(A2, gl, gb, 0);
    } else {
        // a reduced observation block is already triangular
        const TIN *rec = slot<TIN>(in.sys_in, jl - in.col0, GE::SREC);
        load_obs_sys<N>(A2, 0, rec, L, CUR, true);
        load_evol_sys<N>(C2, N, rec + GE::OREC, L, LEFT, CUR, true);
    }
#pragma unroll
    for (int r = 0; r < N; ++r) C2[r] = r < RO ? A2[r] : T(0);
    hqr<HC, N, T, N>(C2, gl, gb, 0);
    store_rrow<N>(slot<T>(a.rrows, t + 1, GE::RREC), C2, gl, true);
    diag_stats<N>(C2, L, true, dmin, dmax, nonfinite);
}

// Onew <- triangle of [Onew ; Z | zeta] (pivots on the right lanes); z holds
// row r of Z | zeta on the right lanes (column rc) and the rhs lane
template <int N, class T>
__device__ __forceinline__ void fold_merge(T (&Onew)[N], const T (&z)[N], int gl, int gb) {
    T B2[2 * N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        B2[r] = Onew[r];
        B2[N + r] = z[r];
    }
    hqr<2 * N, N, T, N>(B2, gl, gb, N);
#pragma unroll
    for (int r = 0; r < N; ++r) Onew[r] = B2[r];
}

// both parts in one unit's lanes (Z moved to the right lanes by ds_bpermute)
template <int N, int MM, bool RAW, class T, class TIN>
__device__ __forceinline__ void fold_part(const FwdArgs &a, const FwdArgs &in, int64_t t, int gl, int gb,
                                          const LaneRole<N> &L, T (&Onew)[N], double &dmin,
                                          double &dmax, bool &bad, bool &nonfinite) {
    T C2[2 * N];
    fold_col<N, MM, RAW, T, TIN>(a, in, t, gl, gb, L, C2, dmin, dmax, bad, nonfinite);
    // Z rows (left lanes) move onto the right lanes; rhs keeps zeta
    const int src = gb + ((L.role == RIGHT) ? gl + N + 1 : gl);
    T z[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const T v = bperm(C2[N + r], src);
        z[r] = (L.role == RIGHT || L.role == RHS) ? v : T(0);
    }
    fold_merge<N, T>(Onew, z, gl, gb);
}

// One unit of a forward level: even column j = 2t and its right neighbour
// (plus, with INLINE_FOLD, the last column when it is the folding unit; the
// per-level kernels leave that to k_fold).  No workgroup barrier.
template <int N, int MM, bool RAW, bool INLINE_FOLD, class T, class TIN>
__device__ __forceinline__ void fwd_unit(const FwdArgs &a, const FwdArgs &src, int64_t t, bool in, int gl,
                                         int gb, double &dmin, double &dmax, bool &bad, bool &nonfinite,
                                         int64_t t_end = -1, T *keep = nullptr) {
    using GE = Geo<N>;
    constexpr int RO = RAW ? MM : N;            // rows of an observation block
    constexpr int HA = RO + N, HB = 2 * RO, HC = 2 * N;
    constexpr int PB = HB < N ? HB : N;         // rows of the step-3 triangle
    const bool valid = in && t < (t_end < 0 ? a.units : t_end);
    const LaneRole<N> L(gl);
    const int64_t j = 2 * t;
    const bool fold = valid && (a.Nl & 1) && t == a.units - 1;

    // Above level 0:
    //   A = [O_j | 0 | w_j ; E-_{j+1} | E+_{j+1} | eta_{j+1}]      (cur, right, rhs lanes)
    //   B = [O_{j+1} | w_{j+1} ; D~_{j+1} | gamma]                  (right, rhs lanes)
    //   C = [R~_j | X_j | rho~_j | 0 ; E+_j | 0 | eta_j | E-_j]     (cur, right, rhs, left lanes)
    // where the observation blocks O_j, O_{j+1} are triangular (from the level
    // below's step 3) and R~_j is: each stack starts with a triangular block
    // whose known zeros the reflectors skip.  At level 0 (raw, whitened
    // inputs; no triangular observation block) B and C hold the same blocks
    // in the order [D~; O] and [E; R~] with dense reflectors, which keeps the
    // kernel within 128 VGPRs.
    constexpr int OB = RAW ? RO : 0;   // first row of O_{j+1} in B
    constexpr int DB = RAW ? 0 : RO;   // first row of D~_{j+1} in B
    constexpr int EC = RAW ? 0 : N;    // first row of the evolution block in C
    constexpr int RC = RAW ? N : 0;    // first row of R~_j in C
    constexpr int TO = RAW ? 0 : N;
    constexpr int TC = RAW ? 0 : N;
    T A[HA], B[HB], C[HC];
    if constexpr (RAW) {
#pragma unroll
        for (int r = N; r < HC; ++r) C[r] = T(0);
        // each block is loaded and whitened in turn (its covariance data live
        // only that long)
        {
            T cv[MM];
            load_obs_raw<N, MM>(A, 0, cv, j, L, gl, CUR, 0, src, valid);
            whiten<HA, MM>(a.C_diag, A, 0, cv, gl, gb, 0, bad);
        }
        {
            T cv[N];
            load_evol_raw<N>(A, RO, cv, j + 1, L, gl, CUR, RIGHT, 0, src, valid);
            whiten<HA, N>(a.K_diag, A, RO, cv, gl, gb, 0, bad);
        }
        {
            T cv[MM];
            load_obs_raw<N, MM>(B, OB, cv, j + 1, L, gl, RIGHT, N, src, valid);
            whiten<HB, MM>(a.C_diag, B, OB, cv, gl, gb, N, bad);
        }
        {
            T cv[N];
            load_evol_raw<N>(C, EC, cv, j, L, gl, LEFT, CUR, 2 * N + 1, src, valid && j >= 1);
            whiten<HC, N>(a.K_diag, C, EC, cv, gl, gb, 2 * N + 1, bad);
        }
    } else {
        const TIN *rec = slot<TIN>(src.sys_in, j - src.col0, GE::SREC);
        load_obs_sys<N>(A, 0, rec, L, CUR, valid);
        const TIN *rec1 = slot<TIN>(src.sys_in, j + 1 - src.col0, GE::SREC);
        load_evol_sys<N>(A, RO, rec1 + GE::OREC, L, CUR, RIGHT, valid);
        load_obs_sys<N>(B, OB, rec1, L, RIGHT, valid);
        load_evol_sys<N>(C, EC, rec + GE::OREC, L, LEFT, CUR, valid && j >= 1);
    }

    // step 1 (pivots on cur lanes)
    hqr<HA, N, T, TO>(A, gl, gb, 0);
#pragma unroll
    for (int r = 0; r < RO; ++r) B[DB + r] = A[N + r];
#pragma unroll
    for (int r = 0; r < N; ++r) C[RC + r] = A[r];

    // step 3 (pivots on right lanes) and step 2 (pivots on cur lanes)
    hqr<HB, N, T, TO>(B, gl, gb, N);
    hqr<HC, N, T, TC>(C, gl, gb, 0);

    store_rrow<N>(slot<T>(a.rrows, t, GE::RREC), C, gl, valid);
    diag_stats<N>(C, L, valid, dmin, dmax, nonfinite);
    // reduced column t, evolution block (Z_j | X~_j | zeta_j) from the bottom of step 2
    if (valid) {
        const int ec = L.role == LEFT ? L.rc
                     : L.role == RIGHT ? N + L.rc
                     : L.role == RHS ? 2 * N : -1;
        if (ec >= 0) {
            T *rec = slot<T>(a.sys_out, t, GE::SREC) + GE::OREC;
#pragma unroll
            for (int r = 0; r < N; ++r) rec[r * (2 * N + 1) + ec] = C[N + r];
        }
    }
    T Onew[N];
#pragma unroll
    for (int r = 0; r < N; ++r) Onew[r] = r < PB ? B[r] : T(0);

    if (INLINE_FOLD && fold) fold_part<N, MM, RAW, T, TIN>(a, src, t, gl, gb, L, Onew, dmin, dmax, bad, nonfinite);
    if (keep && fold) {
        // the caller folds the last column in (split fold) and stores the block
#pragma unroll
        for (int r = 0; r < N; ++r) keep[r] = Onew[r];
        return;
    }

    // reduced column t, observation block from step 3 (with the fold, if any)
    if (valid) {
        const int oc = L.role == RIGHT ? L.rc : (L.role == RHS ? N : -1);
        if (oc >= 0) {
            T *rec = slot<T>(a.sys_out, t, GE::SREC);
#pragma unroll
            for (int r = 0; r < N; ++r) rec[r * (N + 1) + oc] = Onew[r];
        }
    }
}

// Base case: a level with a single column; R = triangular factor of its
// observation block (Section III, recursion end; Algorithm 2, one column).
template <int N, int MM, bool RAW, class TIN>
__device__ __forceinline__ void base_unit(const FwdArgs &a, bool valid, int gl, int gb,
                                          double &dmin, double &dmax, bool &bad, bool &nonfinite) {
    constexpr int RO = RAW ? MM : N;
    const LaneRole<N> L(gl);
    double A[RO];
    if constexpr (RAW) {
        double cv[MM];
        load_obs_raw<N, MM>(A, 0, cv, 0, L, gl, CUR, 0, a, valid);
        whiten<RO, MM>(a.C_diag, A, 0, cv, gl, gb, 0, bad);
    } else {
        load_obs_sys<N>(A, 0, slot<TIN>(a.sys_in, 0, Geo<N>::SREC), L, CUR, valid);
    }
    if constexpr (RAW) hqr<RO, N>(A, gl, gb, 0);  // a reduced observation block is already triangular
    double R[N];
#pragma unroll
    for (int r = 0; r < N; ++r) R[r] = (r < RO && (L.role == CUR || L.role == RHS)) ? A[r] : 0.0;
    store_rrow<N>(a.rrows, R, gl, valid);
    diag_stats<N>(R, L, valid, dmin, dmax, nonfinite);
}

// min/max of the nprev per-block slots of earlier launches into (dmin, dmax),
// eight independent loads in flight per thread
__device__ __forceinline__ void reduce_slots(const double *slots, int64_t nprev, double &dmin,
                                             double &dmax) {
    for (int64_t s0 = threadIdx.x; s0 < nprev; s0 += 8 * (int64_t)blockDim.x) {
        double lo[8], hi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t s = s0 + (int64_t)u * blockDim.x;
            lo[u] = s < nprev ? slots[2 * s] : INFINITY;
            hi[u] = s < nprev ? slots[2 * s + 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dmin = fmin(dmin, lo[u]);
            dmax = fmax(dmax, hi[u]);
        }
    }
}

__device__ __forceinline__ void rank_flag(double dmin, double dmax, double tol, unsigned *flags) {
    if (threadIdx.x == 0 && !(dmin > tol * dmax))
        atomicOr(flags, FLAG_RANK);
}

// The units of block blk of a forward level.  With FOLD, the workgroup of
// the last unit of an odd level also eliminates the last column: where a
// wavefront after the last unit's is idle, that wavefront factors the last
// column (fold_col) while the units run, and after one barrier the last unit
// merges its Z rows (fold_merge); else the last unit does both in turn.
template <int N, int MM, bool RAW, bool FOLD, class T, class TIN>
__device__ __forceinline__ void fwd_level(const FwdArgs &a, const FwdArgs &src, int64_t blk, const Grp<N> &g,
                                          double &dmin, double &dmax, bool &bad, bool &nonfinite) {
    using GE = Geo<N>;
    const int64_t t = blk * GE::UPB + g.ui;
    if constexpr (!FOLD) {
        fwd_unit<N, MM, RAW, false, T, TIN>(a, src, t, g.in, g.gl, g.gbase, dmin, dmax, bad, nonfinite);
        return;
    }
    const int64_t tl = a.units - 1;
    const bool fold_wg = (a.Nl & 1) && blk == tl / GE::UPB;  // uniform over the workgroup
    const int wl = (int)(tl % GE::UPB) / GE::UPW;           // wavefront of the last unit
    if (!(fold_wg && wl + 1 < kBlock / 64)) {
        fwd_unit<N, MM, RAW, FOLD, T, TIN>(a, src, t, g.in, g.gl, g.gbase, dmin, dmax, bad, nonfinite);
        return;
    }
    __shared__ T zb[N * (N + 1)];  // Z | zeta of the last column, row-major
    T keep[N];
    fwd_unit<N, MM, RAW, false, T, TIN>(a, src, t, g.in, g.gl, g.gbase, dmin, dmax, bad, nonfinite, -1, keep);
    const LaneRole<N> L(g.gl);
    if (g.in && g.ui == (wl + 1) * GE::UPW) {  // first unit slot of the next (idle) wavefront
        T C2[2 * N];
        fold_col<N, MM, RAW, T, TIN>(a, src, tl, g.gl, g.gbase, L, C2, dmin, dmax, bad, nonfinite);
        const int c = L.role == LEFT ? L.rc : (L.role == RHS ? N : -1);
        if (c >= 0) {
#pragma unroll
            for (int r = 0; r < N; ++r) zb[r * (N + 1) + c] = C2[N + r];
        }
    }
    __syncthreads();
    if (g.in && t == tl) {
        const int c = L.role == RIGHT ? L.rc : (L.role == RHS ? N : -1);
        T z[N];
#pragma unroll
        for (int r = 0; r < N; ++r) z[r] = c >= 0 ? zb[r * (N + 1) + c] : T(0);
        fold_merge<N, T>(keep, z, g.gl, g.gbase);
        if (c >= 0) {
            T *rec = slot<T>(a.sys_out, tl, GE::SREC);
#pragma unroll
            for (int r = 0; r < N; ++r) rec[r * (N + 1) + c] = keep[r];
        }
    }
}

// Staging of a workgroup's inputs in LDS.  The workgroup's units read
// columns [J0, J0 + NC) of the level (NC = 2 UPB + 1: two per unit and the
// fold column): consecutive threads copy consecutive words of those columns'
// records (reduced systems) or of their slices of the raw per-step arrays
// (level 0), so every global load is a full, coalesced line; each lane then
// reads its own column's entries from LDS.  Used at level 0 where the copy
// fits in 40 KB (several workgroups per CU): there a unit's inputs are six
// arrays' scattered slices (n = 6: level-0 forward 123 -> 110 us).  Above it
// a unit reads two whole records and the per-lane loads are already close to
// coalesced; the barrier the copy adds made those levels slower.
template <int N, int MM, bool RAW>
struct Stage {
    static constexpr int NC = 2 * Geo<N>::UPB + 1;
    // words per column: raw G, o, C (dense), F, H, c, K (dense); or one record
    static constexpr int PER = RAW ? MM * N + MM + MM * MM + 2 * N * N + N + N * N : Geo<N>::SREC;
    static constexpr int WORDS = NC * PER;
    static constexpr bool ON = RAW && WORDS * 8 <= 40 * 1024;
};

__device__ __forceinline__ void stage_copy(double *dst, const double *src, int64_t count) {
    for (int64_t e = threadIdx.x; e < count; e += kBlock) dst[e] = src[e];
}

// Copies what the workgroup's units read into lds and points `v` (a copy of
// the level's arguments) at it, indexed as the originals.  Ends with a
// workgroup barrier.
template <int N, int MM, bool RAW, class TIN>
__device__ __forceinline__ void stage_inputs(const FwdArgs &a, int64_t blk, double *lds, FwdArgs &v) {
    using SG = Stage<N, MM, RAW>;
    const int64_t J0 = 2 * blk * Geo<N>::UPB;
    const int64_t nc = a.Nl - J0 < SG::NC ? a.Nl - J0 : SG::NC;  // columns that exist
    if constexpr (RAW) {
        const int64_t m = a.m;
        const int64_t cm = a.C_diag ? m : m * m, kk = a.K_diag ? N : N * N;
        // observation steps J0 .. J0+nc-1; evolution entries J0-1 .. J0+nc-2 (>= 0)
        const int64_t e0 = J0 > 0 ? J0 - 1 : 0, ne = J0 + nc - 1 - e0;
        // every view points at the start of its section; loads index relative
        // to col0 (observation steps) and ent0 (evolution entries)
        double *p = lds;
        auto put = [&](const double *src, int64_t first, int64_t count, int64_t w, const double *&view) {
            stage_copy(p, src + first * w, count * w);
            view = p;
            p += SG::NC * w;
        };
        put(a.G, J0, nc, m * N, v.G);
        put(a.o, J0, nc, m, v.o);
        put(a.C, J0, nc, cm, v.C);
        put(a.F, e0, ne, N * N, v.F);
        put(a.c, e0, ne, N, v.c);
        put(a.K, e0, ne, kk, v.K);
        if (a.H) put(a.H, e0, ne, N * N, v.H);
        v.col0 = J0;
        v.ent0 = e0;
    } else {
        constexpr int SR = Geo<N>::SREC;
        if constexpr (sizeof(TIN) == 4) {
            // FP32 records fill the first half of their slot (SR floats, rounded up to whole words)
            constexpr int HW = (SR + 1) / 2;
            const double *src = a.sys_in + J0 * SR;
            for (int64_t e = threadIdx.x; e < nc * HW; e += kBlock) {
                const int64_t col = e / HW, off = e - col * HW;
                lds[col * SR + off] = src[col * SR + off];
            }
        } else {
            stage_copy(lds, a.sys_in + J0 * SR, nc * SR);
        }
        v.sys_in = lds;
        v.col0 = J0;
    }
    __syncthreads();
}

// one forward level, one unit per G lanes, many workgroups
// With FOLD, the last unit of an odd level also folds the last column in
// (its statistics join its block's slot; the level's fold slot is set neutral).
template <int N, int MM, bool RAW, class T, class TIN, bool BATCH, bool FOLD = false, bool STG = true>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(wf_min_waves(N)))) void k_forward(
    FwdArgs a0, const FwdArgs *tab, BlockMap bm) {
    const FwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    // with FOLD the workgroup holding the last unit (which also folds the
    // last column in, the longest chain of the launch) is dispatched first
    const int64_t blk = BATCH  ? bm.blk[blockIdx.x]
                        : FOLD ? (int64_t)(gridDim.x - 1 - blockIdx.x)
                               : (int64_t)blockIdx.x;
    const Grp<N> g;
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    if constexpr (STG && Stage<N, MM, RAW>::ON) {
        __shared__ double lds[Stage<N, MM, RAW>::WORDS];
        FwdArgs v = a;
        stage_inputs<N, MM, RAW, TIN>(a, blk, lds, v);
        fwd_level<N, MM, RAW, FOLD, T, TIN>(a, v, blk, g, dmin, dmax, bad, nonfinite);
    } else {
        fwd_level<N, MM, RAW, FOLD, T, TIN>(a, a, blk, g, dmin, dmax, bad, nonfinite);
    }
    block_minmax<kBlock>(dmin, dmax, bad, nonfinite, a.flags);
    if (threadIdx.x == 0) {
        a.slots[2 * blk] = dmin;
        a.slots[2 * blk + 1] = dmax;
        if (FOLD && (a.Nl & 1) && blk == (a.units - 1) / Geo<N>::UPB) {
            a.fold_slot[0] = INFINITY;
            a.fold_slot[1] = 0.0;
        }
    }
}

// The fold of a level with N_l odd, after that level's k_forward: one unit
// reloads the last unit's step-3 triangle, eliminates the last column and
// re-triangularizes.  Writes one slot (a.fold_slot).
template <int N, int MM, bool RAW, class T, class TIN, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_fold(FwdArgs a0, const FwdArgs *tab, BlockMap bm) {
    const FwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    using GE = Geo<N>;
    const Grp<N> g;
    const bool valid = g.in && g.ui == 0;
    const LaneRole<N> L(g.gl);
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    const int64_t t = a.units - 1;
    if (g.ui == 0) {  // one unit: lanes of the other units stay idle
        T Onew[N];
        load_obs_sys<N>(Onew, 0, slot<T>(a.sys_out, t, GE::SREC), L, RIGHT, valid);
        fold_part<N, MM, RAW, T, TIN>(a, a, t, g.gl, g.gbase, L, Onew, dmin, dmax, bad, nonfinite);
        if (valid) {
            const int oc = L.role == RIGHT ? L.rc : (L.role == RHS ? N : -1);
            if (oc >= 0) {
                T *rec = slot<T>(a.sys_out, t, GE::SREC);
#pragma unroll
                for (int r = 0; r < N; ++r) rec[r * (N + 1) + oc] = Onew[r];
            }
        }
    }
    block_minmax<kBlock>(dmin, dmax, bad, nonfinite, a.flags);
    if (threadIdx.x == 0) {
        a.fold_slot[0] = dmin;
        a.fold_slot[1] = dmax;
    }
}

// Levels l0..L in one workgroup (the small levels at the top of the
// recursion): each level is a loop of unit passes, levels are separated by a
// workgroup barrier (a level reads only what this workgroup wrote one level
// down, or what earlier launches wrote).  Ends with the rank test over
// the per-block slots of the earlier launches and its own diagonal.
template <int N, int MM, bool RAW0, bool BATCH>
__global__ __launch_bounds__(kTailBlock) void k_fwd_tail(FwdTailArgs ta0, const FwdTailArgs *tab,
                                                       BlockMap bm) {
    const FwdTailArgs &ta = BATCH ? tab[bm.item[blockIdx.x]] : ta0;
    using GE = Geo<N>;
    constexpr int UPB = (kTailBlock / 64) * GE::UPW;
    const Grp<N> g;
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    for (int l = ta.l0; l <= ta.L; ++l) {
        FwdArgs a = ta.a;
        a.Nl = ta.Nl[l];
        a.units = a.Nl == 1 ? 1 : a.Nl / 2;
        a.level = l;
        a.sys_in = l >= 1 ? ta.sys + ta.sys_off[l] : nullptr;
        a.sys_out = l < ta.L ? ta.sys + ta.sys_off[l + 1] : nullptr;
        a.rrows = ta.rrows + ta.rec_off[l] * GE::RREC;
        if (a.Nl == 1) {
            if (RAW0 && l == 0)
                base_unit<N, MM, true, double>(a, g.in && g.ui == 0, g.gl, g.gbase, dmin, dmax, bad, nonfinite);
            else
                base_unit<N, MM, false, double>(a, g.in && g.ui == 0, g.gl, g.gbase, dmin, dmax, bad, nonfinite);
        } else {
            for (int64_t t0 = 0; t0 < a.units; t0 += UPB) {
                if (RAW0 && l == 0)
                    fwd_unit<N, MM, true, true, double, double>(a, a, t0 + g.ui, g.in, g.gl, g.gbase, dmin, dmax, bad, nonfinite);
                else
                    fwd_unit<N, MM, false, true, double, double>(a, a, t0 + g.ui, g.in, g.gl, g.gbase, dmin, dmax, bad, nonfinite);
            }
        }
        __syncthreads();  // the next level reads what this workgroup wrote: workgroup scope suffices
    }
    reduce_slots(ta.slots, ta.nprev, dmin, dmax);
    block_minmax<kTailBlock>(dmin, dmax, bad, nonfinite, ta.a.flags);
    rank_flag(dmin, dmax, ta.rank_tol, ta.a.flags);
}

// A group of consecutive forward levels l_first .. l_first + nlev - 1 in one
// launch (subtree fusion).  Workgroup w owns the level-l_first units
// [w U, (w+1) U) -- the last workgroup also the rest of the level -- and, at
// level l_first + x, the units [w U / 2^x, (w+1) U / 2^x) (the last one again
// to the level's end).  Those units read exactly the reduced columns the
// workgroup wrote one level down (unit t of level l writes reduced column t of
// level l+1 and reads columns 2t, 2t+1 and, for the fold, the level's last
// column), so levels are separated by workgroup barriers only.  U is a
// multiple of 2^(nlev-1).  The arithmetic of every unit is that of the
// per-level kernels.  One [min, max] slot per workgroup.
template <int N, int MM, bool RAW0, class T, class TIN>
__global__ __launch_bounds__(kBlock) void k_fwd_multi(FwdMultiArgs ma) {
    using GE = Geo<N>;
    const Grp<N> g;
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    const int64_t w = blockIdx.x;
    for (int x = 0; x < ma.nlev; ++x) {
        const int l = ma.l_first + x;
        FwdArgs a = ma.a;
        a.Nl = ma.Nl[l];
        a.units = a.Nl / 2;
        a.level = l;
        a.sys_in = l >= 1 ? ma.sys + ma.sys_off[l] : nullptr;
        a.sys_out = ma.sys + ma.sys_off[l + 1];
        a.rrows = ma.rrows + ma.rec_off[l] * GE::RREC;
        const int64_t span = ma.U >> x;
        const int64_t lo = w * span;
        const int64_t hi = (w == ma.groups - 1) ? a.units : lo + span;
        for (int64_t t0 = lo; t0 < hi; t0 += GE::UPB) {
            if (x == 0) {
                fwd_unit<N, MM, RAW0, true, T, TIN>(a, a, t0 + g.ui, g.in, g.gl, g.gbase, dmin, dmax, bad,
                                                    nonfinite, hi);
            } else {
                fwd_unit<N, MM, false, true, T, T>(a, a, t0 + g.ui, g.in, g.gl, g.gbase, dmin, dmax, bad,
                                                   nonfinite, hi);
            }
        }
        if (x + 1 < ma.nlev) __syncthreads();  // the next level reads what this one wrote
    }
    block_minmax<kBlock>(dmin, dmax, bad, nonfinite, ma.a.flags);
    if (threadIdx.x == 0) {
        ma.slots[2 * w] = dmin;
        ma.slots[2 * w + 1] = dmax;
    }
    // the rest of the group's slot region (read by the rank test) is neutral
    for (int64_t q = ma.groups + w * kBlock + threadIdx.x; q < ma.slot_pairs; q += ma.groups * kBlock) {
        ma.slots[2 * q] = INFINITY;
        ma.slots[2 * q + 1] = 0.0;
    }
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
    // P = T_I S_II overwrites the rows of S_II it came from (lane g reads and
    // writes only column g), S_ii overwrites the R row (dead after the solves)
    static constexpr int PER = RR + YI + SI + TT + RI;
};

// One block row of level l (record t): back-substitution and/or the SelInv
// step of Algorithm 2.  Uses this unit's LDS region and workgroup barriers, so
// every thread of the workgroup must call it the same number of times.
template <int N, bool DO_Y, bool DO_COV, class TR>
__device__ __forceinline__ void bwd_unit(const BwdArgs &a, int l, int64_t t, int64_t units,
                                         bool store_s, bool in, int gl, double *Rr) {
    using GE = Geo<N>;
    using SM = BwdSmem<N, DO_Y, DO_COV>;
    constexpr int G = GE::G;
    constexpr int W = 3 * N + 1;      // R-row width
    constexpr int TW = 2 * N + 1;     // T columns: [T+ | z | T-]
    const bool valid = in && t < units;
    const int64_t i = ((2 * t + 1) << l) - 1;
    const int64_t aa = i - ((int64_t)1 << l), bb = i + ((int64_t)1 << l);
    const bool va = valid && aa >= 0, vb = valid && bb <= a.k;

    double *yI = Rr + SM::RR;
    double *SII = yI + SM::YI;
    double *TT = SII + SM::SI;
    double *RI = TT + SM::TT;
    double *PP = SII;  // rows 0..n-1 of S_II, column by column
    double *SS = Rr;

    // stage the record and the neighbour data (lanes outside a unit skip)
    if (in) {
        const TR *rec = slot<TR>(a.rrows_all, a.rec_off[l] + t, GE::RREC);
        for (int e = gl; e < SM::RR; e += G) Rr[e] = valid ? double(rec[e]) : (e % (W + 1) == 0 ? 1.0 : 0.0);
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
    }
    __syncthreads();

    // triangular solves with R_ii: lanes < n -> columns of R_ii^{-1},
    // lanes n..3n -> T+ columns, z = R_ii^{-1} rho, T- columns
    if (gl < W && (DO_COV || gl >= N)) {
        double x[N], dinv[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            x[r] = gl < N ? (r == gl ? 1.0 : 0.0) : Rr[r * W + gl];
            dinv[r] = rcp_nr(Rr[r * W + r]);
        }
#pragma unroll
        for (int r = N - 1; r >= 0; --r) {
            double acc = x[r];
#pragma unroll
            for (int s = r + 1; s < N; ++s) acc = fma(-Rr[r * W + s], x[s], acc);
            x[r] = acc * dinv[r];
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
            double y0 = TT[gl * TW + N], y1 = 0.0;
#pragma unroll
            for (int d = 0; d < 2 * N; d += 2) y0 = fma(-TI(gl, d), yI[d], y0);
#pragma unroll
            for (int d = 1; d < 2 * N; d += 2) y1 = fma(-TI(gl, d), yI[d], y1);
            a.u_out[i * N + gl] = y0 + y1;
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
            if (valid && store_s) {
                const int64_t ri = a.rec_off[l] + t - a.spm_first;
                double *dst = a.spm + ri * 2 * N * N + (gl < N ? 0 : N * N);
                const int c = gl < N ? gl : gl - N;
#pragma unroll
                for (int r = 0; r < N; ++r) dst[r * N + c] = -p[r];
            }
            // level 0: S_{i,i+1} = -P_b, and S_{i-1,i} = S_{i,i-1}^T = -P_a^T
            if (l == 0 && a.lag1 && (gl < N ? va : vb)) {
                if (gl >= N) {
#pragma unroll
                    for (int r = 0; r < N; ++r) a.lag1[i * N * N + r * N + (gl - N)] = -p[r];
                } else {
#pragma unroll
                    for (int r = 0; r < N; ++r) a.lag1[(i - 1) * N * N + gl * N + r] = -p[r];
                }
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
    __syncthreads();  // the LDS region is reused by the next call
}

template <int N, bool DO_Y, bool DO_COV, class TR, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_backward(BwdArgs a0, const BwdArgs *tab, BlockMap bm) {
    using SM = BwdSmem<N, DO_Y, DO_COV>;
    const BwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    __shared__ double smem[Geo<N>::UPB * SM::PER];
    const Grp<N> g;
    const int l = BATCH ? bm.level[blockIdx.x] : a.level;
    const int64_t blk = BATCH ? bm.blk[blockIdx.x] : (int64_t)blockIdx.x;
    const int64_t t = blk * Geo<N>::UPB + g.ui;
    bwd_unit<N, DO_Y, DO_COV, TR>(a, l, t, (a.Nl[l] + 1) / 2, a.store_s && l >= 1, g.in, g.gl,
                              smem + g.ui * SM::PER);
}

// levels a.level down to a.l_lo in one workgroup of TB threads
template <int N, bool DO_Y, bool DO_COV, int TB, bool BATCH>
__global__ __launch_bounds__(TB) void k_bwd_tail(BwdArgs a0, const BwdArgs *tab, BlockMap bm) {
    const BwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    using SM = BwdSmem<N, DO_Y, DO_COV>;
    constexpr int UPB = (TB / 64) * Geo<N>::UPW;
    __shared__ double smem[UPB * SM::PER];
    const Grp<N> g;
    for (int l = a.level; l >= a.l_lo; --l) {
        const int64_t units = (a.Nl[l] + 1) / 2;
        for (int64_t t0 = 0; t0 < units; t0 += UPB)
            bwd_unit<N, DO_Y, DO_COV, double>(a, l, t0 + g.ui, units, a.store_s && l >= 1, g.in, g.gl,
                                      smem + g.ui * SM::PER);
        __syncthreads();  // the next level reads what this workgroup wrote: workgroup scope suffices
    }
}

// -------------------------------------------------------------- dispatch

template <int N, bool Y, bool COV>
struct BwdTailBlock {
    // largest of 512 / 256 threads whose LDS stays within 96 KB
    static constexpr int PER = BwdSmem<N, Y, COV>::PER;
    static constexpr int TB = (8 * Geo<N>::UPW * PER * 8 <= 96 * 1024) ? 512 : kBlock;
};

template <int N, int MM, bool RAW, class T, class TIN, bool STG = true>
static void launch_fwd_t(const FwdArgs &a, hipStream_t s) {
    const int64_t blocks = (a.units + Geo<N>::UPB - 1) / Geo<N>::UPB;
    hipLaunchKernelGGL((k_forward<N, MM, RAW, T, TIN, false, false, STG>), dim3((unsigned)blocks), dim3(kBlock),
                       0, s, a, nullptr, BlockMap{});
}

template <int N, int MM, class T, bool STG = true>
static void launch_fwd_fold_raw_t(const FwdArgs &a, hipStream_t s) {
    const int64_t blocks = (a.units + Geo<N>::UPB - 1) / Geo<N>::UPB;
    hipLaunchKernelGGL((k_forward<N, MM, true, T, double, false, true, STG>), dim3((unsigned)blocks), dim3(kBlock),
                       0, s, a, nullptr, BlockMap{});
}

template <int N, int MM, class T, class TIN>
static void launch_fwd_fold_t(const FwdArgs &a, hipStream_t s) {
    const int64_t blocks = (a.units + Geo<N>::UPB - 1) / Geo<N>::UPB;
    hipLaunchKernelGGL((k_forward<N, MM, false, T, TIN, false, true>), dim3((unsigned)blocks), dim3(kBlock), 0,
                       s, a, nullptr, BlockMap{});
}

template <int N, int MM, bool RAW0, class T, class TIN>
static void launch_fwd_multi_t(const FwdMultiArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd_multi<N, MM, RAW0, T, TIN>), dim3((unsigned)a.groups), dim3(kBlock), 0, s, a);
}

template <int N, int MM, bool RAW, class T, class TIN, bool STG = true>
static void launch_fwd_bt(const FwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_forward<N, MM, RAW, T, TIN, true, false, STG>), dim3((unsigned)blocks), dim3(kBlock),
                       0, s, FwdArgs{}, tab, bm);
}

template <int N, int MM, bool RAW, class T, class TIN>
static void launch_fold_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_fold<N, MM, RAW, T, TIN, false>), dim3(1), dim3(kBlock), 0, s, a, nullptr,
                       BlockMap{});
}

template <int N, int MM, bool RAW, class T, class TIN>
static void launch_fold_bt(const FwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_fold<N, MM, RAW, T, TIN, true>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       FwdArgs{}, tab, bm);
}

template <int N, int MM, bool RAW0>
static void launch_fwd_tail_t(const FwdTailArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd_tail<N, MM, RAW0, false>), dim3(1), dim3(kTailBlock), 0, s, a, nullptr,
                       BlockMap{});
}

template <int N, int MM, bool RAW0>
static void launch_fwd_tail_bt(const FwdTailArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd_tail<N, MM, RAW0, true>), dim3((unsigned)blocks), dim3(kTailBlock), 0, s,
                       FwdTailArgs{}, tab, bm);
}

template <int N, bool Y, bool COV, class TR>
static void launch_bwd_t(const BwdArgs &a, hipStream_t s) {
    const int64_t units = (a.Nl[a.level] + 1) / 2;
    const int64_t blocks = (units + Geo<N>::UPB - 1) / Geo<N>::UPB;
    hipLaunchKernelGGL((k_backward<N, Y, COV, TR, false>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       a, nullptr, BlockMap{});
}

template <int N, bool Y, bool COV, class TR>
static void launch_bwd_bt(const BwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_backward<N, Y, COV, TR, true>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       BwdArgs{}, tab, bm);
}

template <int N, bool Y, bool COV>
static void launch_bwd_tail_t(const BwdArgs &a, hipStream_t s) {
    constexpr int TB = BwdTailBlock<N, Y, COV>::TB;
    hipLaunchKernelGGL((k_bwd_tail<N, Y, COV, TB, false>), dim3(1), dim3(TB), 0, s, a, nullptr,
                       BlockMap{});
}

template <int N, bool Y, bool COV>
static void launch_bwd_tail_bt(const BwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    constexpr int TB = BwdTailBlock<N, Y, COV>::TB;
    hipLaunchKernelGGL((k_bwd_tail<N, Y, COV, TB, true>), dim3((unsigned)blocks), dim3(TB), 0, s,
                       BwdArgs{}, tab, bm);
}

// variants: forward [FP64 | FP32 | FP64 from FP32 records (switch level)],
// backward [mode][record type FP64 | FP32]
template <int N, int MM>
constexpr KernelSet make_set_base() {
    return KernelSet{N,
                     MM,
                     {&launch_fwd_t<N, MM, true, double, double>, &launch_fwd_t<N, MM, true, float, double>},
                     {&launch_fwd_t<N, MM, false, double, double>, &launch_fwd_t<N, MM, false, float, float>,
                      &launch_fwd_t<N, MM, false, double, float>},
                     {&launch_fold_t<N, MM, true, double, double>, &launch_fold_t<N, MM, true, float, double>},
                     {&launch_fold_t<N, MM, false, double, double>, &launch_fold_t<N, MM, false, float, float>,
                      &launch_fold_t<N, MM, false, double, float>},
                     &launch_fwd_tail_t<N, MM, true>,
                     &launch_fwd_tail_t<N, MM, false>,
                     {{&launch_bwd_t<N, true, false, double>, &launch_bwd_t<N, true, false, float>},
                      {&launch_bwd_t<N, false, true, double>, &launch_bwd_t<N, false, true, float>},
                      {&launch_bwd_t<N, true, true, double>, &launch_bwd_t<N, true, true, float>}},
                     {&launch_bwd_tail_t<N, true, false>, &launch_bwd_tail_t<N, false, true>,
                      &launch_bwd_tail_t<N, true, true>},
                     {&launch_fwd_bt<N, MM, true, double, double>, &launch_fwd_bt<N, MM, true, float, double>},
                     {&launch_fwd_bt<N, MM, false, double, double>, &launch_fwd_bt<N, MM, false, float, float>,
                      &launch_fwd_bt<N, MM, false, double, float>},
                     {&launch_fold_bt<N, MM, true, double, double>, &launch_fold_bt<N, MM, true, float, double>},
                     {&launch_fold_bt<N, MM, false, double, double>, &launch_fold_bt<N, MM, false, float, float>,
                      &launch_fold_bt<N, MM, false, double, float>},
                     &launch_fwd_tail_bt<N, MM, true>,
                     &launch_fwd_tail_bt<N, MM, false>,
                     {{&launch_bwd_bt<N, true, false, double>, &launch_bwd_bt<N, true, false, float>},
                      {&launch_bwd_bt<N, false, true, double>, &launch_bwd_bt<N, false, true, float>},
                      {&launch_bwd_bt<N, true, true, double>, &launch_bwd_bt<N, true, true, float>}},
                     {&launch_bwd_tail_bt<N, true, false>, &launch_bwd_tail_bt<N, false, true>,
                      &launch_bwd_tail_bt<N, true, true>},
                     Geo<N>::UPB,
                     (kTailBlock / 64) * Geo<N>::UPW,
                     {Geo<N>::UPB, Geo<N>::UPB, Geo<N>::UPB},
                     {(BwdTailBlock<N, true, false>::TB / 64) * Geo<N>::UPW,
                      (BwdTailBlock<N, false, true>::TB / 64) * Geo<N>::UPW,
                      (BwdTailBlock<N, true, true>::TB / 64) * Geo<N>::UPW},
                     {&launch_fwd_fold_t<N, MM, double, double>, &launch_fwd_fold_t<N, MM, float, float>,
                      &launch_fwd_fold_t<N, MM, double, float>}};
}

template <int N, int MM>
constexpr KernelSet make_set() {
    KernelSet s = make_set_base<N, MM>();
    s.fwd_fold_raw[0] = &launch_fwd_fold_raw_t<N, MM, double>;
    s.fwd_fold_raw[1] = &launch_fwd_fold_raw_t<N, MM, float>;
    s.fwd_multi_raw[0] = &launch_fwd_multi_t<N, MM, true, double, double>;
    s.fwd_multi_raw[1] = &launch_fwd_multi_t<N, MM, true, float, double>;
    s.fwd_multi[FV_F64] = &launch_fwd_multi_t<N, MM, false, double, double>;
    s.fwd_multi[FV_F32] = &launch_fwd_multi_t<N, MM, false, float, float>;
    s.fwd_multi[FV_F64_FROM_F32] = &launch_fwd_multi_t<N, MM, false, double, float>;
    s.upb_multi = Geo<N>::UPB;
    return s;
}

// forward variant 1: the level-0 kernels without LDS staging (where the
// default stages), everything else as the default
template <int N, int MM>
constexpr KernelSet make_set_unstaged() {
    KernelSet s = make_set<N, MM>();
    s.fwd_raw[0] = &launch_fwd_t<N, MM, true, double, double, false>;
    s.fwd_raw[1] = &launch_fwd_t<N, MM, true, float, double, false>;
    s.fwd_raw_b[0] = &launch_fwd_bt<N, MM, true, double, double, false>;
    s.fwd_raw_b[1] = &launch_fwd_bt<N, MM, true, float, double, false>;
    s.fwd_fold_raw[0] = &launch_fwd_fold_raw_t<N, MM, double, false>;
    s.fwd_fold_raw[1] = &launch_fwd_fold_raw_t<N, MM, float, false>;
    s.fv = 1;
    return s;
}

}  // namespace ks
