// ks_device_blk.h -- the workgroup family of the odd-even smoother kernels,
// for state dimensions whose stacks need more than one wavefront of lanes.
//
// Same algebra as the wavefront family (ks_device.h): one unit per even
// column of a level, step 1 then steps 2 and 3, back-substitution and
// Algorithm 2 on the way back.  Here a unit is a whole workgroup: lane g owns
// one stack column,
//   [0, n) u_j  [n, 2n) u_{j+1}  2n rhs  (2n, 3n] u_{j-1}     (steps 1 and 2)
//   [3n+1, 4n+1) u_{j+1}  4n+1 rhs                          (step 3)
// so steps 2 and 3 run as one Householder sweep on disjoint lanes.  The pivot
// lane of each sweep writes its reflector to a double-buffered LDS slot; one
// workgroup barrier per pivot publishes it and every lane updates its own
// column.  Stacks are padded to 2n rows in VGPRs.
#pragma once

#include "ks_device.h"

namespace ks {

template <int N>
struct BGeo {
    static constexpr int COLS = 4 * N + 2;
    static constexpr int TB = (COLS + 63) / 64 * 64;       // forward workgroup
    static constexpr int W = 3 * N + 1;
    static constexpr int TBB = (W + 63) / 64 * 64;         // backward workgroup
    static constexpr int BOFF = 3 * N + 1;                 // first step-3 lane
    static constexpr int RREC = N * (3 * N + 1);
    static constexpr int OREC = N * (N + 1);
    static constexpr int EREC = N * (2 * N + 1);
    static constexpr int SREC = OREC + EREC;
};

template <int N>
struct BRole {
    int role, rc;
    __device__ explicit BRole(int g) {
        if (g < N) { role = CUR; rc = g; }
        else if (g < 2 * N) { role = RIGHT; rc = g - N; }
        else if (g == 2 * N) { role = RHS; rc = 0; }
        else if (g <= 3 * N) { role = LEFT; rc = g - 2 * N - 1; }
        else if (g < 4 * N + 1) { role = BRIGHT; rc = g - 3 * N - 1; }
        else if (g == 4 * N + 1) { role = BRHS; rc = 0; }
        else { role = IDLE; rc = 0; }
    }
};

// Householder QR of rows [0, HR) of a column-distributed stack (see hqr), the
// reflector published through LDS: buf holds two slots of H + 2 doubles, slot
// = [x' | c] with x' = (0, .., 0, alpha - beta, x_{p+1}, .., x_{HR-1}) and
// c = 1 / (beta (beta - alpha)).  Rows are processed in chunks of 8; chunks
// wholly above the pivot row are skipped (a workgroup-uniform branch), so no
// row needs a select.  `part` lanes apply the reflector, others leave their
// column untouched.  The pivot diagonal ends as beta up to rounding; strictly
// lower parts of pivot columns are set to zero at the end.
template <int H, int HR, int NP, class T>
__device__ __forceinline__ void hqr_lds(T (&x)[H], int gl, int pl0, bool part, T *buf,
                                        int &ph) {
    constexpr int P = NP < HR ? NP : HR;
    constexpr int CH = 8;
#pragma unroll 1
    for (int p = 0; p < P; ++p) {
        T *bp = buf + (ph & 1) * (H + 2);
        ++ph;
        if (gl == pl0 + p) {
            T alpha = 0, am = 0;
#pragma unroll
            for (int r = 0; r < HR; ++r) {
                if (r == p) alpha = x[r];
                if (r >= p) am = fmax(am, fabs(x[r]));
            }
            // sum of squares scaled by the largest entry in FP32, plain in FP64
            const T sc = sizeof(T) == 4 ? (am > T(0) ? rcp_nr(am) : T(0)) : T(1);
            if (sizeof(T) != 4) am = T(1);
            T s0 = 0, s1 = 0;
#pragma unroll
            for (int r = 0; r < HR; ++r) {
                const T m = r > p ? x[r] * sc : T(0);
                if (r & 1) s0 = fma(m, m, s0);
                else s1 = fma(m, m, s1);
            }
            const T as = alpha * sc;
            const T xn2 = s0 + s1;
            const T s = fma(as, as, xn2);
            const T nrs = sqrt(s);
            const T beta = -copysign(nrs * am, alpha);
            bp[H] = xn2 != T(0) ? sc * sc * rcp_nr(fma(fabs(as), nrs, s)) : T(0);
            const T v0 = alpha - beta;
#pragma unroll
            for (int r = 0; r < HR; ++r) bp[r] = r < p ? T(0) : (r == p ? v0 : x[r]);
        }
        __syncthreads();
        if (part) {
            T w0 = 0, w1 = 0;
#pragma unroll
            for (int c0 = 0; c0 < HR; c0 += CH) {
                if (c0 + CH > p) {
#pragma unroll
                    for (int r = c0; r < c0 + CH && r < HR; ++r) {
                        if (r & 1) w0 = fma(bp[r], x[r], w0);
                        else w1 = fma(bp[r], x[r], w1);
                    }
                }
            }
            const T w = (w0 + w1) * bp[H];
            __asm__ volatile("" ::: "memory");  // re-read the slot instead of holding it in VGPRs
#pragma unroll
            for (int c0 = 0; c0 < HR; c0 += CH) {
                if (c0 + CH > p) {
#pragma unroll
                    for (int r = c0; r < c0 + CH && r < HR; ++r) x[r] = fma(-w, bp[r], x[r]);
                }
            }
        }
    }
    const unsigned q = (unsigned)(gl - pl0);
#pragma unroll
    for (int r = 1; r < HR; ++r)
        if (q < (unsigned)(r < P ? r : P)) x[r] = T(0);
}

// dense whitening with the Cholesky column published through LDS (see
// whiten_dense); buf holds two slots of H + 2 doubles (the same slots as
// hqr_lds, so consecutive sweeps never write a slot another lane still reads)
template <int H, int D, class T>
__device__ __forceinline__ void whiten_lds(T (&x)[H], int roff, T (&cv)[D], int gl,
                                           int cl0, bool part, T *buf, int &ph, bool &bad) {
#pragma unroll 1
    for (int p = 0; p < D; ++p) {
        T *bp = buf + (ph & 1) * (H + 2);
        ++ph;
        if (gl == cl0 + p) {
            T piv = 0;
#pragma unroll
            for (int r = 0; r < D; ++r)
                if (r == p) piv = cv[r];
            if (!(piv > T(0) && isfinite(piv))) bad = true;
            const T il = rsq_nr(piv);
            bp[0] = il;
#pragma unroll
            for (int r = 0; r < D; ++r) bp[1 + r] = r > p ? cv[r] * il : T(0);
        }
        __syncthreads();
        const T ilb = bp[0];
        T cp = 0, xq = 0;
#pragma unroll
        for (int r = 0; r < D; ++r)
            if (r == p) {
                cp = cv[r];
                xq = x[roff + r];
            }
        const T f = cp * ilb, xp = xq * ilb;
#pragma unroll
        for (int r = 0; r < D; ++r) cv[r] = fma(-bp[1 + r], f, cv[r]);
        if (part) {
#pragma unroll
            for (int r = 0; r < D; ++r)
                x[roff + r] = r == p ? xp : fma(-bp[1 + r], xp, x[roff + r]);
        }
    }
}

template <int H, int D, class T>
__device__ __forceinline__ void whiten_blk(bool diag, T (&x)[H], int roff, T (&cv)[D],
                                           int gl, int cl0, bool part, T *buf, int &ph,
                                           bool &bad) {
    if (diag) {
        if (part) whiten_diag<H, D, T>(x, roff, cv, gl, bad);
    } else {
        whiten_lds<H, D, T>(x, roff, cv, gl, cl0, part, buf, ph, bad);
    }
}

// ------------------------------------------------------------- forward level

// The last column of a level with N_l odd (see fold_part): the u_j lanes
// eliminate it, its Z rows go to the step-3 lanes and are stacked under
// Onew, the last unit's step-3 triangle.  Whole workgroup, uniform.
template <int N, int MM, bool RAW, class T, class TIN>
__device__ __forceinline__ void blk_fold_part(const FwdArgs &a, int64_t t, T *bufs,
                                              T *exch, T (&Onew)[N], double &dmin,
                                              double &dmax, bool &bad, bool &nonfinite) {
    using BG = BGeo<N>;
    constexpr int RO = RAW ? MM : N;
    constexpr int H = 2 * N;
    const int gl = threadIdx.x;
    const BRole<N> L(gl);
    const bool isB = L.role == BRIGHT || L.role == BRHS;
    const bool isAC = L.role <= LEFT;
    T *bufAC = bufs, *bufB = bufs + 2 * (H + 2);
    int ph = 0;
    const int64_t jl = a.Nl - 1;
    T X2[H];
#pragma unroll
    for (int r = 0; r < H; ++r) X2[r] = T(0);
    if constexpr (RAW) {
        T cvO[MM];
        if (isAC) load_obs_raw<N, MM>(X2, 0, cvO, jl, L, gl, CUR, 0, a, true);
        else {
#pragma unroll
            for (int r = 0; r < MM; ++r) cvO[r] = T(0);
        }
        whiten_blk<H, MM>(a.C_diag, X2, 0, cvO, gl, 0, isAC, bufAC, ph, bad);
    } else {
        if (isAC) load_obs_sys<N>(X2, 0, slot<TIN>(a.sys_in, jl, BG::SREC), L, CUR, true);
    }
    hqr_lds<H, RO, N>(X2, gl, 0, isAC, bufAC, ph);
    if (isAC) {
#pragma unroll
        for (int r = N - 1; r >= 0; --r) X2[N + r] = r < RO ? X2[r] : T(0);
    }
    if constexpr (RAW) {
        T cvE[N];
#pragma unroll
        for (int r = 0; r < N; ++r) cvE[r] = T(0);
        if (isAC) load_evol_raw<N>(X2, 0, cvE, jl, L, gl, LEFT, CUR, 2 * N + 1, a, true);
        whiten_blk<H, N>(a.K_diag, X2, 0, cvE, gl, 2 * N + 1, isAC, bufAC, ph, bad);
    } else {
        if (isAC) load_evol_sys<N>(X2, 0, slot<TIN>(a.sys_in, jl, BG::SREC) + BG::OREC, L, LEFT, CUR, true);
    }
    hqr_lds<H, H, N>(X2, gl, 0, isAC, bufAC, ph);
    store_rrow<N>(slot<T>(a.rrows, t + 1, BG::RREC), X2, gl, true);
    diag_stats<N>(X2, L, true, dmin, dmax, nonfinite);
    // Z rows (u_{j-1} lanes) and zeta -> the step-3 lanes, stacked under O'
    if (L.role == LEFT || L.role == RHS) {
        const int col = L.role == LEFT ? L.rc : N;
#pragma unroll
        for (int r = 0; r < N; ++r) exch[r * (N + 1) + col] = X2[N + r];
    }
    __syncthreads();
    T X3[H];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        X3[r] = Onew[r];
        X3[N + r] = T(0);
    }
    if (isB) {
        const int col = L.role == BRIGHT ? L.rc : N;
#pragma unroll
        for (int r = 0; r < N; ++r) X3[N + r] = exch[r * (N + 1) + col];
    }
    hqr_lds<H, H, N>(X3, gl, BG::BOFF, isB, bufB, ph);
#pragma unroll
    for (int r = 0; r < N; ++r) Onew[r] = X3[r];
}

template <int N, int MM, bool RAW, bool INLINE_FOLD, class T, class TIN>
__device__ __forceinline__ void blk_fwd_unit(const FwdArgs &a, int64_t t, T *bufs,
                                             T *exch, double &dmin, double &dmax, bool &bad,
                                             bool &nonfinite) {
    using BG = BGeo<N>;
    constexpr int RO = RAW ? MM : N;
    constexpr int H = 2 * N;
    constexpr int HA = RO + N;
    constexpr int PB = 2 * RO < N ? 2 * RO : N;
    static_assert(RO <= N, "observation blocks taller than n are not in this family");
    const int gl = threadIdx.x;
    const BRole<N> L(gl);
    const bool isB = L.role == BRIGHT || L.role == BRHS;
    const bool isAC = L.role <= LEFT;
    T *bufAC = bufs, *bufB = bufs + 2 * (H + 2);
    int ph = 0;
    const bool valid = t < a.units;
    const int64_t j = 2 * t;
    const bool fold = (a.Nl & 1) && t == a.units - 1;  // uniform over the workgroup

    T X[H];
#pragma unroll
    for (int r = 0; r < H; ++r) X[r] = T(0);
    if constexpr (RAW) {
        T cvO[MM], cvE[N];
#pragma unroll
        for (int r = 0; r < N; ++r) cvE[r] = T(0);
        if (isB) {
            load_obs_raw<N, MM>(X, 0, cvO, j + 1, L, gl, BRIGHT, BG::BOFF, a, valid, BRHS);
        } else {
            load_obs_raw<N, MM>(X, 0, cvO, j, L, gl, CUR, 0, a, valid);
            load_evol_raw<N>(X, RO, cvE, j + 1, L, gl, CUR, RIGHT, 0, a, valid);
        }
        whiten_blk<H, MM>(a.C_diag, X, 0, cvO, gl, isB ? BG::BOFF : 0, true, isB ? bufB : bufAC, ph, bad);
        whiten_blk<H, N>(a.K_diag, X, RO, cvE, gl, 0, isAC, bufAC, ph, bad);
    } else {
        if (isB) {
            load_obs_sys<N>(X, 0, slot<TIN>(a.sys_in, j + 1, BG::SREC), L, BRIGHT, valid, BRHS);
        } else {
            load_obs_sys<N>(X, 0, slot<TIN>(a.sys_in, j, BG::SREC), L, CUR, valid);
            load_evol_sys<N>(X, RO, slot<TIN>(a.sys_in, j + 1, BG::SREC) + BG::OREC, L, CUR, RIGHT, valid);
        }
    }

    // step 1 on the u_j / u_{j+1} / rhs lanes
    hqr_lds<H, HA, N>(X, gl, 0, isAC, bufAC, ph);

    // D~_{j+1} and gamma go to the step-3 lanes; C = [E_j ; R~_j X_j rho~_j]
    if (L.role == RIGHT || L.role == RHS) {
        const int col = L.role == RIGHT ? L.rc : N;
#pragma unroll
        for (int r = 0; r < RO; ++r) exch[r * (N + 1) + col] = X[N + r];
    }
    if (isAC) {
#pragma unroll
        for (int r = N - 1; r >= 0; --r) X[N + r] = X[r];
    }
    if constexpr (RAW) {
        T cvE[N];
#pragma unroll
        for (int r = 0; r < N; ++r) cvE[r] = T(0);
        if (isAC) {
            load_evol_raw<N>(X, 0, cvE, j, L, gl, LEFT, CUR, 2 * N + 1, a, valid && j >= 1);
        }
        whiten_blk<H, N>(a.K_diag, X, 0, cvE, gl, 2 * N + 1, isAC, bufAC, ph, bad);
    } else {
        if (isAC) load_evol_sys<N>(X, 0, slot<TIN>(a.sys_in, j, BG::SREC) + BG::OREC, L, LEFT, CUR, valid && j >= 1);
    }
    __syncthreads();
    if (isB) {
        const int col = L.role == BRIGHT ? L.rc : N;
#pragma unroll
        for (int r = 0; r < RO; ++r) X[RO + r] = exch[r * (N + 1) + col];
    }

    // steps 2 (pivots u_j lanes) and 3 (pivots step-3 lanes) in one sweep
    hqr_lds<H, H, N>(X, gl, isB ? BG::BOFF : 0, isAC || isB, isB ? bufB : bufAC, ph);

    store_rrow<N>(slot<T>(a.rrows, t, BG::RREC), X, gl, valid);
    diag_stats<N>(X, L, valid, dmin, dmax, nonfinite);
    if (valid) {
        const int ec = L.role == LEFT ? L.rc
                     : L.role == RIGHT ? N + L.rc
                     : L.role == RHS ? 2 * N : -1;
        if (ec >= 0) {
            T *rec = slot<T>(a.sys_out, t, BG::SREC) + BG::OREC;
#pragma unroll
            for (int r = 0; r < N; ++r) rec[r * (2 * N + 1) + ec] = X[N + r];
        }
    }
    T Onew[N];
#pragma unroll
    for (int r = 0; r < N; ++r) Onew[r] = (isB && r < PB) ? X[r] : T(0);

    if (INLINE_FOLD && fold && valid) {
        __syncthreads();
        blk_fold_part<N, MM, RAW, T, TIN>(a, t, bufs, exch, Onew, dmin, dmax, bad, nonfinite);
    }

    if (valid && isB) {
        const int oc = L.role == BRIGHT ? L.rc : N;
        T *rec = slot<T>(a.sys_out, t, BG::SREC);
#pragma unroll
        for (int r = 0; r < N; ++r) rec[r * (N + 1) + oc] = Onew[r];
    }
}

template <int N, int MM, bool RAW, class T, class TIN, bool BATCH>
__global__ __launch_bounds__(BGeo<N>::TB) void k_blk_forward(FwdArgs a0, const FwdArgs *tab,
                                                             BlockMap bm) {
    const FwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    const int64_t blk = BATCH ? bm.blk[blockIdx.x] : (int64_t)blockIdx.x;
    constexpr int H = 2 * N;
    __shared__ T bufs[4 * (H + 2)];
    __shared__ T exch[N * (N + 1)];
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    blk_fwd_unit<N, MM, RAW, false, T, TIN>(a, blk, bufs, exch, dmin, dmax, bad, nonfinite);
    block_minmax<BGeo<N>::TB>(dmin, dmax, bad, nonfinite, a.flags);
    if (threadIdx.x == 0) {
        a.slots[2 * blk] = dmin;
        a.slots[2 * blk + 1] = dmax;
    }
}

// the fold of an odd level after its k_blk_forward (one workgroup)
template <int N, int MM, bool RAW, class T, class TIN, bool BATCH>
__global__ __launch_bounds__(BGeo<N>::TB) void k_blk_fold(FwdArgs a0, const FwdArgs *tab, BlockMap bm) {
    const FwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    using BG = BGeo<N>;
    constexpr int H = 2 * N;
    __shared__ T bufs[4 * (H + 2)];
    __shared__ T exch[N * (N + 1)];
    const BRole<N> L(threadIdx.x);
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    const int64_t t = a.units - 1;
    T Onew[N];
    load_obs_sys<N>(Onew, 0, slot<T>(a.sys_out, t, BG::SREC), L, BRIGHT, true, BRHS);
    blk_fold_part<N, MM, RAW, T, TIN>(a, t, bufs, exch, Onew, dmin, dmax, bad, nonfinite);
    if (L.role == BRIGHT || L.role == BRHS) {
        const int oc = L.role == BRIGHT ? L.rc : N;
        T *rec = slot<T>(a.sys_out, t, BG::SREC);
#pragma unroll
        for (int r = 0; r < N; ++r) rec[r * (N + 1) + oc] = Onew[r];
    }
    block_minmax<BG::TB>(dmin, dmax, bad, nonfinite, a.flags);
    if (threadIdx.x == 0) {
        a.fold_slot[0] = dmin;
        a.fold_slot[1] = dmax;
    }
}

// forward levels l0..L in one workgroup (in this family only the base level,
// or the whole problem when it is tiny), then the rank test
template <int N, int MM, bool RAW0, bool BATCH>
__global__ __launch_bounds__(BGeo<N>::TB) void k_blk_fwd_tail(FwdTailArgs ta0, const FwdTailArgs *tab,
                                                              BlockMap bm) {
    const FwdTailArgs &ta = BATCH ? tab[bm.item[blockIdx.x]] : ta0;
    using BG = BGeo<N>;
    constexpr int H = 2 * N;
    __shared__ double bufs[4 * (H + 2)];
    __shared__ double exch[N * (N + 1)];
    const int gl = threadIdx.x;
    const BRole<N> L(gl);
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    for (int l = ta.l0; l <= ta.L; ++l) {
        FwdArgs a = ta.a;
        a.Nl = ta.Nl[l];
        a.units = a.Nl == 1 ? 1 : a.Nl / 2;
        a.level = l;
        a.sys_in = l >= 1 ? ta.sys + ta.sys_off[l] : nullptr;
        a.sys_out = l < ta.L ? ta.sys + ta.sys_off[l + 1] : nullptr;
        a.rrows = ta.rrows + ta.rec_off[l] * BG::RREC;
        if (a.Nl == 1) {
            constexpr int RO0 = RAW0 ? MM : N;
            double X[H];
#pragma unroll
            for (int r = 0; r < H; ++r) X[r] = 0.0;
            int ph = 0;
            const bool isAC = L.role <= LEFT;
            if (RAW0 && l == 0) {
                double cv[MM];
                if (isAC) load_obs_raw<N, MM>(X, 0, cv, 0, L, gl, CUR, 0, a, true);
                else {
#pragma unroll
                    for (int r = 0; r < MM; ++r) cv[r] = 0.0;
                }
                whiten_blk<H, MM>(a.C_diag, X, 0, cv, gl, 0, isAC, bufs, ph, bad);
                hqr_lds<H, RO0, N>(X, gl, 0, isAC, bufs, ph);
            } else {
                if (isAC) load_obs_sys<N>(X, 0, slot<double>(a.sys_in, 0, BG::SREC), L, CUR, true);
                hqr_lds<H, N, N>(X, gl, 0, isAC, bufs, ph);
            }
            const int rows = (RAW0 && l == 0) ? RO0 : N;
#pragma unroll
            for (int r = 0; r < N; ++r)
                if (!(r < rows && (L.role == CUR || L.role == RHS))) X[r] = 0.0;
            store_rrow<N>(a.rrows, X, gl, true);
            diag_stats<N>(X, L, true, dmin, dmax, nonfinite);
        } else {
            for (int64_t t = 0; t < a.units; ++t) {
                if (RAW0 && l == 0)
                    blk_fwd_unit<N, MM, true, true, double, double>(a, t, bufs, exch, dmin, dmax, bad, nonfinite);
                else
                    blk_fwd_unit<N, MM, false, true, double, double>(a, t, bufs, exch, dmin, dmax, bad, nonfinite);
                __syncthreads();
            }
        }
        __threadfence();
        __syncthreads();
    }
    reduce_slots(ta.slots, ta.nprev, dmin, dmax);
    block_minmax<BG::TB>(dmin, dmax, bad, nonfinite, ta.a.flags);
    rank_flag(dmin, dmax, ta.rank_tol, ta.a.flags);
}

// ------------------------------------------------------------ backward level

// one block row (record t of level l); TBB threads, lane g < 3n+1 owns column g
// of the R row: [R_ii | R_i,b | rho_i | R_i,a]
template <int N, bool DO_Y, bool DO_COV, class TR>
__device__ __forceinline__ void blk_bwd_unit(const BwdArgs &a, int l, int64_t t, int64_t units,
                                             bool store_s, double *sm) {
    using BG = BGeo<N>;
    constexpr int W = BG::W;
    constexpr int TW = 2 * N + 1;   // T columns [T+ | z | T-]
    double *Rd = sm;                // R_ii, later S_ii
    double *TT = Rd + N * N;
    double *RI = TT + N * TW;
    double *PP = RI + N * N;
    const int gl = threadIdx.x;
    const bool valid = t < units;
    const int64_t i = ((2 * t + 1) << l) - 1;
    const int64_t aa = i - ((int64_t)1 << l), bb = i + ((int64_t)1 << l);
    const bool va = valid && aa >= 0, vb = valid && bb <= a.k;
    const TR *rec = slot<TR>(a.rrows_all, a.rec_off[l] + t, BG::RREC);

    double x[N];
    if (gl < W) {
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] = valid ? double(rec[r * W + gl]) : (r == gl ? 1.0 : 0.0);
        if (gl < N) {
#pragma unroll
            for (int r = 0; r < N; ++r) Rd[r * N + gl] = x[r];
        }
    }
    __syncthreads();
    if (gl < W && (DO_COV || gl >= N)) {
        if (gl < N) {
#pragma unroll
            for (int r = 0; r < N; ++r) x[r] = r == gl ? 1.0 : 0.0;
        }
#pragma unroll
        for (int r = N - 1; r >= 0; --r) {
            double acc = x[r];
#pragma unroll
            for (int s = r + 1; s < N; ++s) acc = fma(-Rd[r * N + s], x[s], acc);
            x[r] = acc * rcp_nr(Rd[r * N + r]);
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
    auto TI = [&](int r, int d) -> double {
        return d < N ? TT[r * TW + N + 1 + d] : TT[r * TW + (d - N)];
    };
    if constexpr (DO_Y) {
        if (valid && gl < N) {
            double y0 = TT[gl * TW + N], y1 = 0.0;
#pragma unroll 4
            for (int d = 0; d < N; ++d) {
                if (va) y0 = fma(-TI(gl, d), a.u_in[aa * N + d], y0);
                if (vb) y1 = fma(-TI(gl, N + d), a.u_in[bb * N + d], y1);
            }
            a.u_out[i * N + gl] = y0 + y1;
        }
    }
    if constexpr (DO_COV) {
        const double *sab = nullptr;
        bool trans = false;
        if (va && vb) {
            const int la = __builtin_ctzll((unsigned long long)(aa + 1));
            if (la == l + 1) {
                sab = a.spm + (rec_of(aa, a.rec_off) - a.spm_first) * 2 * N * N + N * N;
            } else {
                sab = a.spm + (rec_of(bb, a.rec_off) - a.spm_first) * 2 * N * N;
                trans = true;
            }
        }
        // S_II(d, c) for d, c < 2n
        auto SII = [&](int d, int c) -> double {
            if (d < N && c < N) return va ? a.cov[aa * N * N + d * N + c] : 0.0;
            if (d >= N && c >= N) return vb ? a.cov[bb * N * N + (d - N) * N + (c - N)] : 0.0;
            if (!sab) return 0.0;
            const int rr = d < N ? d : c, cc = d < N ? c - N : d - N;  // S_ab(rr, cc)
            return trans ? sab[cc * N + rr] : sab[rr * N + cc];
        };
        if (gl < 2 * N) {
            double p[N];
#pragma unroll
            for (int r = 0; r < N; ++r) p[r] = 0.0;
#pragma unroll 2
            for (int d = 0; d < 2 * N; ++d) {
                const double s = SII(d, gl);
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
        }
        __syncthreads();
        if (gl < N) {
            double s[N];
#pragma unroll
            for (int r = 0; r < N; ++r) s[r] = 0.0;
#pragma unroll 2
            for (int q = 0; q < N; ++q) {
                const double rc = RI[gl * N + q];
#pragma unroll
                for (int r = 0; r < N; ++r) s[r] = fma(RI[r * N + q], rc, s[r]);
            }
#pragma unroll 2
            for (int d = 0; d < 2 * N; ++d) {
                const double tc = TI(gl, d);
#pragma unroll
                for (int r = 0; r < N; ++r) s[r] = fma(PP[r * 2 * N + d], tc, s[r]);
            }
#pragma unroll
            for (int r = 0; r < N; ++r) Rd[r * N + gl] = s[r];
        }
        __syncthreads();
        if (valid && gl < N) {
#pragma unroll
            for (int r = 0; r < N; ++r)
                a.cov[i * N * N + r * N + gl] = 0.5 * (Rd[r * N + gl] + Rd[gl * N + r]);
        }
    }
    __syncthreads();
}

template <int N>
struct BSmem {
    static constexpr int PER = N * N + N * (2 * N + 1) + N * N + 2 * N * N;
};

template <int N, bool DO_Y, bool DO_COV, class TR, bool BATCH>
__global__ __launch_bounds__(BGeo<N>::TBB) void k_blk_backward(BwdArgs a0, const BwdArgs *tab,
                                                               BlockMap bm) {
    const BwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    __shared__ double sm[BSmem<N>::PER];
    const int l = BATCH ? bm.level[blockIdx.x] : a.level;
    const int64_t blk = BATCH ? bm.blk[blockIdx.x] : (int64_t)blockIdx.x;
    blk_bwd_unit<N, DO_Y, DO_COV, TR>(a, l, blk, (a.Nl[l] + 1) / 2, a.store_s && l >= 1, sm);
}

template <int N, bool DO_Y, bool DO_COV, bool BATCH>
__global__ __launch_bounds__(BGeo<N>::TBB) void k_blk_bwd_tail(BwdArgs a0, const BwdArgs *tab,
                                                               BlockMap bm) {
    const BwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    __shared__ double sm[BSmem<N>::PER];
    for (int l = a.level; l >= a.l_lo; --l) {
        const int64_t units = (a.Nl[l] + 1) / 2;
        for (int64_t t = 0; t < units; ++t)
            blk_bwd_unit<N, DO_Y, DO_COV, double>(a, l, t, units, a.store_s && l >= 1, sm);
        __threadfence();
        __syncthreads();
    }
}

// -------------------------------------------------------------- dispatch

template <int N, int MM, bool RAW, class T, class TIN>
static void launch_blk_fwd_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_forward<N, MM, RAW, T, TIN, false>), dim3((unsigned)a.units), dim3(BGeo<N>::TB),
                       0, s, a, nullptr, BlockMap{});
}
template <int N, int MM, bool RAW, class T, class TIN>
static void launch_blk_fwd_bt(const FwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_forward<N, MM, RAW, T, TIN, true>), dim3((unsigned)blocks), dim3(BGeo<N>::TB),
                       0, s, FwdArgs{}, tab, bm);
}
template <int N, int MM, bool RAW, class T, class TIN>
static void launch_blk_fold_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_fold<N, MM, RAW, T, TIN, false>), dim3(1), dim3(BGeo<N>::TB), 0, s, a,
                       nullptr, BlockMap{});
}
template <int N, int MM, bool RAW, class T, class TIN>
static void launch_blk_fold_bt(const FwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_fold<N, MM, RAW, T, TIN, true>), dim3((unsigned)blocks), dim3(BGeo<N>::TB), 0,
                       s, FwdArgs{}, tab, bm);
}
template <int N, int MM, bool RAW0>
static void launch_blk_fwd_tail_t(const FwdTailArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_fwd_tail<N, MM, RAW0, false>), dim3(1), dim3(BGeo<N>::TB), 0, s, a, nullptr,
                       BlockMap{});
}
template <int N, int MM, bool RAW0>
static void launch_blk_fwd_tail_bt(const FwdTailArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_fwd_tail<N, MM, RAW0, true>), dim3((unsigned)blocks), dim3(BGeo<N>::TB), 0, s,
                       FwdTailArgs{}, tab, bm);
}
template <int N, bool Y, bool COV, class TR>
static void launch_blk_bwd_t(const BwdArgs &a, hipStream_t s) {
    const int64_t units = (a.Nl[a.level] + 1) / 2;
    hipLaunchKernelGGL((k_blk_backward<N, Y, COV, TR, false>), dim3((unsigned)units), dim3(BGeo<N>::TBB), 0,
                       s, a, nullptr, BlockMap{});
}
template <int N, bool Y, bool COV, class TR>
static void launch_blk_bwd_bt(const BwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_backward<N, Y, COV, TR, true>), dim3((unsigned)blocks), dim3(BGeo<N>::TBB), 0,
                       s, BwdArgs{}, tab, bm);
}
template <int N, bool Y, bool COV>
static void launch_blk_bwd_tail_t(const BwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_bwd_tail<N, Y, COV, false>), dim3(1), dim3(BGeo<N>::TBB), 0, s, a, nullptr,
                       BlockMap{});
}
template <int N, bool Y, bool COV>
static void launch_blk_bwd_tail_bt(const BwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_bwd_tail<N, Y, COV, true>), dim3((unsigned)blocks), dim3(BGeo<N>::TBB), 0, s,
                       BwdArgs{}, tab, bm);
}

template <int N, int MM>
constexpr KernelSet make_blk_set() {
    return KernelSet{N,
                     MM,
                     {&launch_blk_fwd_t<N, MM, true, double, double>, &launch_blk_fwd_t<N, MM, true, float, double>},
                     {&launch_blk_fwd_t<N, MM, false, double, double>, &launch_blk_fwd_t<N, MM, false, float, float>,
                      &launch_blk_fwd_t<N, MM, false, double, float>},
                     {&launch_blk_fold_t<N, MM, true, double, double>, &launch_blk_fold_t<N, MM, true, float, double>},
                     {&launch_blk_fold_t<N, MM, false, double, double>, &launch_blk_fold_t<N, MM, false, float, float>,
                      &launch_blk_fold_t<N, MM, false, double, float>},
                     &launch_blk_fwd_tail_t<N, MM, true>,
                     &launch_blk_fwd_tail_t<N, MM, false>,
                     {{&launch_blk_bwd_t<N, true, false, double>, &launch_blk_bwd_t<N, true, false, float>},
                      {&launch_blk_bwd_t<N, false, true, double>, &launch_blk_bwd_t<N, false, true, float>},
                      {&launch_blk_bwd_t<N, true, true, double>, &launch_blk_bwd_t<N, true, true, float>}},
                     {&launch_blk_bwd_tail_t<N, true, false>, &launch_blk_bwd_tail_t<N, false, true>,
                      &launch_blk_bwd_tail_t<N, true, true>},
                     {&launch_blk_fwd_bt<N, MM, true, double, double>, &launch_blk_fwd_bt<N, MM, true, float, double>},
                     {&launch_blk_fwd_bt<N, MM, false, double, double>, &launch_blk_fwd_bt<N, MM, false, float, float>,
                      &launch_blk_fwd_bt<N, MM, false, double, float>},
                     {&launch_blk_fold_bt<N, MM, true, double, double>, &launch_blk_fold_bt<N, MM, true, float, double>},
                     {&launch_blk_fold_bt<N, MM, false, double, double>, &launch_blk_fold_bt<N, MM, false, float, float>,
                      &launch_blk_fold_bt<N, MM, false, double, float>},
                     &launch_blk_fwd_tail_bt<N, MM, true>,
                     &launch_blk_fwd_tail_bt<N, MM, false>,
                     {{&launch_blk_bwd_bt<N, true, false, double>, &launch_blk_bwd_bt<N, true, false, float>},
                      {&launch_blk_bwd_bt<N, false, true, double>, &launch_blk_bwd_bt<N, false, true, float>},
                      {&launch_blk_bwd_bt<N, true, true, double>, &launch_blk_bwd_bt<N, true, true, float>}},
                     {&launch_blk_bwd_tail_bt<N, true, false>, &launch_blk_bwd_tail_bt<N, false, true>,
                      &launch_blk_bwd_tail_bt<N, true, true>},
                     1,
                     0,
                     {1, 1, 1},
                     {0, 0, 0}};
}

#define KS_BLK_SETS(N) make_blk_set<N, (N + 1) / 2>(), make_blk_set<N, N>()

}  // namespace ks
