// ks_device_blk.h -- the workgroup family of the odd-even smoother kernels,
// for state dimensions whose units need more than one wavefront of lanes.
//
// Same algebra as the wavefront family (ks_device.h).  The forward levels
// (load, whitening, steps 1 to 3, the fold of odd levels, the base) are in
// ks_device_wg.h on a two-dimensional register tiling of each unit; this file
// holds the backward levels -- back-substitution and Algorithm 2 -- with one
// block row per workgroup, the covariance products on FP64 MFMA, and the
// kernel table of the family.
#pragma once

#include <type_traits>

#include "ks_device_wg.h"

namespace ks {

// records per backward workgroup, the default of each n (measured): one
// wavefront per record up to n = 12 (an R row fits its lanes, at most two P
// tiles), two up to n = 24, all four above (n = 32 loses with two: its LDS
// then allows one workgroup per CU).  Other counts are compiled as variants
// the autotuner can pick.
constexpr int blk_rpw(int n) { return (n <= 12) ? 4 : (n <= 24) ? 2 : 1; }

template <int N, int RPW_ = blk_rpw(N)>
struct BGeo {
    static constexpr int W = 3 * N + 1;                    // columns of an R row
    static constexpr int TBB = 256;                        // backward workgroup (four MFMA wavefronts)
    static constexpr int RPW = RPW_;                       // records per workgroup
    static constexpr int UT = TBB / RPW;                   // threads per record
    static constexpr int WPU = UT / 64;                    // wavefronts per record
    static constexpr int RREC = N * (3 * N + 1);
    static constexpr int OREC = N * (N + 1);
    static constexpr int EREC = N * (2 * N + 1);
    static constexpr int SREC = OREC + EREC;
};


// ------------------------------------------------------------ backward level

typedef double mf_d4 __attribute__((ext_vector_type(4)));

// LDS of one backward unit (doubles): region 0 holds R_ii, later P = T_I S_II,
// later S_ii; then T = R_ii^{-1} [R_i,b | rho | R_i,a], RI = R_ii^{-1}, the
// neighbour blocks S_aa, S_bb, S_ab, and 1 / R_ii(r, r)
template <int N, bool COV>
struct BSmem {
    static constexpr int LR = N + 1;                 // row stride of R_ii, RI, S_ii, S blocks
    static constexpr int LT = 2 * N + 1;             // row stride of T and P
    static constexpr int R0 = COV ? N * LT : N * LR; // region 0
    static constexpr int TO = R0;                    // T
    static constexpr int RO = TO + N * LT;           // RI and the S blocks (covariances only)
    static constexpr int DO = RO + (COV ? 4 * N * LR : 0);
    static constexpr int PER = DO + 3 * N;           // 1 / R_ii(r, r), y_a, y_b
};

// From n = 32 on, a record runs in the blocked form (blk_bwd_unit_bf): one
// wavefront forms R_ii^{-1} by substitution while another solves for the
// state, T_I comes from an MFMA product with R_ii^{-1}, the neighbours'
// covariance blocks pass through LDS one block at a time, and P stays in
// registers between its two products.  A record then needs 76 KB of LDS at
// n = 48 (151 KB in the form above), so two records share a CU.
constexpr bool blk_bf(int n) { return n >= 32; }  // n = 24: measured 2x slower than the LDS form

// LDS of one record in the blocked form (doubles): region 0 holds R_ii, then
// the neighbour block in use (S_aa, S_ab, S_bb in turn), then S_ii; then
// [R_i,b | rho | R_i,a] (later [T_b | . | T_a]), RI = R_ii^{-1}, and
// 1 / R_ii(r, r), y_a, y_b, w = rho - R_i,a y_a - R_i,b y_b
template <int N, bool COV>
struct BFSmem {
    static constexpr int LR = N + 1;
    static constexpr int LT = 2 * N + 1;
    static constexpr int TO = N * LR;
    static constexpr int IO = TO + N * LT;
    static constexpr int DO = IO + N * LR;
    static constexpr int PER = DO + 4 * N;
};

template <int N, bool COV>
constexpr int blk_per() { return blk_bf(N) ? BFSmem<N, COV>::PER : BSmem<N, COV>::PER; }

// wavefronts per SIMD the backward kernel is compiled for: two for the blocked
// form with covariances (its LDS admits two workgroups per CU), else one
template <int N, bool COV>
constexpr int blk_min_waves() { return (COV && blk_bf(N)) ? 2 : 1; }

// Synchronization inside one record's work.  A record taken by one
// wavefront (n <= 12) shares its LDS region with no other wavefront, and a
// wavefront's LDS accesses complete in order: fences that keep the compiler
// from reordering around a wavefront barrier suffice, and the other records
// of the workgroup run on without waiting.  Larger records span several
// wavefronts and use the workgroup barrier.
template <int WPU>
__device__ __forceinline__ void rec_sync() {
    if constexpr (WPU == 1) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One block row (record t of level l): back-substitution and Algorithm 2.
//  1. T = R_ii^{-1} [R_i,b | rho_i | R_i,a] and RI = R_ii^{-1}: one right-hand
//     side column per thread, column-oriented substitution (independent
//     updates after each x_r, so the dependent chain is n steps long).
//  2. y_i = z - T_a y_a - T_b y_b.
//  3. P = T_I S_II (T_I = [T_a | T_b], n x 2n; S_II the 2n x 2n covariance of
//     the neighbours, S_ab from whichever of them sits one level up) and
//     S_ii = RI RI^T + P T_I^T, both as 16x16x4 FP64 MFMA tiles (rows padded
//     to a multiple of 16); -P gives the blocks S_i,a S_i,b kept for lower
//     levels, S_ii is symmetrized on the way out.
// BGeo<N>::UT threads per record (the record's own LDS region sm); every
// thread of the workgroup must call it the same number of times.
template <int N, bool DO_Y, bool DO_COV, class TR, int RPW = blk_rpw(N)>
__device__ __forceinline__ void blk_bwd_unit_lds(const BwdArgs &a, int l, int64_t t, int64_t units,
                                                 bool store_s, double *sm) {
    using BG = BGeo<N, RPW>;
    using SM = BSmem<N, DO_COV>;
    constexpr int W = BG::W;
    constexpr int LR = SM::LR, LT = SM::LT;
    constexpr int NT = BG::UT;
    constexpr int WPU = BG::WPU;
    double *Rd = sm;                 // R_ii; then P; then S_ii
    double *TT = sm + SM::TO;        // [T_b | z | T_a]
    double *RI = sm + SM::RO;
    double *SA = RI + N * LR;        // S_aa, S_bb, S_ab (each n x LR)
    double *SB = SA + N * LR;
    double *SX = SB + N * LR;
    double *DI = sm + SM::DO;        // 1 / R_ii(r, r), then y_a, y_b
    const int g = threadIdx.x % NT;
    const bool valid = t < units;
    const int64_t i = ((2 * t + 1) << l) - 1;
    const int64_t aa = i - ((int64_t)1 << l), bb = i + ((int64_t)1 << l);
    const bool va = valid && aa >= 0, vb = valid && bb <= a.k;
    const TR *rec = slot<TR>(a.rrows_all, a.rec_off[l] + t, BG::RREC);

    // the neighbours' covariance blocks are fetched first and land in LDS after
    // the substitution, so their latency overlaps it
    constexpr int SPT = DO_COV ? (N * N + NT - 1) / NT : 1;
    double sa_[SPT], sb_[SPT], sx_[SPT];
    const double *sab = nullptr;
    bool trans = false;
    if constexpr (DO_COV) {
        if (va && vb) {
            const int la = __builtin_ctzll((unsigned long long)(aa + 1));
            if (la == l + 1) {
                sab = a.spm + (rec_of(aa, a.rec_off) - a.spm_first) * 2 * N * N + N * N;
            } else {
                sab = a.spm + (rec_of(bb, a.rec_off) - a.spm_first) * 2 * N * N;
                trans = true;
            }
        }
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int idx = g + NT * u;
            const bool in = idx < N * N;
            sa_[u] = (in && va) ? a.cov[aa * N * N + idx] : 0.0;
            sb_[u] = (in && vb) ? a.cov[bb * N * N + idx] : 0.0;
            sx_[u] = (in && sab) ? sab[idx] : 0.0;
        }
    }

    // the R row: every load issued before the first LDS store
    constexpr int RPL = (N * W + NT - 1) / NT;
    double rv[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
        const int idx = g + NT * u;
        rv[u] = (idx < N * W && valid) ? double(rec[idx]) : 0.0;
    }
    double ya = 0.0, yb = 0.0;  // neighbour states, element g
    if (DO_Y && g < N) {
        ya = va ? a.u_in[aa * N + g] : 0.0;
        yb = vb ? a.u_in[bb * N + g] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
        const int idx = g + NT * u;
        if (idx < N * W) {
            const int r = idx / W, c = idx - r * W;
            const double v = valid ? rv[u] : (c == r ? 1.0 : 0.0);
            // one store through a selected address (no branch per element)
            *(c < N ? Rd + r * LR + c : TT + r * LT + (c - N)) = v;
        }
    }
    if (DO_Y && g < N) {
        DI[N + g] = ya;
        DI[2 * N + g] = yb;
    }
    rec_sync<WPU>();
    if (g < N) DI[g] = rcp_nr(Rd[g * LR + g]);
    rec_sync<WPU>();
    if (g < W && (DO_COV || g >= N)) {
        double x[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            // x = e_g (g < n) or column g - n of the R part: one read by every
            // lane and a multiply-add (a select would become a branch per row)
            const double tv = TT[r * LT + (g < N ? 0 : g - N)];
            x[r] = fma(tv, g < N ? 0.0 : 1.0, r == g ? 1.0 : 0.0);
        }
#pragma unroll
        for (int r = N - 1; r >= 0; --r) {
            const double xr = x[r] * DI[r];
            x[r] = xr;
#pragma unroll
            for (int s = 0; s < r; ++s) x[s] = fma(-Rd[s * LR + r], xr, x[s]);
        }
        double *dst = g < N ? RI + g : TT + (g - N);
        const int ld = g < N ? LR : LT;
#pragma unroll
        for (int r = 0; r < N; ++r) dst[r * ld] = x[r];
    }
    if constexpr (DO_COV) {
        // S_ab(rr, cc) into SX[rr][cc] (S_ab is stored as S+ of a, or as S- of b, transposed)
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int idx = g + NT * u;
            if (idx < N * N) {
                const int r = idx / N, c = idx - r * N;
                SA[r * LR + c] = sa_[u];
                SB[r * LR + c] = sb_[u];
                if (trans) SX[c * LR + r] = sx_[u];
                else SX[r * LR + c] = sx_[u];
            }
        }
    }
    rec_sync<WPU>();
    // T_I(r, d): d < n the a-part (T_a), d >= n the b-part (T_b)
    auto TI = [&](int r, int d) -> double {
        return d < N ? TT[r * LT + N + 1 + d] : TT[r * LT + (d - N)];
    };
    if constexpr (DO_Y) {
        if (valid && g < N) {
            const double *ua = DI + N, *ub = DI + 2 * N;  // zero where a neighbour is missing
            double y0 = TT[g * LT + N], y1 = 0.0;
#pragma unroll 8
            for (int d = 0; d < N; ++d) {
                y0 = fma(-TI(g, d), ua[d], y0);
                y1 = fma(-TI(g, N + d), ub[d], y1);
            }
            a.u_out[i * N + g] = y0 + y1;
        }
    }
    if constexpr (DO_COV) {
        constexpr int TM = (N + 15) / 16;      // row tiles (rows >= n are zero)
        constexpr int TC = (2 * N + 15) / 16;  // column tiles of P (columns >= 2n are zero)
        constexpr int QP = (TM * TC + WPU - 1) / WPU;  // P tiles per wavefront
        constexpr int QS = (TM * TM + WPU - 1) / WPU;  // S tiles per wavefront
        constexpr int KP = (2 * N + 3) / 4;    // K steps of P (inner index >= 2n is zero)
        constexpr int KS = (3 * N + 3) / 4;    // K steps of S_ii (inner index >= 3n is zero)
        const int wave = __builtin_amdgcn_readfirstlane(g >> 6), lane = g & 63;
        const int lr = lane & 15, lk = lane >> 4;
        // S_II(d, c) for d, c < 2n (missing neighbours give zero blocks)
        auto SII = [&](int d, int c) -> double {
            if (d < N && c < N) return SA[d * LR + c];
            if (d >= N && c >= N) return SB[(d - N) * LR + (c - N)];
            return d < N ? SX[d * LR + (c - N)] : SX[c * LR + (d - N)];
        };
        // P = T_I S_II.  MFMA 16x16x4 FP64 operands: lane l holds A(l % 16, l / 16)
        // and B(l / 16, l % 16); the result D(l / 16 + 4 j, l % 16) in element j.
        // Tile q = ti + TM tj runs on wavefront q % WPU of the record.
        mf_d4 acc[QP];
#pragma unroll
        for (int u = 0; u < QP; ++u) acc[u] = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) {
            const int d = 4 * kk + lk;
#pragma unroll
            for (int u = 0; u < QP; ++u) {
                const int q = wave + WPU * u;
                if (q < TM * TC) {
                    const int ti = q % TM, tj = q / TM;
                    const int r = 16 * ti + lr;
                    const int cb = 16 * tj + lr;
                    const bool dk = (2 * N) % 4 == 0 || d < 2 * N;
                    const double av = r < N && dk ? TI(r, d) : 0.0;
                    const double bv = cb < 2 * N && dk ? SII(d, cb) : 0.0;
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
                }
            }
        }
        rec_sync<WPU>();  // R_ii no longer read: region 0 takes P
        double *PP = Rd;
#pragma unroll
        for (int u = 0; u < QP; ++u) {
            const int q = wave + WPU * u;
            if (q < TM * TC) {
                const int ti = q % TM, tj = q / TM;
                const int c = 16 * tj + lr;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = 16 * ti + lk + 4 * j;
                    if (r < N && c < 2 * N) {
                        PP[r * LT + c] = acc[u][j];
                        if (valid && store_s) {
                            const int64_t ri = a.rec_off[l] + t - a.spm_first;
                            double *dst = a.spm + ri * 2 * N * N + (c < N ? 0 : N * N);
                            dst[r * N + (c < N ? c : c - N)] = -acc[u][j];
                        }
                        // level 0: S_{i,i+1} = -P_b, and S_{i-1,i} = S_{i,i-1}^T = -P_a^T
                        if (l == 0 && a.lag1 && (c < N ? va : vb)) {
                            const int64_t off = c >= N ? i * N * N + r * N + (c - N) : (i - 1) * N * N + c * N + r;
                            a.lag1[off] = -acc[u][j];
                        }
                    }
                }
            }
        }
        rec_sync<WPU>();
        // S_ii = RI RI^T + P T_I^T: A = [RI | P] (n x 3n), B(k, c) = [RI | T_I](c, k)
        mf_d4 sc[QS];
#pragma unroll
        for (int u = 0; u < QS; ++u) sc[u] = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int k = 4 * kk + lk;
            const bool kin = (3 * N) % 4 == 0 || k < 3 * N;
#pragma unroll
            for (int u = 0; u < QS; ++u) {
                const int q = wave + WPU * u;
                if (q < TM * TM) {
                    const int ti = q % TM, tj = q / TM;
                    const int r = 16 * ti + lr, c = 16 * tj + lr;
                    double av = 0.0, bv = 0.0;
                    if (r < N && kin) av = k < N ? RI[r * LR + k] : PP[r * LT + (k - N)];
                    if (c < N && kin) bv = k < N ? RI[c * LR + k] : TI(c, k - N);
                    sc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, sc[u], 0, 0, 0);
                }
            }
        }
        rec_sync<WPU>();  // P no longer read: region 0 takes S_ii
        double *SS = Rd;
#pragma unroll
        for (int u = 0; u < QS; ++u) {
            const int q = wave + WPU * u;
            if (q < TM * TM) {
                const int ti = q % TM, tj = q / TM;
                const int c = 16 * tj + lr;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = 16 * ti + lk + 4 * j;
                    if (r < N && c < N) SS[r * LR + c] = sc[u][j];
                }
            }
        }
        rec_sync<WPU>();
        if (valid) {
            for (int idx = g; idx < N * N; idx += NT) {
                const int r = idx / N, c = idx - r * N;
                a.cov[i * N * N + idx] = 0.5 * (SS[r * LR + c] + SS[c * LR + r]);
            }
        }
    }
    rec_sync<WPU>();
}

__device__ __forceinline__ double blk_readlane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, lane);
    const long long hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((hi << 32) | lo);
}

// One block row in the blocked form (32 <= n <= 48, two or more wavefronts
// per record):
//  1. RI = R_ii^{-1} blocked by 16 (the recurrence of LAPACK's blocked
//     triangular inverse): wavefront 0 inverts the diagonal blocks by
//     substitution (lane 16 b + j: column j of block b), then the blocks above
//     them come from MFMA products, X_01 = -A^{-1} B D^{-1},
//     X_12 = -D^{-1} E F^{-1}, X_02 = -A^{-1} (B X_12 + C F^{-1}) for
//     R_ii = [A B C; 0 D E; 0 0 F].  Meanwhile wavefront 1 forms
//     w = rho_i - R_i,a y_a - R_i,b y_b and the others fetch S_aa, S_ab, S_bb;
//     then y_i = RI w.  A states-only pass stops there.
//  2. T_I = RI [R_i,a | R_i,b] on MFMA, written over the R part of the row.
//  3. P^T = S_II T_I^T: wavefront ti owns row tile ti of S_ii and forms the
//     column tiles (tk, ti) of P^T, with the operand S_II read from LDS in
//     three passes (S_aa, then S_ab, then S_bb in region 0; each tile takes
//     its K steps in increasing order across the passes).  Tile (tk, ti) in
//     the MFMA result layout is, element e, the A operand of K step 4 tk + e
//     of P T_I^T, so P goes from one product to the next in registers.
//  4. S_ii row tile ti = RI RI^T + P T_I^T, symmetrized on the way out; -P
//     gives the blocks S_i,a, S_i,b kept for lower levels (and the lag-one
//     blocks at level 0).
template <int N, bool DO_Y, bool DO_COV, class TR, int RPW>
__device__ __forceinline__ void blk_bwd_unit_bf(const BwdArgs &a, int l, int64_t t, int64_t units,
                                                bool store_s, double *sm) {
    using BG = BGeo<N, RPW>;
    using SM = BFSmem<N, DO_COV>;
    constexpr int W = BG::W;
    constexpr int LR = SM::LR, LT = SM::LT;
    constexpr int NT = BG::UT;
    constexpr int WPU = BG::WPU;
    constexpr int TM = (N + 15) / 16;      // row tiles of S_ii, T_I; column tiles of P^T
    constexpr int TC = (2 * N + 15) / 16;  // column tiles of T_I, row tiles of P^T
    static_assert(WPU >= 2 && WPU >= TM && N <= 48 && N % 4 == 0, "blocked form: record shape");
    double *Rd = sm;  // R_ii; then S_aa, S_ab, S_bb in turn; then S_ii
    double *TT = sm + SM::TO;
    double *RI = sm + SM::IO;
    double *DI = sm + SM::DO;
    const int g = threadIdx.x % NT;
    const int wave = __builtin_amdgcn_readfirstlane(g >> 6), lane = g & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const bool valid = t < units;
    const int64_t i = ((2 * t + 1) << l) - 1;
    const int64_t aa = i - ((int64_t)1 << l), bb = i + ((int64_t)1 << l);
    const bool va = valid && aa >= 0, vb = valid && bb <= a.k;
    const TR *rec = slot<TR>(a.rrows_all, a.rec_off[l] + t, BG::RREC);

    // the R row: every load issued before the first LDS store
    constexpr int RPL = (N * W + NT - 1) / NT;
    double rv[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
        const int idx = g + NT * u;
        rv[u] = (idx < N * W && valid) ? double(rec[idx]) : 0.0;
    }
    double ya = 0.0, yb = 0.0;  // neighbour states, element g
    if (DO_Y && g < N) {
        ya = va ? a.u_in[aa * N + g] : 0.0;
        yb = vb ? a.u_in[bb * N + g] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
        const int idx = g + NT * u;
        if (idx < N * W) {
            const int r = idx / W, c = idx - r * W;
            const double v = valid ? rv[u] : (c == r ? 1.0 : 0.0);
            // one store through a selected address (no branch per element)
            *(c < N ? Rd + r * LR + c : TT + r * LT + (c - N)) = v;
        }
    }
    if (DO_Y && g < N) {
        DI[N + g] = ya;
        DI[2 * N + g] = yb;
    }
    rec_sync<WPU>();
    if (g < N) DI[g] = rcp_nr(Rd[g * LR + g]);
    rec_sync<WPU>();

    // the neighbour blocks, one slice per thread of wavefronts 1 .. WPU-1
    constexpr int NTS = NT - 64;
    constexpr int NQ = DO_COV ? (N * N + NTS - 1) / NTS : 1;
    double q_aa[NQ], q_ab[NQ], q_bb[NQ];
    const double *sab = nullptr;
    bool trans = false;
    if constexpr (DO_COV) {
        if (va && vb) {
            const int la = __builtin_ctzll((unsigned long long)(aa + 1));
            if (la == l + 1) {
                sab = a.spm + (rec_of(aa, a.rec_off) - a.spm_first) * 2 * N * N + N * N;
            } else {
                sab = a.spm + (rec_of(bb, a.rec_off) - a.spm_first) * 2 * N * N;
                trans = true;
            }
        }
    }
    double *WV = DI + 3 * N;
    constexpr int NB = (N + 15) / 16;  // diagonal blocks of R_ii
    if (wave == 0) {
        // the diagonal blocks' inverses; rows and columns >= n (a last block
        // narrower than 16) are skipped through selects
        const int o = 16 * (lane >> 4), j = lane & 15;
        if (lane < 16 * NB && o + j < N) {
            double x[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) x[r] = r == j ? 1.0 : 0.0;
#pragma unroll
            for (int r = 15; r >= 0; --r) {
                const bool rin = o + r < N;
                const double xr = rin ? x[r] * DI[o + r] : 0.0;
                x[r] = xr;
#pragma unroll
                for (int s2 = 0; s2 < r; ++s2) {
                    const double rv = rin ? Rd[(o + s2) * LR + o + r] : 0.0;
                    x[s2] = fma(-rv, xr, x[s2]);
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (o + r < N) RI[(o + r) * LR + o + j] = x[r];
        }
    } else {
        if constexpr (DO_COV) {
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int idx = (g - 64) + NTS * u;
                const bool in = idx < N * N;
                q_aa[u] = (in && va) ? a.cov[aa * N * N + idx] : 0.0;
                q_ab[u] = (in && sab) ? sab[idx] : 0.0;
                q_bb[u] = (in && vb) ? a.cov[bb * N * N + idx] : 0.0;
            }
        }
        if (wave == 1) {
            if (DO_Y && lane < N) {
                // w = rho - R_i,a y_a - R_i,b y_b (lane g: row g)
                double w = TT[lane * LT + N];
#pragma unroll 8
                for (int d = 0; d < N; ++d) {
                    w = fma(-TT[lane * LT + N + 1 + d], DI[N + d], w);
                    w = fma(-TT[lane * LT + d], DI[2 * N + d], w);
                }
                WV[lane] = w;
            }
        }
        if (wave == WPU - 1) {
            // RI is upper triangular: zero the blocks below the diagonal ones
            for (int idx = lane; idx < N * N; idx += 64) {
                const int r = idx / N, c = idx - r * N;
                if ((r >> 4) > (c >> 4)) RI[r * LR + c] = 0.0;
            }
        }
    }
    rec_sync<WPU>();
    // the blocks above the diagonal: X_01 on wavefront 1, X_12 then X_02 on
    // wavefront 2 (1 when the record has two).  In each chain the first product
    // is formed transposed, so that its result layout is the next product's
    // operand layout.
    {
        // RI(o1 + r, o2 + c) = -(inv(o1) R(o1 : , o2 : ) inv(o2))(r, c) into
        // registers (result layout) and LDS
        auto x_above = [&](int o1, int o2) -> mf_d4 {
            mf_d4 t1 = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const bool in = o2 + lr < N && o1 + k < N;
                const double av = in ? Rd[(o1 + k) * LR + o2 + lr] : 0.0;  // R(o1 + k, o2 + lr)
                const bool bin = o1 + k < N && o1 + lr < N;
                const double bv = bin ? RI[(o1 + lr) * LR + o1 + k] : 0.0;  // inv(o1)(lr, k)
                t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, t1, 0, 0, 0);
            }
            // t1[e] = (inv(o1) R_12)(lr, lk + 4 e)
            mf_d4 x = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const bool in = o2 + k < N && o2 + lr < N;
                const double bv = in ? RI[(o2 + k) * LR + o2 + lr] : 0.0;  // inv(o2)(k, lr)
                x = __builtin_amdgcn_mfma_f64_16x16x4f64(t1[kk], bv, x, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                x[e] = -x[e];
                if (o2 + lr < N) RI[(o1 + lk + 4 * e) * LR + o2 + lr] = x[e];
            }
            return x;
        };
        if (NB >= 2 && wave == 1) (void)x_above(0, 16);
        if constexpr (NB == 3) {
            if (wave == (WPU >= 3 ? 2 : 1)) {
                const mf_d4 x12 = x_above(16, 32);
                // Z = R_01 X_12 + R_02 inv(2), then X_02 = -inv(0) Z
                mf_d4 z = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    z = __builtin_amdgcn_mfma_f64_16x16x4f64(Rd[lr * LR + 16 + k], x12[kk], z, 0, 0, 0);
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    z = __builtin_amdgcn_mfma_f64_16x16x4f64(Rd[lr * LR + 32 + k], RI[(32 + k) * LR + 32 + lr], z, 0,
                                                              0, 0);
                }
                mf_d4 x02 = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    x02 = __builtin_amdgcn_mfma_f64_16x16x4f64(RI[lr * LR + k], z[kk], x02, 0, 0, 0);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) RI[(lk + 4 * e) * LR + 32 + lr] = -x02[e];
            }
        }
    }
    rec_sync<WPU>();  // RI complete; R_ii no longer read: region 0 takes S_aa
    if (DO_Y && wave == WPU - 1 && lane < N) {
        // y_i = RI w
        double y = 0.0;
#pragma unroll 8
        for (int k = 0; k < N; ++k) y = fma(RI[lane * LR + k], WV[k], y);
        if (valid) a.u_out[i * N + lane] = y;
    }
    if constexpr (!DO_COV) {
        rec_sync<WPU>();
        return;
    }

    // T_I(r, d) = [T_a | T_b](r, d) in [T_b | . | T_a] (same place as the R part)
    auto TX = [&](int r, int d) -> double { return d < N ? TT[r * LT + N + 1 + d] : TT[r * LT + (d - N)]; };
    if (wave > 0) {
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int idx = (g - 64) + NTS * u;
            if (idx < N * N) Rd[(idx / N) * LR + idx % N] = q_aa[u];
        }
    }
    constexpr int QT = (TM * TC + WPU - 1) / WPU;  // T_I tiles per wavefront
    constexpr int KN = N / 4;                      // K steps over n
    mf_d4 tacc[QT];
#pragma unroll
    for (int u = 0; u < QT; ++u) {
        tacc[u] = mf_d4{0.0, 0.0, 0.0, 0.0};
        const int q = wave + WPU * u;
        if (q < TM * TC) {
            const int ti = q % TM, tj = q / TM;
            const int r = 16 * ti + lr, cb = 16 * tj + lr;
#pragma unroll
            for (int kk = 0; kk < KN; ++kk) {  // RI(r, k) = 0 for k < 16 ti
                const int k = 4 * kk + lk;
                const double av = r < N ? RI[r * LR + k] : 0.0;
                const double bv = cb < 2 * N ? TX(k, cb) : 0.0;
                tacc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, tacc[u], 0, 0, 0);
            }
        }
    }
    rec_sync<WPU>();  // the R part is no longer read: T_I takes its place
#pragma unroll
    for (int u = 0; u < QT; ++u) {
        const int q = wave + WPU * u;
        if (q < TM * TC) {
            const int ti = q % TM, tj = q / TM;
            const int cb = 16 * tj + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * ti + lk + 4 * e;
                if (r < N && cb < 2 * N) TT[r * LT + (cb < N ? N + 1 + cb : cb - N)] = tacc[u][e];
            }
        }
    }
    rec_sync<WPU>();

    // P^T column tile ti = wave: three passes over the neighbour blocks
    const int ti = wave;
    const bool own = ti < TM;
    const int c = 16 * ti + lr;  // the row of T_I this lane's B operand reads
    mf_d4 pt[TC];
#pragma unroll
    for (int tk = 0; tk < TC; ++tk) pt[tk] = mf_d4{0.0, 0.0, 0.0, 0.0};
    // pass Q: S_aa (Q = 0), S_ab (1), S_bb (2) in region 0, S_ab as S_ab(x, y) at x LR + y
    auto pass = [&](auto qc) {
        constexpr int Q = decltype(qc)::value;
        if (!own) return;
#pragma unroll
        for (int kk = 0; kk < 2 * KN; ++kk) {
            const bool dlo = kk < KN;  // d = 4 kk + lk < n
            const int d = 4 * kk + lk;
            const double bv = c < N ? TX(c, d) : 0.0;
#pragma unroll
            for (int tk = 0; tk < TC; ++tk) {
                const bool plo = 16 * tk < N, phi = 16 * tk + 15 >= N;  // tile has rows p < n / p >= n
                const bool run = Q == 0 ? (plo && dlo) : Q == 1 ? ((plo && !dlo) || (phi && dlo)) : (phi && !dlo);
                if (!run) continue;
                const int p = 16 * tk + lr;
                double av;
                if constexpr (Q == 0) {
                    av = p < N ? Rd[p * LR + d] : 0.0;
                } else if constexpr (Q == 1) {
                    av = p < N ? (dlo ? 0.0 : Rd[p * LR + (d - N)])
                               : (p < 2 * N && dlo ? Rd[d * LR + (p - N)] : 0.0);
                } else {
                    av = (p >= N && p < 2 * N) ? Rd[(p - N) * LR + (d - N)] : 0.0;
                }
                pt[tk] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, pt[tk], 0, 0, 0);
            }
        }
    };
    pass(std::integral_constant<int, 0>{});
    rec_sync<WPU>();
    if (wave > 0) {
        // S_ab(rr, cc) into [rr][cc] (stored as S+ of a, or as S- of b, transposed)
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int idx = (g - 64) + NTS * u;
            if (idx < N * N) {
                const int rr = idx / N, cc = idx - rr * N;
                Rd[trans ? cc * LR + rr : rr * LR + cc] = q_ab[u];
            }
        }
    }
    rec_sync<WPU>();
    pass(std::integral_constant<int, 1>{});
    rec_sync<WPU>();
    if (wave > 0) {
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int idx = (g - 64) + NTS * u;
            if (idx < N * N) Rd[(idx / N) * LR + idx % N] = q_bb[u];
        }
    }
    rec_sync<WPU>();
    pass(std::integral_constant<int, 2>{});

    mf_d4 sc[TM];
    if (own) {
        // pt[tk][e] = P(c, 16 tk + lk + 4 e): -P into the S blocks / lag-one blocks
#pragma unroll
        for (int tk = 0; tk < TC; ++tk) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int cc = 16 * tk + lk + 4 * e;
                if (c < N && cc < 2 * N) {
                    const double v = pt[tk][e];
                    if (valid && store_s) {
                        const int64_t ri = a.rec_off[l] + t - a.spm_first;
                        double *dst = a.spm + ri * 2 * N * N + (cc < N ? 0 : N * N);
                        dst[c * N + (cc < N ? cc : cc - N)] = -v;
                    }
                    // level 0: S_{i,i+1} = -P_b, and S_{i-1,i} = S_{i,i-1}^T = -P_a^T
                    if (l == 0 && a.lag1 && (cc < N ? va : vb)) {
                        if (cc >= N) a.lag1[i * N * N + c * N + (cc - N)] = -v;
                        else a.lag1[(i - 1) * N * N + cc * N + c] = -v;
                    }
                }
            }
        }
        // S_ii row tile ti: RI RI^T over k < n, then P T_I^T over d < 2n with P from pt
#pragma unroll
        for (int tj = 0; tj < TM; ++tj) sc[tj] = mf_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
        for (int kk = 0; kk < KN; ++kk) {
            const int k = 4 * kk + lk;
            const double av = c < N ? RI[c * LR + k] : 0.0;
#pragma unroll
            for (int tj = 0; tj < TM; ++tj) {
                const int cb = 16 * tj + lr;
                const double bv = cb < N ? RI[cb * LR + k] : 0.0;
                sc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, sc[tj], 0, 0, 0);
            }
        }
#pragma unroll
        for (int kk = 0; kk < 4 * TC; ++kk) {
            const int d = 4 * kk + lk;
            const double av = pt[kk / 4][kk % 4];
#pragma unroll
            for (int tj = 0; tj < TM; ++tj) {
                const int cb = 16 * tj + lr;
                const double bv = (cb < N && d < 2 * N) ? TX(cb, d) : 0.0;
                sc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, sc[tj], 0, 0, 0);
            }
        }
    }
    rec_sync<WPU>();  // S_bb no longer read: region 0 takes S_ii
    if (own) {
#pragma unroll
        for (int tj = 0; tj < TM; ++tj) {
            const int cb = 16 * tj + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * ti + lk + 4 * e;
                if (r < N && cb < N) Rd[r * LR + cb] = sc[tj][e];
            }
        }
    }
    rec_sync<WPU>();
    if (valid) {
        for (int idx = g; idx < N * N; idx += NT) {
            const int r = idx / N, cc = idx - r * N;
            a.cov[i * N * N + idx] = 0.5 * (Rd[r * LR + cc] + Rd[cc * LR + r]);
        }
    }
    rec_sync<WPU>();
}

// the record slot of this thread's wavefront in its workgroup; a record spans
// whole wavefronts (UT a multiple of 64), so the value is uniform over the
// wavefront, and read from its first lane the compiler knows it: the record's
// indices, pointers and validity then live in scalar registers and the
// branches on them are scalar
template <int UT>
__device__ __forceinline__ int blk_record_slot() {
    static_assert(UT % 64 == 0, "a record spans whole wavefronts");
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / UT));
}

template <int N, bool DO_Y, bool DO_COV, class TR, int RPW = blk_rpw(N)>
__device__ __forceinline__ void blk_bwd_unit(const BwdArgs &a, int l, int64_t t, int64_t units, bool store_s,
                                             double *sm) {
    if constexpr (blk_bf(N))
        blk_bwd_unit_bf<N, DO_Y, DO_COV, TR, RPW>(a, l, t, units, store_s, sm);
    else
        blk_bwd_unit_lds<N, DO_Y, DO_COV, TR, RPW>(a, l, t, units, store_s, sm);
}

template <int N, bool DO_Y, bool DO_COV, class TR, bool BATCH, int RPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(blk_min_waves<N, DO_COV>()))) void
k_blk_backward(BwdArgs a0, const BwdArgs *tab, BlockMap bm) {
    const BwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    using BG = BGeo<N, RPW>;
    constexpr int PER = blk_per<N, DO_COV>();
    __shared__ double sm[BG::RPW * PER];
    const int l = BATCH ? bm.level[blockIdx.x] : a.level;
    const int64_t blk = BATCH ? bm.blk[blockIdx.x] : (int64_t)blockIdx.x;
    const int u = blk_record_slot<BG::UT>();
    blk_bwd_unit<N, DO_Y, DO_COV, TR, RPW>(a, l, blk * BG::RPW + u, (a.Nl[l] + 1) / 2, a.store_s && l >= 1,
                                           sm + u * PER);
}

template <int N, bool DO_Y, bool DO_COV, bool BATCH, int RPW>
__global__ __launch_bounds__(256) void k_blk_bwd_tail(BwdArgs a0, const BwdArgs *tab, BlockMap bm) {
    const BwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    using BG = BGeo<N, RPW>;
    constexpr int PER = blk_per<N, DO_COV>();
    __shared__ double sm[BG::RPW * PER];
    const int u = blk_record_slot<BG::UT>();
    for (int l = a.level; l >= a.l_lo; --l) {
        const int64_t units = (a.Nl[l] + 1) / 2;
        for (int64_t t0 = 0; t0 < units; t0 += BG::RPW)
            blk_bwd_unit<N, DO_Y, DO_COV, double, RPW>(a, l, t0 + u, units, a.store_s && l >= 1, sm + u * PER);
        __syncthreads();  // the next level reads what this workgroup wrote: workgroup scope suffices
    }
}

// Backward levels a.level down to a.l_lo in one launch (subtree fusion):
// workgroup c owns the records whose columns i satisfy
// c 2^(level+1) < i + 1 < (c+1) 2^(level+1), i.e. records
// [c 2^(level-l), (c+1) 2^(level-l)) of level l.  Every neighbour such a record
// reads (i +- 2^l, and the S block one of them stored) lies inside that range,
// where this workgroup wrote it one level up, or on its ends, which earlier
// launches wrote; so levels are separated by workgroup barriers only.
template <int N, bool DO_Y, bool DO_COV, class TR, int RPW>
__global__ __launch_bounds__(256) void k_blk_bwd_multi(BwdArgs a) {
    using BG = BGeo<N, RPW>;
    constexpr int PER = blk_per<N, DO_COV>();
    __shared__ double sm[BG::RPW * PER];
    const int u = blk_record_slot<BG::UT>();
    const int64_t c = blockIdx.x;
    for (int l = a.level; l >= a.l_lo; --l) {
        const int64_t recs = (a.Nl[l] + 1) / 2;
        const int64_t span = (int64_t)1 << (a.level - l);
        const int64_t lo = c * span;
        const int64_t hi = lo + span < recs ? lo + span : recs;
        for (int64_t t0 = lo; t0 < hi; t0 += BG::RPW)
            blk_bwd_unit<N, DO_Y, DO_COV, TR, RPW>(a, l, t0 + u, hi, a.store_s && l >= 1, sm + u * PER);
        __syncthreads();  // the next level reads what this workgroup's records wrote
    }
}

// -------------------------------------------------------------- dispatch

template <int N, bool Y, bool COV, class TR, int RPW>
static void launch_blk_bwd_t(const BwdArgs &a, hipStream_t s) {
    const int64_t units = (a.Nl[a.level] + 1) / 2;
    const int64_t blocks = (units + RPW - 1) / RPW;
    hipLaunchKernelGGL((k_blk_backward<N, Y, COV, TR, false, RPW>), dim3((unsigned)blocks), dim3(256), 0, s, a,
                       nullptr, BlockMap{});
}
template <int N, bool Y, bool COV, class TR, int RPW>
static void launch_blk_bwd_bt(const BwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_backward<N, Y, COV, TR, true, RPW>), dim3((unsigned)blocks), dim3(256), 0, s,
                       BwdArgs{}, tab, bm);
}
template <int N, bool Y, bool COV, int RPW>
static void launch_blk_bwd_tail_t(const BwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_bwd_tail<N, Y, COV, false, RPW>), dim3(1), dim3(256), 0, s, a, nullptr,
                       BlockMap{});
}
template <int N, bool Y, bool COV, int RPW>
static void launch_blk_bwd_tail_bt(const BwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_blk_bwd_tail<N, Y, COV, true, RPW>), dim3((unsigned)blocks), dim3(256), 0, s,
                       BwdArgs{}, tab, bm);
}
template <int N, bool Y, bool COV, class TR, int RPW>
static void launch_blk_bwd_multi_t(const BwdArgs &a, hipStream_t s) {
    const int64_t recs = (a.Nl[a.l_lo] + 1) / 2;
    const int64_t span = (int64_t)1 << (a.level - a.l_lo);
    const int64_t blocks = (recs + span - 1) / span;
    hipLaunchKernelGGL((k_blk_bwd_multi<N, Y, COV, TR, RPW>), dim3((unsigned)blocks), dim3(256), 0, s, a);
}

// Every backward entry of a kernel set from the MFMA family with RPW records
// per workgroup (all three modes, both record types, single / batched /
// tail / group launches), so every mode comes from one family.
template <int N, int RPW>
constexpr void set_blk_bwd(KernelSet &s) {
    s.bwd[BWD_Y][0] = &launch_blk_bwd_t<N, true, false, double, RPW>;
    s.bwd[BWD_Y][1] = &launch_blk_bwd_t<N, true, false, float, RPW>;
    s.bwd[BWD_COV][0] = &launch_blk_bwd_t<N, false, true, double, RPW>;
    s.bwd[BWD_COV][1] = &launch_blk_bwd_t<N, false, true, float, RPW>;
    s.bwd[BWD_BOTH][0] = &launch_blk_bwd_t<N, true, true, double, RPW>;
    s.bwd[BWD_BOTH][1] = &launch_blk_bwd_t<N, true, true, float, RPW>;
    s.bwd_tail[BWD_Y] = &launch_blk_bwd_tail_t<N, true, false, RPW>;
    s.bwd_tail[BWD_COV] = &launch_blk_bwd_tail_t<N, false, true, RPW>;
    s.bwd_tail[BWD_BOTH] = &launch_blk_bwd_tail_t<N, true, true, RPW>;
    s.bwd_b[BWD_Y][0] = &launch_blk_bwd_bt<N, true, false, double, RPW>;
    s.bwd_b[BWD_Y][1] = &launch_blk_bwd_bt<N, true, false, float, RPW>;
    s.bwd_b[BWD_COV][0] = &launch_blk_bwd_bt<N, false, true, double, RPW>;
    s.bwd_b[BWD_COV][1] = &launch_blk_bwd_bt<N, false, true, float, RPW>;
    s.bwd_b[BWD_BOTH][0] = &launch_blk_bwd_bt<N, true, true, double, RPW>;
    s.bwd_b[BWD_BOTH][1] = &launch_blk_bwd_bt<N, true, true, float, RPW>;
    s.bwd_tail_b[BWD_Y] = &launch_blk_bwd_tail_bt<N, true, false, RPW>;
    s.bwd_tail_b[BWD_COV] = &launch_blk_bwd_tail_bt<N, false, true, RPW>;
    s.bwd_tail_b[BWD_BOTH] = &launch_blk_bwd_tail_bt<N, true, true, RPW>;
    s.bwd_multi[BWD_Y][0] = &launch_blk_bwd_multi_t<N, true, false, double, RPW>;
    s.bwd_multi[BWD_Y][1] = &launch_blk_bwd_multi_t<N, true, false, float, RPW>;
    s.bwd_multi[BWD_COV][0] = &launch_blk_bwd_multi_t<N, false, true, double, RPW>;
    s.bwd_multi[BWD_COV][1] = &launch_blk_bwd_multi_t<N, false, true, float, RPW>;
    s.bwd_multi[BWD_BOTH][0] = &launch_blk_bwd_multi_t<N, true, true, double, RPW>;
    s.bwd_multi[BWD_BOTH][1] = &launch_blk_bwd_multi_t<N, true, true, float, RPW>;
    for (int q = 0; q < 3; ++q) {
        s.upb_bwd[q] = RPW;
        s.upb_bwd_tail[q] = 0;
    }
    s.rpp_multi = RPW;
}

template <int N, int MM>
constexpr KernelSet make_blk_set_base() {
    return KernelSet{N,
                     MM,
                     {&launch_wg_fwd_t<N, MM, true, double, double>, &launch_wg_fwd_t<N, MM, true, float, double>},
                     {&launch_wg_fwd_t<N, MM, false, double, double>, &launch_wg_fwd_t<N, MM, false, float, float>,
                      &launch_wg_fwd_t<N, MM, false, double, float>},
                     {&launch_wg_fold_t<N, MM, true, double, double>, &launch_wg_fold_t<N, MM, true, float, double>},
                     {&launch_wg_fold_t<N, MM, false, double, double>, &launch_wg_fold_t<N, MM, false, float, float>,
                      &launch_wg_fold_t<N, MM, false, double, float>},
                     &launch_wg_fwd_tail_t<N, MM, true>,
                     &launch_wg_fwd_tail_t<N, MM, false>,
                     {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}},  // backward: set_blk_bwd
                     {nullptr, nullptr, nullptr},
                     {&launch_wg_fwd_bt<N, MM, true, double, double>, &launch_wg_fwd_bt<N, MM, true, float, double>},
                     {&launch_wg_fwd_bt<N, MM, false, double, double>, &launch_wg_fwd_bt<N, MM, false, float, float>,
                      &launch_wg_fwd_bt<N, MM, false, double, float>},
                     {&launch_wg_fold_bt<N, MM, true, double, double>, &launch_wg_fold_bt<N, MM, true, float, double>},
                     {&launch_wg_fold_bt<N, MM, false, double, double>, &launch_wg_fold_bt<N, MM, false, float, float>,
                      &launch_wg_fold_bt<N, MM, false, double, float>},
                     &launch_wg_fwd_tail_bt<N, MM, true>,
                     &launch_wg_fwd_tail_bt<N, MM, false>,
                     {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}},
                     {nullptr, nullptr, nullptr},
                     1,
                     1,
                     {0, 0, 0},
                     {0, 0, 0},
                     {&launch_wg_fwd_fold_t<N, MM, double, double>, &launch_wg_fwd_fold_t<N, MM, float, float>,
                      &launch_wg_fwd_fold_t<N, MM, double, float>}};
}

// Forward on the two-dimensional tiling, backward on MFMA with RPW records
// per workgroup (backward variant bv of the set)
template <int N, int MM, int RPW, int BV>
constexpr KernelSet make_blk_set() {
    KernelSet s = make_blk_set_base<N, MM>();
    set_blk_bwd<N, RPW>(s);
    s.bv = BV;
    return s;
}

// the default of each n first, then its backward variants
#define KS_BLK_SETS_MM(N, MM)                                                                         \
    make_blk_set<N, MM, blk_rpw(N), 0>(), make_blk_set<N, MM, (blk_rpw(N) == 1 ? 2 : 1), 1>()
#define KS_BLK_SETS(N) KS_BLK_SETS_MM(N, wg_mm_small(N)), KS_BLK_SETS_MM(N, N)
#define KS_BLK_SETS_ONE(N) make_blk_set<N, wg_mm_small(N), 1, 0>(), make_blk_set<N, N, 1, 0>()

// Wavefront-family forward (register-resident units, no barriers) with the
// workgroup-family backward (MFMA SelInv; any n: rows, columns and inner
// indices beyond the block sizes are zero-padded to the 16 x 16 x 4 tiles).
// Both families write and read the same R-record layout [R_ii | R_i,right |
// rho_i | R_i,left] (FP32 records in the first half of their slot), so the
// halves combine freely.  Every backward mode (states only, covariances only,
// both) comes from the same family, so the states of a states-only pass are
// bitwise those of a full pass.  Backward variants: RPW records per
// workgroup; forward variant 1: the level-0 kernel without LDS staging.
template <int N, int MM, int RPW, int BV>
constexpr KernelSet make_hyb_set() {
    KernelSet s = make_set<N, MM>();
    set_blk_bwd<N, RPW>(s);
    s.bv = BV;
    return s;
}

#define KS_HYB_SETS_MM(N, MM)                                                                         \
    make_hyb_set<N, MM, 4, 0>(), make_hyb_set<N, MM, 2, 1>(), make_hyb_set<N, MM, 1, 2>(),            \
        make_set_unstaged<N, MM>()
#define KS_HYB_SETS(N) KS_HYB_SETS_MM(N, (N + 1) / 2), KS_HYB_SETS_MM(N, N), KS_HYB_SETS_MM(N, 2 * N)

// Wavefront family throughout (n = 1, 2, 3, 5), with the MFMA backward as
// backward variant 1 and the unstaged level 0 as forward variant 1
#define KS_SETS_MM(N, MM) make_set<N, MM>(), make_hyb_set<N, MM, 4, 1>(), make_set_unstaged<N, MM>()
#define KS_SETS(N) KS_SETS_MM(N, (N + 1) / 2), KS_SETS_MM(N, N), KS_SETS_MM(N, 2 * N)

}  // namespace ks
