// ks_device_mf.h -- forward elimination on the FP64 matrix cores (MFMA) for
// state dimensions that are multiples of 16 (n = 32, 48).
//
// One unit (Section III's steps 1 to 3 for even column j = 2t of a level and
// its right neighbour) per 256-thread workgroup.  Every stack lives in
// registers as 16 x 16 tiles in the result layout of the 16x16x4 FP64 MFMA:
// lane l holds rows l/16 + 4e (e = 0..3) of column l%16 of a tile.  Column
// tile ct belongs to wavefront ct % 4, with all of its row tiles, so a column
// never leaves its wavefront.
//
// Each QR runs blocked, with the compact WY form of a product of Householder
// reflectors (Q = H_0 .. H_15 = I - V T V^T, T upper triangular; Golub & Van
// Loan, Matrix Computations, 5.2.3): the wavefront owning panel P (16 pivot
// columns) factors it with unblocked Householder steps in registers (column
// sums over the four lanes of a column by lane shuffles, each reflector
// published in LDS for the lanes of the other columns) and writes V and T to
// LDS; then every wavefront applies Q^T = I - V T^T V^T to its tiles right of
// the panel as three MFMA chains (Y = V^T C, W = T^T Y, C -= V W).  The owner
// of the next panel updates that tile first and factors it while the others
// finish their updates; V and T are double-buffered, so a panel costs one
// workgroup barrier.
//
// Column tiles: step 1 [u_j | u_{j+1} | rhs], step 2 [u_j | u_{j+1} | rhs |
// u_{j-1}] (the order of non-pivot columns is free: the tiles step 1 leaves
// in rows [0, n) keep their wavefront and move down to rows [n, 2n) by
// renaming), step 3 [u_{j+1} | rhs].  Level 0 reads the raw inputs and
// whitens them by row scaling: the kernel set that uses this forward is only
// chosen for problems with diagonal covariances (problems with dense ones run
// the workgroup family; should one reach this kernel it reports KS_E_NOT_SPD
// rather than a wrong result).  Levels >= 1 read the reduced systems.  Inputs
// and outputs are those of the workgroup family: the same records,
// statistics and flags.
#pragma once

#include <type_traits>

#include "ks_device_blk.h"

namespace ks {

typedef double mf4 __attribute__((ext_vector_type(4)));

constexpr int mf_max(int a, int b) { return a > b ? a : b; }

// wavefronts per SIMD the kernel is compiled for: two units per CU at n = 48
// (its tiles take 144 of 256 registers), three at n = 32
constexpr int mf_min_waves(int n) { return n <= 32 ? 3 : 2; }

template <int N, int MM, bool RAW>
struct MfGeo {
    static_assert(N % 16 == 0, "the MFMA forward needs n a multiple of 16");
    static constexpr int NB = N / 16;               // pivot panels of every QR
    static constexpr int RO = RAW ? MM : N;         // observation rows of a column
    static_assert(2 * RO >= N && RO <= N, "observation class outside the MFMA forward");
    static constexpr int R1 = (RO + N + 15) / 16;   // row tiles: step 1 [O_j ; E_{j+1}]
    static constexpr int R2 = 2 * NB;               // step 2 [E_j ; R~_j]
    static constexpr int R3 = (2 * RO + 15) / 16;   // step 3 [D~_{j+1} ; O_{j+1}]
    static constexpr int C1 = 2 * NB + 1, C2 = 3 * NB + 1, C3 = NB + 1;  // column tiles
    static constexpr int RM = mf_max(R1, mf_max(R2, R3));
    static constexpr int KM = (C2 + 3) / 4;         // column tiles per wavefront
    // V of a panel, reflector i's entries in this lane order: [i][q][rt][e]
    // holds row 16 rt + 4 e + q (odd stride: conflict-free column reads)
    static constexpr int VLDT = 16 * RM + 1;
    static constexpr int DLD = N + 1;               // [D~ | gamma] rows in LDS
    // Steps 2 and 3 at once: where n = 48 and the step-3 stack has three row
    // tiles, its four column tiles fit, two by two, in the column-tile slot
    // KM - 1 that wavefronts 2 and 3 leave empty in step 2
    static constexpr bool CONC = NB == 3 && 2 * R3 <= RM && 2 + 4 * (KM - 1) >= C2;
    static constexpr int RREC = N * (3 * N + 1);
    static constexpr int OREC = N * (N + 1);
    static constexpr int EREC = N * (2 * N + 1);
    static constexpr int SREC = OREC + EREC;
};

template <int B, int E, class F>
__device__ __forceinline__ void mf_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        mf_for<B + 1, E>(f);
    }
}

// v on lane `lane` (a wavefront-uniform lane index)
__device__ __forceinline__ double mf_readlane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, lane);
    const long long hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)((unsigned long long)hi << 32) | lo);
}

// x + (x of lane l ^ D) for D = 16 or 32, by the lane-swap instructions (no
// LDS); both lanes of a pair add the same two operands in the same order, so
// they get the same bits
template <int D>
__device__ __forceinline__ double mf_swapsum(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)b, hi = (unsigned)((unsigned long long)b >> 32);
    if constexpr (D == 16) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    }
}

// sum over the four lanes holding one tile column (lanes c, c+16, c+32, c+48);
// all four get the same bits
__device__ __forceinline__ double mf_colsum(double v) { return mf_swapsum<32>(mf_swapsum<16>(v)); }

__device__ __forceinline__ void mf_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ mf4 mf_mma(double a, double b, mf4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// the register tiles of one wavefront: column tiles w + 4k, row tiles rt
template <int N, int MM, bool RAW>
using MfTiles = mf4[MfGeo<N, MM, RAW>::KM][MfGeo<N, MM, RAW>::RM];

// LDS of one unit
template <int N, int MM, bool RAW>
struct MfLds {
    using G = MfGeo<N, MM, RAW>;
    double v[2][16 * G::VLDT];   // V of the current and the next panel
    double t[2][256];            // T of the current and the next panel
    double g[256];               // V^T V of the panel being factored
    double tau[16];              // its reflector coefficients
    double d[G::RO * G::DLD];    // [D~_{j+1} | gamma] between steps 1 and 3
    // the same for step 3 while step 2 runs (CONC)
    double v3[G::CONC ? 2 : 1][G::CONC ? 16 * G::VLDT : 1];
    double t3[G::CONC ? 2 : 1][G::CONC ? 256 : 1];
    double g3[G::CONC ? 256 : 1];
    double tau3[16];
};

// index of V(row, i) in a V buffer
template <int RM>
__device__ __forceinline__ int mf_vidx(int i, int row) {
    return i * (16 * RM + 1) + (row & 3) * (4 * RM) + (row >> 4) * 4 + ((row & 15) >> 2);
}

// ----------------------------------------------------------------- panel QR

// One unblocked Householder step, pivot I of panel P, on the owner's column
// tile x (rows [16P, 16R) take part): H_I = I - tau v v^T with v = (1,
// x_{p+1} / (alpha - beta), ...), beta = -sign(alpha) ||x_{p:}|| (sign(+0) =
// +1), tau = (beta - alpha) / beta; the identity when the part below the pivot
// is zero.  Every lane applies it to its own column; the pivot column itself
// becomes (.., beta, ~0, ..) and columns left of the pivot change only below
// their diagonal, which no later step reads as R.
// sum of squares of this lane's column over rows 16P + I + 1 .. 16R - 1, over
// the four lanes of the column (four partial sums: short dependency chains)
template <int RM, int R, int P, int OFF>
__device__ __forceinline__ double mf_below(const mf4 (&x)[RM], int I, int q) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rt = P; rt < R; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double v = x[OFF + rt][e];
            s4[e] = (rt > P || 4 * e + q > I) ? fma(v, v, s4[e]) : s4[e];
        }
    return mf_colsum((s4[0] + s4[1]) + (s4[2] + s4[3]));
}

// ss: mf_below for pivot I on entry, for pivot I + 1 on return (formed right
// after the update that fixes column I + 1, so the next pivot starts from it)
template <int RM, int R, int P, int OFF>
__device__ __forceinline__ void mf_pivot(mf4 (&x)[RM], int I, double &ss, double *vl, double *tau_lds, int c,
                                         int q) {
    const double xn2 = mf_readlane(ss, I);
    const int ei = I >> 2;
    const double xa = ei == 0 ? x[OFF + P][0] : ei == 1 ? x[OFF + P][1] : ei == 2 ? x[OFF + P][2] : x[OFF + P][3];
    const double alpha = mf_readlane(xa, ((I & 3) << 4) | I);
    const bool nz = xn2 > 0.0;
    const double beta = nz ? -copysign(sqrt(fma(alpha, alpha, xn2)), alpha) : alpha;
    // the two reciprocals by Newton-refined hardware estimates (independent
    // of each other); unused (and possibly infinite) when nz is false
    const double tau = nz ? (beta - alpha) * rcp_nr(beta) : 0.0;
    const double scal = nz ? rcp_nr(alpha - beta) : 0.0;
    double *vi = vl + I * (16 * RM + 1) + q * (4 * RM);
    if (c == I) {
#pragma unroll
        for (int rt = P; rt < R; ++rt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * e + q;  // row within the tile
                vi[rt * 4 + e] = (rt > P || r > I) ? x[OFF + rt][e] * scal : (r == I ? 1.0 : 0.0);
            }
    }
    mf_wave_sync();
    // v is read from LDS twice (for the dot product, for the update) rather
    // than held: registers are the scarce resource here
    double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rt = P; rt < R; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) d4[e] = fma(vi[rt * 4 + e], x[OFF + rt][e], d4[e]);
    const double w = tau * mf_colsum((d4[0] + d4[1]) + (d4[2] + d4[3]));
#pragma unroll
    for (int rt = P; rt < R; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) x[OFF + rt][e] = fma(-w, vi[rt * 4 + e], x[OFF + rt][e]);
    if (c == 0 && q == 0) tau_lds[I] = tau;
    ss = mf_below<RM, R, P, OFF>(x, I + 1, q);
}

// Factor panel P (this wavefront's column tile: row tiles OFF + [0, R) of x):
// V into vl (rows from 16P),
// then T of Q = H_0 .. H_15 = I - V T V^T into tb: T_ii = tau_i,
// T[0:i, i] = -tau_i T[0:i, 0:i] (V^T V)[0:i, i].
template <int RM, int R, int P, int OFF = 0>
__device__ __forceinline__ void mf_factor(mf4 (&x)[RM], double *vl, double *tb, double *gb, double *tau_lds,
                                          int c, int q) {
    double ss = mf_below<RM, R, P, OFF>(x, 0, q);
#pragma unroll 1
    for (int i = 0; i < 16; ++i) mf_pivot<RM, R, P, OFF>(x, i, ss, vl, tau_lds, c, q);
    mf4 gram = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rt = P; rt < R; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // A(i, k) = V(k, i) and B(k, j) = V(k, j): for i = j = c the same value
            const double v = vl[c * (16 * RM + 1) + q * (4 * RM) + rt * 4 + e];
            gram = mf_mma(v, v, gram);
        }
#pragma unroll
    for (int e = 0; e < 4; ++e) gb[(q + 4 * e) * 16 + c] = gram[e];
    mf_wave_sync();
    double tr[16];  // row c of T
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) s = fma(tr[k], gb[k * 16 + i], s);
        const double ti = tau_lds[i];
        tr[i] = c < i ? -ti * s : (c == i ? ti : 0.0);
    }
    if (q == 0) {
#pragma unroll
        for (int i = 0; i < 16; ++i) tb[c * 16 + i] = tr[i];
    }
}

// C -= V (T^T (V^T C)) on one column tile (row tiles OFF + [P, R) of x)
template <int RM, int R, int P, int OFF = 0>
__device__ __forceinline__ void mf_apply(mf4 (&x)[RM], const double *vl, const double *tb, int c, int q) {
    mf4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rt = P; rt < R; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            y = mf_mma(vl[c * (16 * RM + 1) + q * (4 * RM) + rt * 4 + e], x[OFF + rt][e], y);  // A = V^T
    mf4 w = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 4; ++e) w = mf_mma(tb[(4 * e + q) * 16 + c], y[e], w);  // A = T^T
#pragma unroll
    for (int rt = P; rt < R; ++rt) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            x[OFF + rt] = mf_mma(-vl[mf_vidx<RM>(4 * e + q, 16 * rt + c)], w[e], x[OFF + rt]);  // A = -V
    }
}

// Blocked Householder QR of a stack of R row tiles and C column tiles, pivots
// in column tiles [0, NB); this wavefront holds column tiles w + 4k.
template <int N, int MM, bool RAW, int R, int C>
__device__ __forceinline__ void mf_qr(MfTiles<N, MM, RAW> &X,
                                      MfLds<N, MM, RAW> &s, int w, int c, int q) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int RM = G::RM, NB = G::NB, KC = (C + 3) / 4;
    if (w == 0) mf_factor<RM, R, 0>(X[0], s.v[0], s.t[0], s.g, s.tau, c, q);
    mf_for<0, NB>([&](auto PC) {
        constexpr int P = decltype(PC)::value;
        __syncthreads();
        mf_for<0, KC>([&](auto KCc) {
            constexpr int K = decltype(KCc)::value;
            const int ct = w + 4 * K;
            if (ct < C && ct > P) {
                mf_apply<RM, R, P>(X[K], s.v[P & 1], s.t[P & 1], c, q);
                if constexpr (P + 1 < NB && K == (P + 1) / 4) {
                    if (ct == P + 1)
                        mf_factor<RM, R, P + 1>(X[K], s.v[(P + 1) & 1], s.t[(P + 1) & 1], s.g, s.tau, c, q);
                }
            }
        });
    });
    __syncthreads();
}

// Steps 2 and 3 at once (CONC).  Step 3's column tiles lie in slot KM - 1 of
// wavefronts 2 and 3, three row tiles each: wavefront 2 holds its column
// tiles 0 (row tiles 0-2 of the slot) and 3, the right-hand side (3-5);
// wavefront 3 its tiles 1 (0-2) and 2 (3-5).  The panels of both QRs advance
// together, one barrier per round: round P applies panel P of each and
// factors panel P + 1 of step 2 on wavefront P + 1 and of step 3 on
// wavefront 3, so no wavefront factors two panels in one round.
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_qr23(MfTiles<N, MM, RAW> &X, MfLds<N, MM, RAW> &s, int w, int c, int q) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int RM = G::RM, NB = G::NB, R2 = G::R2, R3 = G::R3, C2 = G::C2, KC = (C2 + 3) / 4, KS = G::KM - 1;
    const int ca = w == 2 ? 0 : 1, cb = w == 2 ? NB : 2;  // step-3 column tiles of the two halves
    if (w == 0) mf_factor<RM, R2, 0>(X[0], s.v[0], s.t[0], s.g, s.tau, c, q);
    if (w == 2) mf_factor<RM, R3, 0, 0>(X[KS], s.v3[0], s.t3[0], s.g3, s.tau3, c, q);
    mf_for<0, NB>([&](auto PC) {
        constexpr int P = decltype(PC)::value;
        __syncthreads();
        mf_for<0, KC>([&](auto KCc) {
            constexpr int K = decltype(KCc)::value;
            const int ct = w + 4 * K;
            if (ct < C2 && ct > P) {
                mf_apply<RM, R2, P>(X[K], s.v[P & 1], s.t[P & 1], c, q);
                if constexpr (P + 1 < NB && K == (P + 1) / 4) {
                    if (ct == P + 1)
                        mf_factor<RM, R2, P + 1>(X[K], s.v[(P + 1) & 1], s.t[(P + 1) & 1], s.g, s.tau, c, q);
                }
            }
        });
        if (w >= 2) {
            if (ca > P) {
                mf_apply<RM, R3, P, 0>(X[KS], s.v3[P & 1], s.t3[P & 1], c, q);
                if constexpr (P + 1 < NB) {
                    if (ca == P + 1)
                        mf_factor<RM, R3, P + 1, 0>(X[KS], s.v3[(P + 1) & 1], s.t3[(P + 1) & 1], s.g3, s.tau3, c, q);
                }
            }
            if (cb > P) {
                mf_apply<RM, R3, P, R3>(X[KS], s.v3[P & 1], s.t3[P & 1], c, q);
                if constexpr (P + 1 < NB) {
                    if (cb == P + 1)
                        mf_factor<RM, R3, P + 1, R3>(X[KS], s.v3[(P + 1) & 1], s.t3[(P + 1) & 1], s.g3, s.tau3, c,
                                                      q);
                }
            }
        }
    });
    __syncthreads();
}

// ----------------------------------------------------------------- loads

// rows of one observation block [O | w] (raw: G_q | o_q with diagonal
// variances var; reduced: the record's [O | w]) and one evolution block
// [E- | E+ | eta] (raw: [-F_q | H_q | c_q] with variances var; reduced: the
// record's)
struct MfObs {
    const double *O, *w, *var;  // var: diagonal covariance (raw) or null
    int ldo, sw, rows;          // row stride of O, of w; rows present
    bool dense;                 // raw with a dense covariance (not handled here)
};
struct MfEvol {
    const double *Em, *Ep, *eta, *var;
    int lde, se;
    bool neg, ident, dense;  // raw: E- = -F; H absent (identity); dense covariance
};

template <int N, bool RAW>
__device__ __forceinline__ MfObs mf_obs(const FwdArgs &a, int64_t q) {
    MfObs b{};
    if constexpr (RAW) {
        const int m = a.m;
        b.O = a.G + q * (int64_t)m * N;
        b.w = a.o + q * (int64_t)m;
        b.ldo = N;
        b.sw = 1;
        b.rows = m;
        if (a.C_diag) b.var = a.C + q * (int64_t)m;
        else b.dense = true;
    } else {
        const double *rec = a.sys_in + q * (int64_t)(N * (N + 1) + N * (2 * N + 1));
        b.O = rec;
        b.w = rec + N;
        b.ldo = b.sw = N + 1;
        b.rows = N;
    }
    return b;
}

template <int N, bool RAW>
__device__ __forceinline__ MfEvol mf_evol(const FwdArgs &a, int64_t q) {
    MfEvol b{};
    if constexpr (RAW) {
        const int64_t e = q - 1;  // ABI entry of step q
        b.Em = a.F + e * N * N;
        b.Ep = a.H ? a.H + e * N * N : nullptr;
        b.ident = a.H == nullptr;
        b.eta = a.c + e * N;
        b.lde = N;
        b.se = 1;
        b.neg = true;
        if (a.K_diag) b.var = a.K + e * N;
        else b.dense = true;
    } else {
        const double *ev = a.sys_in + q * (int64_t)(N * (N + 1) + N * (2 * N + 1)) + N * (N + 1);
        b.Em = ev;
        b.Ep = ev + N;
        b.eta = ev + 2 * N;
        b.lde = b.se = 2 * N + 1;
    }
    return b;
}

// Rows [r0, r0 + nr) of one tile column from p (the element of row r0 in
// this lane's column; row stride ld), for lanes with ok, row tiles [T0, T1);
// other rows and lanes keep their value.  Branch-free: every load reads a
// valid address (row r0 where the row is not taken), so all of them can be in
// flight at once.
template <int RM, int T0, int T1>
__device__ __forceinline__ void mf_ld(mf4 (&x)[RM], int q, const double *p, int ld, int r0, int nr, bool ok,
                                      bool neg) {
#pragma unroll
    for (int rt = T0; rt < T1; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 16 * rt + 4 * e + q;
            const bool take = ok && row >= r0 && row < r0 + nr;
            const double v = p[(int64_t)(take ? row - r0 : 0) * ld];
            x[rt][e] = take ? (neg ? -v : v) : x[rt][e];
        }
}

// rows [r0, r0 + n) of an identity block: 1 where row - r0 == col
template <int RM, int T0, int T1>
__device__ __forceinline__ void mf_ld_ident(mf4 (&x)[RM], int q, int col, int r0, int nr) {
#pragma unroll
    for (int rt = T0; rt < T1; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 16 * rt + 4 * e + q;
            if (row >= r0 && row < r0 + nr) x[rt][e] = row - r0 == col ? 1.0 : 0.0;
        }
}

// scale rows [r0, r0 + nr) of the tiles [0, KC) by 1/sqrt(var[row - r0]) (a
// diagonal whitening); flags a variance that is not positive and finite
template <int RM, int KM, int KC, int T0, int T1>
__device__ __forceinline__ void mf_scale(mf4 (&X)[KM][RM], int q, const double *var, int r0, int nr, bool &bad) {
    if (!var) return;
#pragma unroll
    for (int rt = T0; rt < T1; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 16 * rt + 4 * e + q;
            const bool take = row >= r0 && row < r0 + nr;
            const double v = var[take ? row - r0 : 0];
            if (take && !(v > 0.0 && isfinite(v))) bad = true;
            const double f = take ? rsq_nr(v) : 1.0;
#pragma unroll
            for (int k = 0; k < KC; ++k) X[k][rt][e] *= f;
        }
}

// Column tiles of the three stacks.  u_j: [0, NB); u_{j+1}: [NB, 2NB) (steps
// 1, 2) or [0, NB) (step 3); rhs: 2NB (steps 1, 2) or NB (step 3); u_{j-1}:
// [2NB + 1, 3NB + 1) (step 2).

// Step-1 stack: rows [0, RO) [O_j | 0 | w_j], rows [RO, RO + n) [E-_{j+1} |
// E+_{j+1} | eta_{j+1}].
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_load_step1(MfTiles<N, MM, RAW> &X, const FwdArgs &a, int64_t j, int w,
                                              int c, int q, bool &bad) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int NB = G::NB, RO = G::RO, RM = G::RM, KC = (G::C1 + 3) / 4;
    constexpr int TO = (RO + 15) / 16, TE0 = RO / 16, TE1 = G::R1;  // row tiles of the two blocks
    const MfObs ob = mf_obs<N, RAW>(a, j);
    const MfEvol ev = mf_evol<N, RAW>(a, j + 1);
    mf_for<0, KC>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const int ct = w + 4 * K;
        if (ct < NB) {
            mf_ld<RM, 0, TO>(X[K], q, ob.O + 16 * ct + c, ob.ldo, 0, ob.rows, true, false);
            mf_ld<RM, TE0, TE1>(X[K], q, ev.Em + 16 * ct + c, ev.lde, RO, N, true, ev.neg);
        } else if (ct < 2 * NB) {
            if (ev.ident) mf_ld_ident<RM, TE0, TE1>(X[K], q, 16 * (ct - NB) + c, RO, N);
            else mf_ld<RM, TE0, TE1>(X[K], q, ev.Ep + 16 * (ct - NB) + c, ev.lde, RO, N, true, false);
        } else if (ct == 2 * NB) {
            mf_ld<RM, 0, TO>(X[K], q, ob.w, ob.sw, 0, ob.rows, c == 0, false);
            mf_ld<RM, TE0, TE1>(X[K], q, ev.eta, ev.se, RO, N, c == 0, false);
        }
    });
    if constexpr (RAW) {
        mf_scale<RM, G::KM, KC, 0, TO>(X, q, ob.var, 0, ob.rows, bad);
        mf_scale<RM, G::KM, KC, TE0, TE1>(X, q, ev.var, RO, N, bad);
        if (ob.dense || ev.dense) bad = true;
    }
}

// Step 1 -> step 2.  [D~_{j+1} | gamma] (rows [n, n + RO) of the u_{j+1} and
// rhs tiles) to LDS; rows [0, n) of the u_j (upper triangle: R~_j), u_{j+1}
// (X_j) and rhs (rho~_j) tiles down to rows [n, 2n); rows [0, n) from the
// evolution rows of step j, [E+_j | 0 | eta_j | E-_j] (none for j = 0).
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_to_step2(MfTiles<N, MM, RAW> &X, MfLds<N, MM, RAW> &s, const FwdArgs &a,
                                            int64_t j, int w, int c, int q, bool &bad) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int NB = G::NB, RO = G::RO, RM = G::RM, KC = (G::C2 + 3) / 4;
    mf_for<0, KC>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const int ct = w + 4 * K;
        if (ct >= NB && ct <= 2 * NB) {
            const int col = ct < 2 * NB ? 16 * (ct - NB) + c : N;
            if (ct < 2 * NB || c == 0) {
#pragma unroll
                for (int rt = NB; rt < G::R1; ++rt)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = 16 * rt + 4 * e + q;
                        if (row < N + RO) s.d[(row - N) * G::DLD + col] = X[K][rt][e];
                    }
            }
        }
        if (ct <= 2 * NB) {
#pragma unroll
            for (int rt = NB - 1; rt >= 0; --rt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * rt + 4 * e + q, col = 16 * ct + c;
                    X[K][rt + NB][e] = (ct < NB && row > col) ? 0.0 : X[K][rt][e];
                    X[K][rt][e] = 0.0;
                }
        }
    });
    if (j < 1) return;  // column 0 has no evolution step (uniform over the workgroup)
    const MfEvol ev = mf_evol<N, RAW>(a, j);
    mf_for<0, KC>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const int ct = w + 4 * K;
        if (ct < NB) {
            if (ev.ident) mf_ld_ident<RM, 0, NB>(X[K], q, 16 * ct + c, 0, N);
            else mf_ld<RM, 0, NB>(X[K], q, ev.Ep + 16 * ct + c, ev.lde, 0, N, true, false);
        } else if (ct == 2 * NB) {
            mf_ld<RM, 0, NB>(X[K], q, ev.eta, ev.se, 0, N, c == 0, false);
        } else if (ct > 2 * NB && ct < G::C2) {
            mf_ld<RM, 0, NB>(X[K], q, ev.Em + 16 * (ct - 2 * NB - 1) + c, ev.lde, 0, N, true, ev.neg);
        }
    });
    if constexpr (RAW) {
        mf_scale<RM, G::KM, KC, 0, NB>(X, q, ev.var, 0, N, bad);
        if (ev.dense) bad = true;
    }
}

// Step-3 stack: rows [0, RO) [D~_{j+1} | gamma] from LDS, rows [RO, 2 RO)
// [O_{j+1} | w_{j+1}].
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_load_step3(MfTiles<N, MM, RAW> &X, MfLds<N, MM, RAW> &s, const FwdArgs &a,
                                              int64_t j, int w, int c, int q, bool &bad) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int NB = G::NB, RO = G::RO, RM = G::RM, KC = (G::C3 + 3) / 4;
    constexpr int TD = (RO + 15) / 16, TO0 = RO / 16, TO1 = G::R3;
    const MfObs ob = mf_obs<N, RAW>(a, j + 1);
#pragma unroll
    for (int k = 0; k < G::KM; ++k)
#pragma unroll
        for (int rt = 0; rt < RM; ++rt) X[k][rt] = mf4{0.0, 0.0, 0.0, 0.0};
    mf_for<0, KC>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const int ct = w + 4 * K;
        if (ct <= NB) {
            const int col = ct < NB ? 16 * ct + c : N;
            const bool ok = ct < NB || c == 0;
#pragma unroll
            for (int rt = 0; rt < TD; ++rt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * rt + 4 * e + q;
                    if (row < RO) X[K][rt][e] = ok ? s.d[row * G::DLD + col] : 0.0;
                }
            if (ct < NB) mf_ld<RM, TO0, TO1>(X[K], q, ob.O + 16 * ct + c, ob.ldo, RO, ob.rows, true, false);
            else mf_ld<RM, TO0, TO1>(X[K], q, ob.w, ob.sw, RO, ob.rows, c == 0, false);
        }
    });
    if constexpr (RAW) {
        mf_scale<RM, G::KM, KC, TO0, TO1>(X, q, ob.var, RO, ob.rows, bad);
        if (ob.dense) bad = true;
    }
}

// Step-3 stack into the halves of slot KM - 1 (CONC, wavefronts 2 and 3):
// rows [0, RO) [D~_{j+1} | gamma] from LDS, rows [RO, 2 RO) [O_{j+1} | w_{j+1}].
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_load_step3_halves(MfTiles<N, MM, RAW> &X, MfLds<N, MM, RAW> &s,
                                                     const FwdArgs &a, int64_t j, int w, int c, int q, bool &bad) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int NB = G::NB, RO = G::RO, R3 = G::R3, KS = G::KM - 1;
    const MfObs ob = mf_obs<N, RAW>(a, j + 1);
    static_assert(RO % 4 == 0, "a row quad must not straddle the two blocks");
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int ct = h == 0 ? (w == 2 ? 0 : 1) : (w == 2 ? NB : 2);
        const bool ok = ct < NB || c == 0;
        const int dcol = ct < NB ? 16 * ct + c : N;
        const double *Op = ct < NB ? ob.O + 16 * ct + c : ob.w;
        const int ld = ct < NB ? ob.ldo : ob.sw;
#pragma unroll
        for (int rt = 0; rt < R3; ++rt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * rt + 4 * e + q;
                double x;
                if (16 * rt + 4 * e < RO) {  // the whole quad lies in [D~ | gamma]
                    x = s.d[row * G::DLD + dcol];
                } else {
                    const int r = row - RO;
                    const bool in_o = r < ob.rows;
                    x = Op[(int64_t)(in_o ? r : 0) * ld];
                    if constexpr (RAW) {
                        if (ob.var) {
                            const double v = ob.var[in_o ? r : 0];
                            if (in_o && !(v > 0.0 && isfinite(v))) bad = true;
                            x *= rsq_nr(v);
                        }
                    }
                    x = in_o ? x : 0.0;
                }
                X[KS][h * R3 + rt][e] = ok ? x : 0.0;
            }
    }
    if (ob.dense) bad = true;
}

// Step-3 triangle from the halves (CONC): [O' | w'] of reduced column t.
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_store_step3_halves(const MfTiles<N, MM, RAW> &X, double *ob, int w, int c,
                                                      int q) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int NB = G::NB, R3 = G::R3, KS = G::KM - 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int ct = h == 0 ? (w == 2 ? 0 : 1) : (w == 2 ? NB : 2);
        if (ct == NB && c != 0) continue;
        const int col = ct < NB ? 16 * ct + c : N;
#pragma unroll
        for (int rt = 0; rt < NB; ++rt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * rt + 4 * e + q;
                ob[row * (N + 1) + col] = (ct == NB || row <= col) ? X[KS][h * R3 + rt][e] : 0.0;
            }
    }
}

// ----------------------------------------------------------------- stores

// After step 2: rows [0, n) are the R row [R_jj | R_j,right | rho | R_j,left],
// rows [n, 2n) the reduced evolution block [Z | X~ | zeta] of column t.
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_store_step2(const MfTiles<N, MM, RAW> &X, double *rec, double *ev, int w,
                                               int c, int q, double &dmin, double &dmax, bool &nonfinite) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int NB = G::NB, W = 3 * N + 1, WE = 2 * N + 1, KC = (G::C2 + 3) / 4;
    mf_for<0, KC>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const int ct = w + 4 * K;
        if (ct < NB) {
            const int col = 16 * ct + c;
#pragma unroll
            for (int rt = 0; rt < NB; ++rt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * rt + 4 * e + q;
                    const double x = X[K][rt][e];
                    rec[row * W + col] = row <= col ? x : 0.0;
                    const double dv = fabs(x);
                    if (row == col && !isfinite(dv)) nonfinite = true;
                    dmin = row == col ? fmin(dmin, dv) : dmin;
                    dmax = row == col ? fmax(dmax, dv) : dmax;
                }
        } else if (ct < G::C2) {
            // R row column and reduced-evolution column of this lane
            const int rcol = ct < 2 * NB ? N + 16 * (ct - NB) + c : (ct == 2 * NB ? 2 * N : 2 * N + 1 + 16 * (ct - 2 * NB - 1) + c);
            const int ecol = ct < 2 * NB ? N + 16 * (ct - NB) + c : (ct == 2 * NB ? 2 * N : 16 * (ct - 2 * NB - 1) + c);
            if (ct != 2 * NB || c == 0) {
#pragma unroll
                for (int rt = 0; rt < 2 * NB; ++rt)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = 16 * rt + 4 * e + q;
                        if (rt < NB) rec[row * W + rcol] = X[K][rt][e];
                        else ev[(row - N) * WE + ecol] = X[K][rt][e];
                    }
            }
        }
    });
}

// After step 3: rows [0, n) of its triangle are the observation block [O' |
// w'] of reduced column t.
template <int N, int MM, bool RAW>
__device__ __forceinline__ void mf_store_step3(const MfTiles<N, MM, RAW> &X, double *ob, int w, int c, int q) {
    using G = MfGeo<N, MM, RAW>;
    constexpr int NB = G::NB, KC = (G::C3 + 3) / 4;
    mf_for<0, KC>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const int ct = w + 4 * K;
        if (ct < NB || (ct == NB && c == 0)) {
            const int col = ct < NB ? 16 * ct + c : N;
#pragma unroll
            for (int rt = 0; rt < NB; ++rt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * rt + 4 * e + q;
                    ob[row * (N + 1) + col] = (ct == NB || row <= col) ? X[K][rt][e] : 0.0;
                }
        }
    });
}

// ------------------------------------------------------------------ kernel

template <int N, int MM, bool RAW, bool BATCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mf_min_waves(N)))) void k_mf_forward(FwdArgs a0, const FwdArgs *tab, BlockMap bm) {
    using G = MfGeo<N, MM, RAW>;
    const FwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    const int64_t t = BATCH ? bm.blk[blockIdx.x] : (int64_t)blockIdx.x;
    __shared__ MfLds<N, MM, RAW> s;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, c = lane & 15, q = lane >> 4;
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    const int64_t j = 2 * t;
    mf4 X[G::KM][G::RM];
#pragma unroll
    for (int k = 0; k < G::KM; ++k)
#pragma unroll
        for (int rt = 0; rt < G::RM; ++rt) X[k][rt] = mf4{0.0, 0.0, 0.0, 0.0};

    mf_load_step1<N, MM, RAW>(X, a, j, w, c, q, bad);
    mf_qr<N, MM, RAW, G::R1, G::C1>(X, s, w, c, q);
    mf_to_step2<N, MM, RAW>(X, s, a, j, w, c, q, bad);
    if constexpr (G::CONC) {
        __syncthreads();  // [D~ | gamma] in LDS
        if (w >= 2) mf_load_step3_halves<N, MM, RAW>(X, s, a, j, w, c, q, bad);
        mf_qr23<N, MM, RAW>(X, s, w, c, q);
        mf_store_step2<N, MM, RAW>(X, a.rrows + t * (int64_t)G::RREC,
                                   a.sys_out + t * (int64_t)G::SREC + G::OREC, w, c, q, dmin, dmax, nonfinite);
        if (w >= 2) mf_store_step3_halves<N, MM, RAW>(X, a.sys_out + t * (int64_t)G::SREC, w, c, q);
    } else {
        mf_qr<N, MM, RAW, G::R2, G::C2>(X, s, w, c, q);
        mf_store_step2<N, MM, RAW>(X, a.rrows + t * (int64_t)G::RREC,
                                   a.sys_out + t * (int64_t)G::SREC + G::OREC, w, c, q, dmin, dmax, nonfinite);
        mf_load_step3<N, MM, RAW>(X, s, a, j, w, c, q, bad);
        mf_qr<N, MM, RAW, G::R3, G::C3>(X, s, w, c, q);
        mf_store_step3<N, MM, RAW>(X, a.sys_out + t * (int64_t)G::SREC, w, c, q);
    }

    block_minmax<256>(dmin, dmax, bad, nonfinite, a.flags);
    if (threadIdx.x == 0) {
        a.slots[2 * t] = dmin;
        a.slots[2 * t + 1] = dmax;
    }
}

template <int N, int MM, bool RAW>
static void launch_mf_fwd_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_mf_forward<N, MM, RAW, false>), dim3((unsigned)a.units), dim3(256), 0, s, a, nullptr,
                       BlockMap{});
}
template <int N, int MM, bool RAW>
static void launch_mf_fwd_bt(const FwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_mf_forward<N, MM, RAW, true>), dim3((unsigned)blocks), dim3(256), 0, s, FwdArgs{}, tab,
                       bm);
}

// Forward variant 1 of n = 32, 48: the MFMA forward wherever the stacks are
// FP64 (level 0 from the raw inputs, FP64 levels >= 1; single plans, batches
// and the engine) with at least 512 units, the workgroup family for narrower
// levels (FV_F64_NARROW) and the FP32-form levels; backward as in the
// default set.  Odd levels of the MFMA forward run the level kernel, then the
// fold kernel.
// Problems with dense covariances get variant 0 instead (raw_diag_only).
template <int N, int MM>
constexpr KernelSet make_mf_set() {
    KernelSet s = make_blk_set<N, MM, blk_rpw(N), 0>();
    s.fwd_raw[0] = &launch_mf_fwd_t<N, MM, true>;
    s.fwd[FV_F64] = &launch_mf_fwd_t<N, MM, false>;
    s.fwd_raw_b[0] = &launch_mf_fwd_bt<N, MM, true>;
    s.fwd_b[FV_F64] = &launch_mf_fwd_bt<N, MM, false>;
    s.fwd_fold[FV_F64] = nullptr;
    // levels too narrow to fill the device: the workgroup family, whose
    // units finish sooner (and fold in the level kernel)
    s.fwd[FV_F64_NARROW] = &launch_wg_fwd_t<N, MM, false, double, double>;
    s.fold[FV_F64_NARROW] = &launch_wg_fold_t<N, MM, false, double, double>;
    s.fwd_b[FV_F64_NARROW] = &launch_wg_fwd_bt<N, MM, false, double, double>;
    s.fold_b[FV_F64_NARROW] = &launch_wg_fold_bt<N, MM, false, double, double>;
    s.fwd_fold[FV_F64_NARROW] = &launch_wg_fwd_fold_t<N, MM, double, double>;
    s.narrow_units = 512;
    s.fv = 1;
    s.raw_diag_only = 1;
    return s;
}
#define KS_MF_SETS(N) make_mf_set<N, wg_mm_small(N)>(), make_mf_set<N, N>()

// Forward variant 2 of n = 32, 48: the 2-D tiled forward compiled for the
// other occupancy target (wg_alt_waves); backward as in the default set.
template <int N, int MM>
constexpr KernelSet make_occ_set() {
    constexpr int MW = wg_alt_waves(N);
    KernelSet s = make_blk_set<N, MM, blk_rpw(N), 0>();
    s.fwd_raw[0] = &launch_wg_fwd_t<N, MM, true, double, double, MW>;
    s.fwd_raw[1] = &launch_wg_fwd_t<N, MM, true, float, double, MW>;
    s.fwd[FV_F64] = &launch_wg_fwd_t<N, MM, false, double, double, MW>;
    s.fwd[FV_F32] = &launch_wg_fwd_t<N, MM, false, float, float, MW>;
    s.fwd[FV_F64_FROM_F32] = &launch_wg_fwd_t<N, MM, false, double, float, MW>;
    s.fwd_raw_b[0] = &launch_wg_fwd_bt<N, MM, true, double, double, MW>;
    s.fwd_raw_b[1] = &launch_wg_fwd_bt<N, MM, true, float, double, MW>;
    s.fwd_b[FV_F64] = &launch_wg_fwd_bt<N, MM, false, double, double, MW>;
    s.fwd_b[FV_F32] = &launch_wg_fwd_bt<N, MM, false, float, float, MW>;
    s.fwd_b[FV_F64_FROM_F32] = &launch_wg_fwd_bt<N, MM, false, double, float, MW>;
    s.fwd_fold[FV_F64] = &launch_wg_fwd_fold_t<N, MM, double, double, MW>;
    s.fwd_fold[FV_F32] = &launch_wg_fwd_fold_t<N, MM, float, float, MW>;
    s.fwd_fold[FV_F64_FROM_F32] = &launch_wg_fwd_fold_t<N, MM, double, float, MW>;
    s.fv = 2;
    return s;
}
#define KS_OCC_SETS(N) make_occ_set<N, wg_mm_small(N)>(), make_occ_set<N, N>()

}  // namespace ks
