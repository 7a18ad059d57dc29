// ks_device_wg.h -- forward elimination of the workgroup family (state
// dimensions whose unit needs more than one wavefront) on a two-dimensional
// register tiling of each unit's stacks.
//
// One unit -- even column j = 2t of a level and its right neighbour, Section
// III's steps 1 to 3 -- per workgroup.  Stack columns are grouped: group
// c < n holds column c of the four blocks the unit touches,
//   slot 0 u_j        (pivot columns of steps 1 and 2)
//   slot 1 u_{j+1}    (group n: the right-hand side of steps 1 and 2)
//   slot 2 u_{j-1}    (step 2 only)
//   slot 3 u_{j+1}    (step 3's stack; group n: its right-hand side)
// and each group is spread over TR adjacent lanes (4 or 8), lane tr holding
// stack rows r = tr + TR i.  Stacks have 2n rows.  In a Householder step the
// pivot group forms the reflector (sums over its lanes by DPP permutations)
// and writes each lane's segment to LDS; after one workgroup barrier every
// lane reads the segment of its own rows once, forms the partial dot products
// of its slots, completes them over its group, and updates.  Steps 2 (pivots
// in slot 0) and 3 (pivots in slot 3) share one sweep.  Rows move between the
// three stacks without leaving their lane because n and the observation class
// are multiples of TR.
#pragma once

#include "ks_device.h"

namespace ks {

// lanes per stack column: 8 (more, lighter lanes per unit) where n and the
// observation classes are multiples of 8, else 4
constexpr int wg_tr(int n) { return n % 8 == 0 ? 8 : 4; }

// observation classes of the family (padded row counts of a level-0
// observation block): the smallest multiple of 8 >= n/2, and n
// Minimum wavefronts per SIMD the forward kernel is compiled for.  n = 32
// needs 130 VGPRs unconstrained (3 wavefronts per SIMD, two 5-wavefront
// workgroups per CU); at 128 (one spilled register) a fourth wavefront per
// SIMD fits and three workgroups share a CU.  n = 48 spills heavily under
// the same constraint and runs unconstrained.
constexpr int wg_min_waves(int n) { return n == 32 ? 4 : 1; }
// the other target, compiled as forward variant 2 of n = 32, 48 (the
// autotuner chooses): n = 32 unconstrained, n = 48 four wavefronts per SIMD
constexpr int wg_alt_waves(int n) { return n == 32 ? 1 : 4; }
constexpr int wg_mm_small(int n) { return ((n + 1) / 2 + 7) / 8 * 8; }

template <int N, class T>
struct WGeo {
    static constexpr int TR = wg_tr(N);               // lanes per stack column
    static constexpr int H = 2 * N;                   // stack rows
    static constexpr int RPT = H / TR;                // stack rows per lane
    static constexpr int HALF = N / TR;               // lane index of stack row n
    static constexpr int NT = (TR * (N + 1) + 63) / 64 * 64;
    static constexpr int RREC = N * (3 * N + 1);
    static constexpr int OREC = N * (N + 1);
    static constexpr int EREC = N * (2 * N + 1);
    static constexpr int SREC = OREC + EREC;
    // LDS stride of one lane's segment [v_0 .. v_{RPT-1} | coefficient]:
    // 16-byte aligned, and the four lanes of a quad on distinct banks
    static constexpr int vs() {
        const int step = sizeof(T) == 8 ? 2 : 4;
        int v = RPT + step;
        for (;;) {
            const int dw = v * (int)sizeof(T) / 4;
            unsigned used = 0;
            bool ok = true;
            for (int k = 0; k < TR; ++k) {
                const unsigned b = 1u << (((k * dw) % 32) / 4);
                ok = ok && !(used & b);
                used |= b;
            }
            if (ok) return v;
            v += step;
        }
    }
    static constexpr int VS = vs();
    static constexpr int VB = TR * VS;                // one published reflector
    static constexpr int CH = RPT % 4 == 0 ? 4 : 2;   // lane indices per skipped chunk
    static_assert(N % TR == 0 && RPT % CH == 0, "n must be a multiple of 8");
};

// value of v on lane perm(lane) of the same quad
template <int CTRL>
__device__ __forceinline__ double qperm(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float qperm(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// sum / max over the TR lanes of a group (4: a quad, 8: a half row); every
// step adds a lane's value and its partner's, so all lanes get the same bits
template <int TR, class T>
__device__ __forceinline__ T qsum(T v) {
    v = v + qperm<0xB1>(v);                   // lanes 1 0 3 2
    v = v + qperm<0x4E>(v);                   // lanes 2 3 0 1
    if (TR == 8) v = v + qperm<0x141>(v);     // lanes 7 6 .. 0 (half-row mirror)
    return v;
}
template <int TR, class T>
__device__ __forceinline__ T qmax(T v) {
    v = fmax(v, qperm<0xB1>(v));
    v = fmax(v, qperm<0x4E>(v));
    if (TR == 8) v = fmax(v, qperm<0x141>(v));
    return v;
}

// threads of a workgroup-family forward launch (one name, so it can stand in
// a macro argument)
template <int N>
struct WThreads {
    static constexpr int NT = WGeo<N, double>::NT;
};

// a unit's stack slots in one lane: X[slot][i] holds stack row tr + TR i
template <int N, class T>
using WStack = T[4][WGeo<N, T>::RPT];
template <int N, class T>
using WCol = T[WGeo<N, T>::RPT];

// lane tr of column group c
template <int N>
struct WLane {
    static constexpr int TR = wg_tr(N);
    int tr, c;
    __device__ WLane() : tr(threadIdx.x & (TR - 1)), c(threadIdx.x / TR) {}
};

// Reflector of pivot p from this lane's rows of its group's column x (rows
// [p, HR) take part): P = I - coef v v^T with v = (0.., alpha - beta,
// x_{p+1}, .., x_{HR-1}), beta = -sign(alpha) ||x_{p:HR}||, coef =
// 1 / (beta (beta - alpha)); the identity when the part below row p is zero.
// In FP32 the norm is formed on entries scaled by the column's largest.
template <int N, int HR, class T>
__device__ __forceinline__ void wg_reflector(const WCol<N, T> &x, int p, int tr, T &coef, T &v0) {
    using G = WGeo<N, T>;
    constexpr int RA = (HR + G::TR - 1) / G::TR;
    T a_own = 0, mx = 0;
#pragma unroll
    for (int i = 0; i < RA; ++i) {
        const int r = tr + G::TR * i;
        if (r == p) a_own = x[i];
        if (sizeof(T) == 4 && r >= p && r < HR) mx = fmax(mx, fabs(x[i]));
    }
    const T alpha = qsum<G::TR>(a_own);
    T am = T(1), sc = T(1);
    if (sizeof(T) == 4) {
        am = qmax<G::TR>(mx);
        sc = am > T(0) ? rcp_nr(am) : T(0);
    }
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int i = 0; i < RA; ++i) {
        const int r = tr + G::TR * i;
        const T m = (r > p && r < HR) ? x[i] * sc : T(0);
        if (i & 1) s0 = fma(m, m, s0);
        else s1 = fma(m, m, s1);
    }
    const T xn2 = qsum<G::TR>(s0 + s1);
    const T as = alpha * sc;
    const T s = fma(as, as, xn2);
    const T nrs = sqrt(s);
    const T beta = -copysign(nrs * am, alpha);
    coef = xn2 != T(0) ? sc * sc * rcp_nr(fma(fabs(as), nrs, s)) : T(0);
    v0 = alpha - beta;
}

// the lane's segment [v | coef] of the reflector of pivot p
template <int N, int HR, class T>
__device__ __forceinline__ void wg_store_reflector(const WCol<N, T> &x, int p, int tr, T coef, T v0, T *seg) {
    using G = WGeo<N, T>;
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
        const int r = tr + G::TR * i;
        seg[i] = (r < p || r >= HR) ? T(0) : (r == p ? v0 : x[i]);
    }
    seg[G::RPT] = coef;
}

// w = coef (v^T x) for the slots taking reflector A (mask MA) and, with HASB,
// for slot 3 taking B; v read from the published segments.  Lane indices
// whose rows all lie above p are skipped in chunks (a uniform test).
template <int N, int HR, int MA, bool HASB, class T>
__device__ __forceinline__ void wg_dots(const WStack<N, T> &X, int p, int tr, const T *vbA, const T *vbB,
                                        T (&w)[4]) {
    using G = WGeo<N, T>;
    constexpr int CH = G::CH;
    constexpr int RA = (HR + G::TR - 1) / G::TR;
    constexpr int NCH = (RA + CH - 1) / CH;
    const T *sa = vbA + tr * G::VS;
    const T *sb = vbB + tr * G::VS;
    T d[4][2] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};  // two chains per slot
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        if (G::TR * CH * (k + 1) > p) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int i = CH * k + u;
                if (i >= RA) continue;
                if (MA) {
                    const T v = sa[i];
#pragma unroll
                    for (int s = 0; s < 3; ++s)
                        if (MA & (1 << s)) d[s][u & 1] = fma(v, X[s][i], d[s][u & 1]);
                }
                if (HASB) d[3][u & 1] = fma(sb[i], X[3][i], d[3][u & 1]);
            }
        }
    }
    const T ca = MA ? sa[G::RPT] : T(0);
    const T cb = HASB ? sb[G::RPT] : T(0);
#pragma unroll
    for (int s = 0; s < 3; ++s) w[s] = (MA & (1 << s)) ? qsum<G::TR>(d[s][0] + d[s][1]) * ca : T(0);
    w[3] = HASB ? qsum<G::TR>(d[3][0] + d[3][1]) * cb : T(0);
}

// x -= w v for the slots in mask MA (reflector A) and, with HASB, slot 3 (B)
template <int N, int HR, int MA, bool HASB, class T>
__device__ __forceinline__ void wg_update(WStack<N, T> &X, int p, int tr, const T *vbA, const T *vbB,
                                          const T (&w)[4]) {
    using G = WGeo<N, T>;
    constexpr int CH = G::CH;
    constexpr int RA = (HR + G::TR - 1) / G::TR;
    constexpr int NCH = (RA + CH - 1) / CH;
    const T *sa = vbA + tr * G::VS;
    const T *sb = vbB + tr * G::VS;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        if (G::TR * CH * (k + 1) > p) {
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int i = CH * k + u;
                if (i >= RA) continue;
                if (MA) {
                    const T v = sa[i];
#pragma unroll
                    for (int s = 0; s < 3; ++s)
                        if (MA & (1 << s)) X[s][i] = fma(-w[s], v, X[s][i]);
                }
                if (HASB) X[3][i] = fma(-w[3], sb[i], X[3][i]);
            }
        }
    }
}

// Householder QR on rows [0, HR): pivots p < PA in slot 0 (applied to the
// slots in MA, which holds slot 0) and p < PB in slot 3 (applied to slot 3),
// one sweep; the strictly lower parts of the pivot columns end as zeros.
// vbuf holds two parities of two reflectors; step p writes parity ph and the
// next step the other, so no lane still reading one is overwritten.
template <int N, int HR, int PA, int MA, int PB, class T>
__device__ __forceinline__ void wg_qr(WStack<N, T> &X, const WLane<N> &L, T *vbuf, int &ph) {
    using G = WGeo<N, T>;
    static_assert(PA == 0 || PB == 0 || PA == PB, "a shared sweep has equal pivot counts");
    static_assert(PA == 0 || (MA & 1), "reflector A is applied to its pivot slot");
    constexpr int P = PA > PB ? PA : PB;
    constexpr int MA_ = PA > 0 ? MA : 0;
    constexpr bool HB = PB > 0;
#pragma unroll 1
    for (int p = 0; p < P; ++p) {
        T *vb = vbuf + (ph & 1) * 2 * G::VB;
        ++ph;
        if (L.c == p) {
            T ca = 0, va0 = 0, cb = 0, vb0 = 0;
            if (PA > 0) wg_reflector<N, HR, T>(X[0], p, L.tr, ca, va0);
            if (HB) wg_reflector<N, HR, T>(X[3], p, L.tr, cb, vb0);
            if (PA > 0) wg_store_reflector<N, HR, T>(X[0], p, L.tr, ca, va0, vb + L.tr * G::VS);
            if (HB) wg_store_reflector<N, HR, T>(X[3], p, L.tr, cb, vb0, vb + G::VB + L.tr * G::VS);
        }
        __syncthreads();
        T w[4];
        wg_dots<N, HR, MA_, HB, T>(X, p, L.tr, vb, vb + G::VB, w);
        wg_update<N, HR, MA_, HB, T>(X, p, L.tr, vb, vb + G::VB, w);
    }
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
        const int r = L.tr + G::TR * i;
        if (PA > 0 && L.c < PA && r > L.c) X[0][i] = T(0);
        if (PB > 0 && L.c < PB && r > L.c) X[3][i] = T(0);
    }
}

// Whitening of stack rows [R0, R0 + D) of the slots in MS by a diagonal
// covariance (variances var[0..dd), padding rows unit): row r scaled by
// 1/sqrt(var_r).
template <int N, int D, int R0, int MS, class T>
__device__ __forceinline__ void wg_whiten_diag(WStack<N, T> &X, const WLane<N> &L,
                                               const double *var, int dd, bool &bad) {
    using G = WGeo<N, T>;
    static_assert(R0 % G::TR == 0 && D % G::TR == 0, "whitening block not aligned to the row tiling");
#pragma unroll
    for (int ib = 0; ib < D / G::TR; ++ib) {
        const int r = L.tr + G::TR * ib;
        const T v = r < dd ? T(var[r]) : T(1);
        if (!(v > T(0) && isfinite(v))) bad = true;
        const T f = rsq_nr(v);
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (MS & (1 << s)) X[s][R0 / G::TR + ib] *= f;
    }
}

// Whitening by a dense covariance block (dd x dd, row-major at cov, padded to
// D with the identity): Cholesky K = L L^T column by column -- column c of K
// on group c, each column of L published through LDS -- fused with the
// forward substitution x <- L^{-1} x of rows [R0, R0 + D) of the slots in MS.
template <int N, int D, int R0, int MS, class T>
__device__ __forceinline__ void wg_whiten_dense(WStack<N, T> &X, const WLane<N> &L,
                                                const double *cov, int dd, T *vbuf, int &ph,
                                                bool &bad) {
    using G = WGeo<N, T>;
    constexpr int RD = D / G::TR;
    constexpr int I0 = R0 / G::TR;
    static_assert(R0 % G::TR == 0 && D % G::TR == 0, "whitening block not aligned to the row tiling");
    T kc[RD];
#pragma unroll
    for (int ib = 0; ib < RD; ++ib) {
        const int r = L.tr + G::TR * ib;
        kc[ib] = L.c >= D ? T(0) : (r < dd && L.c < dd) ? T(cov[r * dd + L.c]) : T(r == L.c ? 1 : 0);
    }
#pragma unroll 1
    for (int p = 0; p < D; ++p) {
        T *vb = vbuf + (ph & 1) * 2 * G::VB;
        ++ph;
        if (L.c == p) {
            T own = 0;
#pragma unroll
            for (int ib = 0; ib < RD; ++ib)
                if (L.tr + G::TR * ib == p) own = kc[ib];
            const T kpp = qsum<G::TR>(own);
            if (!(kpp > T(0) && isfinite(kpp))) bad = true;
            const T il = rsq_nr(kpp);
            T *seg = vb + L.tr * G::VS;
#pragma unroll
            for (int ib = 0; ib < RD; ++ib) seg[ib] = (L.tr + G::TR * ib > p) ? kc[ib] * il : T(0);
            seg[G::RPT] = il;
        }
        __syncthreads();
        const T *seg = vb + L.tr * G::VS;
        const T il = seg[G::RPT];
        T l[RD];
#pragma unroll
        for (int ib = 0; ib < RD; ++ib) l[ib] = seg[ib];
        // L(c, p): row c of the published column (zero for c <= p)
        const T lcp = L.c < D ? vb[(L.c & (G::TR - 1)) * G::VS + L.c / G::TR] : T(0);
#pragma unroll
        for (int ib = 0; ib < RD; ++ib) kc[ib] = fma(-l[ib], lcp, kc[ib]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (!(MS & (1 << s))) continue;
            T own = 0;
#pragma unroll
            for (int ib = 0; ib < RD; ++ib)
                if (L.tr + G::TR * ib == p) own = X[s][I0 + ib];
            const T xp = qsum<G::TR>(own) * il;
#pragma unroll
            for (int ib = 0; ib < RD; ++ib)
                X[s][I0 + ib] = (L.tr + G::TR * ib == p) ? xp : fma(-l[ib], xp, X[s][I0 + ib]);
        }
    }
}

template <int N, int D, int R0, int MS, class T>
__device__ __forceinline__ void wg_whiten(bool diag, WStack<N, T> &X, const WLane<N> &L,
                                          const double *cov, int dd, T *vbuf, int &ph, bool &bad) {
    if (diag) wg_whiten_diag<N, D, R0, MS, T>(X, L, cov, dd, bad);
    else wg_whiten_dense<N, D, R0, MS, T>(X, L, cov, dd, vbuf, ph, bad);
}

// ------------------------------------------------------------- stack loads

// observation rows of column/step q, rows [0, RO): [O | w] into slot S (group
// c < n) and slot SR (group n)
template <int N, int MM, bool RAW, int S, int SR, class T, class TIN>
__device__ __forceinline__ void wg_load_obs(WStack<N, T> &X, const WLane<N> &L, const FwdArgs &a,
                                            int64_t q) {
    using G = WGeo<N, T>;
    if constexpr (RAW) {
        const int m = a.m;
        const double *Gq = a.G + q * (int64_t)m * N;
        const double *oq = a.o + q * (int64_t)m;
#pragma unroll
        for (int ib = 0; ib < MM / G::TR; ++ib) {
            const int r = L.tr + G::TR * ib;
            if (r < m) {
                if (L.c < N) X[S][ib] = T(Gq[r * N + L.c]);
                else if (L.c == N) X[SR][ib] = T(oq[r]);
            }
        }
    } else {
        const TIN *rec = slot<TIN>(a.sys_in, q, G::SREC);
#pragma unroll
        for (int ib = 0; ib < G::HALF; ++ib) {
            const int r = L.tr + G::TR * ib;
            if (L.c < N) X[S][ib] = T(rec[r * (N + 1) + L.c]);
            else if (L.c == N) X[SR][ib] = T(rec[r * (N + 1) + N]);
        }
    }
}

// evolution rows of step q (raw: [-F_q | H_q | c_q]; reduced: [E- | E+ | eta])
// into rows [R0, R0 + n): E- into slot SM, E+ into slot SP, rhs into slot 1
// of group n
template <int N, bool RAW, int R0, int SM, int SP, class T, class TIN>
__device__ __forceinline__ void wg_load_evol(WStack<N, T> &X, const WLane<N> &L, const FwdArgs &a,
                                             int64_t q) {
    using G = WGeo<N, T>;
    constexpr int I0 = R0 / G::TR;
    if constexpr (RAW) {
        const int64_t e = q - 1;  // ABI entry of step q
        const double *F = a.F + e * N * N;
        const double *Hm = a.H ? a.H + e * N * N : nullptr;
        const double *cq = a.c + e * N;
#pragma unroll
        for (int ib = 0; ib < G::HALF; ++ib) {
            const int r = L.tr + G::TR * ib;
            if (L.c < N) {
                X[SM][I0 + ib] = T(-F[r * N + L.c]);
                X[SP][I0 + ib] = T(Hm ? Hm[r * N + L.c] : (r == L.c ? 1.0 : 0.0));
            } else if (L.c == N) {
                X[1][I0 + ib] = T(cq[r]);
            }
        }
    } else {
        const TIN *ev = slot<TIN>(a.sys_in, q, G::SREC) + G::OREC;
#pragma unroll
        for (int ib = 0; ib < G::HALF; ++ib) {
            const int r = L.tr + G::TR * ib;
            if (L.c < N) {
                X[SM][I0 + ib] = T(ev[r * (2 * N + 1) + L.c]);
                X[SP][I0 + ib] = T(ev[r * (2 * N + 1) + N + L.c]);
            } else if (L.c == N) {
                X[1][I0 + ib] = T(ev[r * (2 * N + 1) + 2 * N]);
            }
        }
    }
}

// R-row record [R_jj | R_j,right | rho | R_j,left] from rows [0, n)
template <int N, class T>
__device__ __forceinline__ void wg_store_rrow(T *rec, const WStack<N, T> &X, const WLane<N> &L) {
    using G = WGeo<N, T>;
    constexpr int W = 3 * N + 1;
#pragma unroll
    for (int i = 0; i < G::HALF; ++i) {
        const int r = L.tr + G::TR * i;
        if (L.c < N) {
            rec[r * W + L.c] = X[0][i];
            rec[r * W + N + L.c] = X[1][i];
            rec[r * W + 2 * N + 1 + L.c] = X[2][i];
        } else if (L.c == N) {
            rec[r * W + 2 * N] = X[1][i];
        }
    }
}

// |R_cc| of the pivot columns (slot 0, rows [0, n)) into the rank statistics
template <int N, class T>
__device__ __forceinline__ void wg_diag_stats(const WStack<N, T> &X, const WLane<N> &L,
                                              double &dmin, double &dmax, bool &nonfinite) {
    using G = WGeo<N, T>;
    if (L.c >= N || L.tr != (L.c & (G::TR - 1))) return;
    T dv = 0;
#pragma unroll
    for (int i = 0; i < G::HALF; ++i)
        if (i == L.c / G::TR) dv = X[0][i];
    const double d = fabs(double(dv));
    if (!isfinite(d)) nonfinite = true;
    dmin = fmin(dmin, d);
    dmax = fmax(dmax, d);
}

// --------------------------------------------------------- forward units

// The last column jl = N_l - 1 of a level with N_l odd: its R row (record
// t + 1) and its Z rows, which touch only column jl - 1, stacked under the
// step-3 triangle O' of the last unit (slot 3 rows [0, n)) and folded in by
// one more QR.  Slots 0-2 are reused.
template <int N, int MM, bool RAW, class T, class TIN>
__device__ __forceinline__ void wg_fold_part(const FwdArgs &a, int64_t t, WStack<N, T> &X,
                                             const WLane<N> &L, T *vbuf, int &ph, double &dmin, double &dmax,
                                             bool &bad, bool &nonfinite) {
    using G = WGeo<N, T>;
    constexpr int RO = RAW ? MM : N;
    constexpr int P1 = RO < N ? RO : N;
    const int64_t jl = a.Nl - 1;
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
        X[0][i] = X[1][i] = X[2][i] = T(0);
        if (i >= G::HALF) X[3][i] = T(0);
    }
    wg_load_obs<N, MM, RAW, 0, 1, T, TIN>(X, L, a, jl);
    if constexpr (RAW)
        wg_whiten<N, MM, 0, 0x3, T>(a.C_diag, X, L, a.C + jl * (int64_t)(a.C_diag ? a.m : a.m * a.m), a.m,
                                    vbuf, ph, bad);
    wg_qr<N, RO, P1, 0x3, 0, T>(X, L, vbuf, ph);
#pragma unroll
    for (int i = 0; i < G::HALF; ++i) {
        X[0][G::HALF + i] = X[0][i];
        X[1][G::HALF + i] = X[1][i];
        X[0][i] = X[1][i] = T(0);
    }
    wg_load_evol<N, RAW, 0, 2, 0, T, TIN>(X, L, a, jl);
    if constexpr (RAW)
        wg_whiten<N, N, 0, 0x7, T>(a.K_diag, X, L, a.K + (jl - 1) * (int64_t)(a.K_diag ? N : N * N), N, vbuf,
                                   ph, bad);
    wg_qr<N, 2 * N, N, 0x7, 0, T>(X, L, vbuf, ph);
    wg_store_rrow<N, T>(slot<T>(a.rrows, t + 1, G::RREC), X, L);
    wg_diag_stats<N, T>(X, L, dmin, dmax, nonfinite);
    // Z (slot 2) and zeta (slot 1 of group n), rows [n, 2n), under O'
#pragma unroll
    for (int i = G::HALF; i < G::RPT; ++i) X[3][i] = L.c < N ? X[2][i] : X[1][i];
    wg_qr<N, 2 * N, 0, 0, N, T>(X, L, vbuf, ph);
}

// The fold split across two workgroups of the level launch: the last
// column's R row and Z rows (they depend on no unit of the level) ...
template <int N, int MM, bool RAW, class T, class TIN>
__device__ __forceinline__ void wg_fold_pre(const FwdArgs &a, int64_t t, T *vbuf, double &dmin, double &dmax,
                                            bool &bad, bool &nonfinite) {
    using G = WGeo<N, T>;
    constexpr int RO = RAW ? MM : N;
    constexpr int P1 = RO < N ? RO : N;
    const WLane<N> L;
    int ph = 0;
    const int64_t jl = a.Nl - 1;
    T X[4][G::RPT];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < G::RPT; ++i) X[s][i] = T(0);
    wg_load_obs<N, MM, RAW, 0, 1, T, TIN>(X, L, a, jl);
    if constexpr (RAW)
        wg_whiten<N, MM, 0, 0x3, T>(a.C_diag, X, L, a.C + jl * (int64_t)(a.C_diag ? a.m : a.m * a.m), a.m,
                                    vbuf, ph, bad);
    wg_qr<N, RO, P1, 0x3, 0, T>(X, L, vbuf, ph);
#pragma unroll
    for (int i = 0; i < G::HALF; ++i) {
        X[0][G::HALF + i] = X[0][i];
        X[1][G::HALF + i] = X[1][i];
        X[0][i] = X[1][i] = T(0);
    }
    wg_load_evol<N, RAW, 0, 2, 0, T, TIN>(X, L, a, jl);
    if constexpr (RAW)
        wg_whiten<N, N, 0, 0x7, T>(a.K_diag, X, L, a.K + (jl - 1) * (int64_t)(a.K_diag ? N : N * N), N, vbuf,
                                   ph, bad);
    wg_qr<N, 2 * N, N, 0x7, 0, T>(X, L, vbuf, ph);
    wg_store_rrow<N, T>(slot<T>(a.rrows, t + 1, G::RREC), X, L);
    wg_diag_stats<N, T>(X, L, dmin, dmax, nonfinite);
    // Z (slot 2) and zeta (slot 1 of group n), rows [n, 2n): row r at r (n + 1)
    T *z = reinterpret_cast<T *>(a.fold_z);
#pragma unroll
    for (int i = G::HALF; i < G::RPT; ++i) {
        const int r = L.tr + G::TR * (i - G::HALF);
        if (L.c <= N) z[r * (N + 1) + L.c] = L.c < N ? X[2][i] : X[1][i];
    }
}

// ... and the merge: each of the two workgroups, done with its part, counts
// its arrival; the second stacks Z under the last unit's step-3 triangle O'
// (as stored) and folds it in by one more QR, then resets the counter.  No
// workgroup waits for the other.
template <int N, class T>
__device__ __forceinline__ void wg_fold_join(const FwdArgs &a, int64_t t, T *vbuf) {
    using G = WGeo<N, T>;
    __shared__ unsigned arrival;
    __threadfence();  // this workgroup's records are visible device-wide before it counts
    __syncthreads();
    if (threadIdx.x == 0) arrival = atomicAdd(a.fold_cnt, 1u);
    __syncthreads();
    if (arrival != 1u) return;
    __threadfence();  // the other workgroup's records are seen
    const WLane<N> L;
    int ph = 0;
    T X[4][G::RPT];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int i = 0; i < G::RPT; ++i) X[s][i] = T(0);
    T *ob = slot<T>(a.sys_out, t, G::SREC);
    const T *z = reinterpret_cast<const T *>(a.fold_z);
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
        const int r = L.tr + G::TR * (i < G::HALF ? i : i - G::HALF);
        X[3][i] = L.c <= N ? (i < G::HALF ? ob[r * (N + 1) + L.c] : z[r * (N + 1) + L.c]) : T(0);
    }
    wg_qr<N, 2 * N, 0, 0, N, T>(X, L, vbuf, ph);
#pragma unroll
    for (int i = 0; i < G::HALF; ++i) {
        const int r = L.tr + G::TR * i;
        if (L.c <= N) ob[r * (N + 1) + L.c] = X[3][i];
    }
    if (threadIdx.x == 0) *a.fold_cnt = 0u;
}

// INLINE_FOLD: the last unit of an odd level also folds the last column in
// (the tail kernel, one workgroup per level)
template <int N, int MM, bool RAW, bool INLINE_FOLD, class T, class TIN>
__device__ __forceinline__ void wg_fwd_unit(const FwdArgs &a, int64_t t, T *vbuf, double &dmin, double &dmax,
                                            bool &bad, bool &nonfinite) {
    using G = WGeo<N, T>;
    constexpr int RO = RAW ? MM : N;
    constexpr int HA = RO + N;
    constexpr int PB = 2 * RO < N ? 2 * RO : N;
    static_assert(RO <= N && RO % G::TR == 0, "observation class not in this family");
    const WLane<N> L;
    int ph = 0;
    const int64_t j = 2 * t;
    const bool fold = (a.Nl & 1) && t == a.units - 1;  // uniform over the workgroup

    T X[4][G::RPT];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < G::RPT; ++i) X[s][i] = T(0);

    // step-1 stack [O_j ; E_{j+1}] in slots 0/1, step-3 observation rows O_{j+1} in slot 3
    wg_load_obs<N, MM, RAW, 0, 1, T, TIN>(X, L, a, j);
    wg_load_obs<N, MM, RAW, 3, 3, T, TIN>(X, L, a, j + 1);
    wg_load_evol<N, RAW, RO, 0, 1, T, TIN>(X, L, a, j + 1);
    if constexpr (RAW) {
        const int64_t cs = a.C_diag ? a.m : (int64_t)a.m * a.m;
        wg_whiten<N, MM, 0, 0x3, T>(a.C_diag, X, L, a.C + j * cs, a.m, vbuf, ph, bad);
        wg_whiten<N, MM, 0, 0x8, T>(a.C_diag, X, L, a.C + (j + 1) * cs, a.m, vbuf, ph, bad);
        wg_whiten<N, N, RO, 0x3, T>(a.K_diag, X, L, a.K + j * (int64_t)(a.K_diag ? N : N * N), N, vbuf, ph,
                                    bad);
    }

    // step 1: pivots u_j over rows [0, RO + n)
    wg_qr<N, HA, N, 0x3, 0, T>(X, L, vbuf, ph);

    // [D~_{j+1} | gamma] (rows [n, n + RO) of slot 1) under O_{j+1}; [R~_j X_j rho~_j] down to rows [n, 2n)
#pragma unroll
    for (int i = G::HALF; i < G::RPT; ++i) X[3][i] = X[1][i];
#pragma unroll
    for (int i = 0; i < G::HALF; ++i) {
        X[0][G::HALF + i] = X[0][i];
        X[1][G::HALF + i] = X[1][i];
        X[0][i] = X[1][i] = T(0);
    }
    // evolution rows of step j on top: [E-_j (u_{j-1}) | E+_j (u_j) | eta_j]
    if (j >= 1) {
        wg_load_evol<N, RAW, 0, 2, 0, T, TIN>(X, L, a, j);
        if constexpr (RAW)
            wg_whiten<N, N, 0, 0x7, T>(a.K_diag, X, L, a.K + (j - 1) * (int64_t)(a.K_diag ? N : N * N), N,
                                       vbuf, ph, bad);
    }

    // steps 2 (pivots u_j, slot 0) and 3 (pivots u_{j+1}, slot 3) in one sweep
    wg_qr<N, 2 * N, N, 0x7, N, T>(X, L, vbuf, ph);

    wg_store_rrow<N, T>(slot<T>(a.rrows, t, G::RREC), X, L);
    wg_diag_stats<N, T>(X, L, dmin, dmax, nonfinite);
    {
        T *ev = slot<T>(a.sys_out, t, G::SREC) + G::OREC;
#pragma unroll
        for (int i = G::HALF; i < G::RPT; ++i) {
            const int r = L.tr + G::TR * (i - G::HALF);
            if (L.c < N) {
                ev[r * (2 * N + 1) + L.c] = X[2][i];
                ev[r * (2 * N + 1) + N + L.c] = X[1][i];
            } else if (L.c == N) {
                ev[r * (2 * N + 1) + 2 * N] = X[1][i];
            }
        }
    }
    // O' = the step-3 triangle (rows >= 2 RO are empty when RO < n/2)
    if (PB < N) {
#pragma unroll
        for (int i = 0; i < G::HALF; ++i)
            if (L.tr + G::TR * i >= PB) X[3][i] = T(0);
    }
    if (INLINE_FOLD && fold) {
        __syncthreads();
        wg_fold_part<N, MM, RAW, T, TIN>(a, t, X, L, vbuf, ph, dmin, dmax, bad, nonfinite);
    }
    {
        T *ob = slot<T>(a.sys_out, t, G::SREC);
#pragma unroll
        for (int i = 0; i < G::HALF; ++i) {
            const int r = L.tr + G::TR * i;
            if (L.c <= N) ob[r * (N + 1) + L.c] = X[3][i];
        }
    }
}

// ------------------------------------------------------------------ kernels

// With FOLD (an odd level of a single plan; units + 1 workgroups), workgroup
// 0 forms the last column's R row and Z rows and writes the level's fold
// slot, workgroups 1 .. units run the units, the last unit first, and the
// later of workgroup 0 and the last unit's folds Z in (wg_fold_join).
// MW: the wavefronts per SIMD the kernel is compiled for (register budget).
template <int N, int MM, bool RAW, class T, class TIN, bool BATCH, bool FOLD = false, int MW = wg_min_waves(N)>
__global__ __launch_bounds__(WThreads<N>::NT) __attribute__((amdgpu_waves_per_eu(MW))) void k_wg_forward(
    FwdArgs a0, const FwdArgs *tab, BlockMap bm) {
    const FwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    if constexpr (FOLD && !BATCH) {
        __shared__ T vb[4 * WGeo<N, T>::VB];
        bool bad = false, nonfinite = false;
        double dmin = INFINITY, dmax = 0.0;
        const bool pre = blockIdx.x == 0;
        const int64_t blk = pre ? a.units - 1 : (int64_t)(gridDim.x - 1 - blockIdx.x);
        if (pre)
            wg_fold_pre<N, MM, RAW, T, TIN>(a, blk, vb, dmin, dmax, bad, nonfinite);
        else
            wg_fwd_unit<N, MM, RAW, false, T, TIN>(a, blk, vb, dmin, dmax, bad, nonfinite);
        block_minmax<WGeo<N, double>::NT>(dmin, dmax, bad, nonfinite, a.flags);
        if (threadIdx.x == 0) {
            double *dst = pre ? a.fold_slot : a.slots + 2 * blk;
            dst[0] = dmin;
            dst[1] = dmax;
        }
        if (blk == a.units - 1) wg_fold_join<N, T>(a, blk, vb);
    } else {
        static_assert(!FOLD, "the batched launches fold in a kernel of their own");
        const int64_t blk = BATCH ? bm.blk[blockIdx.x] : (int64_t)blockIdx.x;
        __shared__ T vbuf[4 * WGeo<N, T>::VB];
        bool bad = false, nonfinite = false;
        double dmin = INFINITY, dmax = 0.0;
        wg_fwd_unit<N, MM, RAW, false, T, TIN>(a, blk, vbuf, dmin, dmax, bad, nonfinite);
        block_minmax<WGeo<N, double>::NT>(dmin, dmax, bad, nonfinite, a.flags);
        if (threadIdx.x == 0) {
            a.slots[2 * blk] = dmin;
            a.slots[2 * blk + 1] = dmax;
        }
    }
}

// the fold of an odd level after its k_wg_forward (one workgroup)
template <int N, int MM, bool RAW, class T, class TIN, bool BATCH>
__global__ __launch_bounds__(WThreads<N>::NT) void k_wg_fold(FwdArgs a0, const FwdArgs *tab, BlockMap bm) {
    using G = WGeo<N, T>;
    const FwdArgs &a = BATCH ? tab[bm.item[blockIdx.x]] : a0;
    __shared__ T vbuf[4 * G::VB];
    const WLane<N> L;
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    int ph = 0;
    const int64_t t = a.units - 1;
    T X[4][G::RPT];
    T *ob = slot<T>(a.sys_out, t, G::SREC);
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
        const int r = L.tr + G::TR * i;
        X[3][i] = (i < G::HALF && L.c <= N) ? ob[r * (N + 1) + L.c] : T(0);
    }
    wg_fold_part<N, MM, RAW, T, TIN>(a, t, X, L, vbuf, ph, dmin, dmax, bad, nonfinite);
#pragma unroll
    for (int i = 0; i < G::HALF; ++i) {
        const int r = L.tr + G::TR * i;
        if (L.c <= N) ob[r * (N + 1) + L.c] = X[3][i];
    }
    block_minmax<WGeo<N, double>::NT>(dmin, dmax, bad, nonfinite, a.flags);
    if (threadIdx.x == 0) {
        a.fold_slot[0] = dmin;
        a.fold_slot[1] = dmax;
    }
}

// forward levels l0..L in one workgroup (in this family the base level, or a
// whole tiny problem), then the rank test over every launch's statistics
template <int N, int MM, bool RAW0, bool BATCH>
__global__ __launch_bounds__(WThreads<N>::NT) void k_wg_fwd_tail(FwdTailArgs ta0, const FwdTailArgs *tab,
                                                                     BlockMap bm) {
    using G = WGeo<N, double>;
    const FwdTailArgs &ta = BATCH ? tab[bm.item[blockIdx.x]] : ta0;
    __shared__ double vbuf[4 * G::VB];
    const WLane<N> L;
    bool bad = false, nonfinite = false;
    double dmin = INFINITY, dmax = 0.0;
    for (int l = ta.l0; l <= ta.L; ++l) {
        FwdArgs a = ta.a;
        a.Nl = ta.Nl[l];
        a.units = a.Nl == 1 ? 1 : a.Nl / 2;
        a.level = l;
        a.sys_in = l >= 1 ? ta.sys + ta.sys_off[l] : nullptr;
        a.sys_out = l < ta.L ? ta.sys + ta.sys_off[l + 1] : nullptr;
        a.rrows = ta.rrows + ta.rec_off[l] * G::RREC;
        if (a.Nl == 1) {
            // base: QR of the last column's observation block
            double X[4][G::RPT];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < G::RPT; ++i) X[s][i] = 0.0;
            int ph = 0;
            if (RAW0 && l == 0) {
                wg_load_obs<N, MM, true, 0, 1, double, double>(X, L, a, 0);
                wg_whiten<N, MM, 0, 0x3, double>(a.C_diag, X, L, a.C, a.m, vbuf, ph, bad);
                wg_qr<N, MM, (MM < N ? MM : N), 0x3, 0, double>(X, L, vbuf, ph);
            } else {
                wg_load_obs<N, MM, false, 0, 1, double, double>(X, L, a, 0);
                wg_qr<N, N, N, 0x3, 0, double>(X, L, vbuf, ph);
            }
            wg_store_rrow<N, double>(a.rrows, X, L);
            wg_diag_stats<N, double>(X, L, dmin, dmax, nonfinite);
        } else {
            for (int64_t t = 0; t < a.units; ++t) {
                if (RAW0 && l == 0)
                    wg_fwd_unit<N, MM, true, true, double, double>(a, t, vbuf, dmin, dmax, bad, nonfinite);
                else
                    wg_fwd_unit<N, MM, false, true, double, double>(a, t, vbuf, dmin, dmax, bad, nonfinite);
                __syncthreads();
            }
        }
        __syncthreads();  // the next level reads what this workgroup wrote: workgroup scope suffices
    }
    reduce_slots(ta.slots, ta.nprev, dmin, dmax);
    block_minmax<G::NT>(dmin, dmax, bad, nonfinite, ta.a.flags);
    rank_flag(dmin, dmax, ta.rank_tol, ta.a.flags);
}

template <int N, int MM, bool RAW, class T, class TIN, int MW = wg_min_waves(N)>
static void launch_wg_fwd_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_wg_forward<N, MM, RAW, T, TIN, false, false, MW>), dim3((unsigned)a.units),
                       dim3(WGeo<N, double>::NT), 0, s, a, nullptr, BlockMap{});
}
template <int N, int MM, class T, class TIN, int MW = wg_min_waves(N)>
static void launch_wg_fwd_fold_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_wg_forward<N, MM, false, T, TIN, false, true, MW>), dim3((unsigned)a.units + 1u),
                       dim3(WGeo<N, double>::NT), 0, s, a, nullptr, BlockMap{});
}
template <int N, int MM, bool RAW, class T, class TIN, int MW = wg_min_waves(N)>
static void launch_wg_fwd_bt(const FwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_wg_forward<N, MM, RAW, T, TIN, true, false, MW>), dim3((unsigned)blocks),
                       dim3(WGeo<N, double>::NT), 0, s, FwdArgs{}, tab, bm);
}
template <int N, int MM, bool RAW, class T, class TIN>
static void launch_wg_fold_t(const FwdArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_wg_fold<N, MM, RAW, T, TIN, false>), dim3(1), dim3(WGeo<N, double>::NT), 0, s, a,
                       nullptr, BlockMap{});
}
template <int N, int MM, bool RAW, class T, class TIN>
static void launch_wg_fold_bt(const FwdArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_wg_fold<N, MM, RAW, T, TIN, true>), dim3((unsigned)blocks),
                       dim3(WGeo<N, double>::NT), 0, s, FwdArgs{}, tab, bm);
}
template <int N, int MM, bool RAW0>
static void launch_wg_fwd_tail_t(const FwdTailArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_wg_fwd_tail<N, MM, RAW0, false>), dim3(1), dim3(WGeo<N, double>::NT), 0, s, a,
                       nullptr, BlockMap{});
}
template <int N, int MM, bool RAW0>
static void launch_wg_fwd_tail_bt(const FwdTailArgs *tab, BlockMap bm, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_wg_fwd_tail<N, MM, RAW0, true>), dim3((unsigned)blocks), dim3(WGeo<N, double>::NT), 0,
                       s, FwdTailArgs{}, tab, bm);
}

}  // namespace ks
