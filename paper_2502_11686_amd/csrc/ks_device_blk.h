// ks_device_blk.h -- the workgroup family of the odd-even smoother kernels,
// for state dimensions whose units need more than one wavefront of lanes.
//
// Same algebra as the wavefront family (ks_device.h).  The forward levels
// (load, whitening, steps 1 to 3, the fold of odd levels, the base) are in
// ks_device_wg.h on a two-dimensional register tiling of each unit; this file
// holds the backward levels -- back-substitution and Algorithm 2 -- with one
// block row per workgroup, lane g owning column g of the R row, and the
// kernel table of the family.
#pragma once

#include "ks_device_wg.h"

namespace ks {

template <int N>
struct BGeo {
    static constexpr int W = 3 * N + 1;                    // columns of an R row
    static constexpr int TBB = (W + 63) / 64 * 64;         // backward workgroup
    static constexpr int RREC = N * (3 * N + 1);
    static constexpr int OREC = N * (N + 1);
    static constexpr int EREC = N * (2 * N + 1);
    static constexpr int SREC = OREC + EREC;
};


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
                     {&launch_wg_fwd_t<N, MM, true, double, double>, &launch_wg_fwd_t<N, MM, true, float, double>},
                     {&launch_wg_fwd_t<N, MM, false, double, double>, &launch_wg_fwd_t<N, MM, false, float, float>,
                      &launch_wg_fwd_t<N, MM, false, double, float>},
                     {&launch_wg_fold_t<N, MM, true, double, double>, &launch_wg_fold_t<N, MM, true, float, double>},
                     {&launch_wg_fold_t<N, MM, false, double, double>, &launch_wg_fold_t<N, MM, false, float, float>,
                      &launch_wg_fold_t<N, MM, false, double, float>},
                     &launch_wg_fwd_tail_t<N, MM, true>,
                     &launch_wg_fwd_tail_t<N, MM, false>,
                     {{&launch_blk_bwd_t<N, true, false, double>, &launch_blk_bwd_t<N, true, false, float>},
                      {&launch_blk_bwd_t<N, false, true, double>, &launch_blk_bwd_t<N, false, true, float>},
                      {&launch_blk_bwd_t<N, true, true, double>, &launch_blk_bwd_t<N, true, true, float>}},
                     {&launch_blk_bwd_tail_t<N, true, false>, &launch_blk_bwd_tail_t<N, false, true>,
                      &launch_blk_bwd_tail_t<N, true, true>},
                     {&launch_wg_fwd_bt<N, MM, true, double, double>, &launch_wg_fwd_bt<N, MM, true, float, double>},
                     {&launch_wg_fwd_bt<N, MM, false, double, double>, &launch_wg_fwd_bt<N, MM, false, float, float>,
                      &launch_wg_fwd_bt<N, MM, false, double, float>},
                     {&launch_wg_fold_bt<N, MM, true, double, double>, &launch_wg_fold_bt<N, MM, true, float, double>},
                     {&launch_wg_fold_bt<N, MM, false, double, double>, &launch_wg_fold_bt<N, MM, false, float, float>,
                      &launch_wg_fold_bt<N, MM, false, double, float>},
                     &launch_wg_fwd_tail_bt<N, MM, true>,
                     &launch_wg_fwd_tail_bt<N, MM, false>,
                     {{&launch_blk_bwd_bt<N, true, false, double>, &launch_blk_bwd_bt<N, true, false, float>},
                      {&launch_blk_bwd_bt<N, false, true, double>, &launch_blk_bwd_bt<N, false, true, float>},
                      {&launch_blk_bwd_bt<N, true, true, double>, &launch_blk_bwd_bt<N, true, true, float>}},
                     {&launch_blk_bwd_tail_bt<N, true, false>, &launch_blk_bwd_tail_bt<N, false, true>,
                      &launch_blk_bwd_tail_bt<N, true, true>},
                     1,
                     1,
                     {1, 1, 1},
                     {0, 0, 0}};
}

#define KS_BLK_SETS(N) make_blk_set<N, (N + 1) / 2>(), make_blk_set<N, N>()

}  // namespace ks