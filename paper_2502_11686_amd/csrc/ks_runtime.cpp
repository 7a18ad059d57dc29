// ks_runtime.cpp -- host side of libks: argument checks, the level schedule,
// the workspace layout and the launch sequence behind the C ABI of ks.h.
//
// Level schedule (Section III): level l has N_l = floor((k+1) / 2^l) block
// columns; level-l column j is original column (j+1) 2^l - 1, so original
// column i is eliminated at level ctz(i+1) and there are L = floor(log2(k+1))
// elimination levels above the single-column base level L.  Every column is
// eliminated exactly once, so the R factor has k+1 block rows, stored level
// by level (ceil(N_l / 2) records at level l).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <new>

#include "ks.h"
#include "ks_internal.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int L;
    int64_t Nl[ks::kMaxLevels];
    int64_t rec_off[ks::kMaxLevels];
    int64_t sys_off[ks::kMaxLevels];   // doubles from the sys segment start (levels >= 1)
    int64_t slot_off[ks::kMaxLevels];  // slots (pairs) before level l
    int64_t nslots;
    int64_t spm_first;                 // first record with stored S blocks (level 1)
    int64_t spm_records;
    size_t off_rrows, off_sys, off_spm, off_slots, off_flags, total;
};

bool valid_desc(const ks_desc *d) {
    if (!d) return false;
    if (d->k < 0 || d->k > ((int64_t)1 << 40)) return false;
    if (d->n < 1 || d->m < 0) return false;
    if (d->precision != KS_FP64 && d->precision != KS_FP32_FORM) return false;
    if ((d->K_layout != KS_COV_DENSE && d->K_layout != KS_COV_DIAG) ||
        (d->C_layout != KS_COV_DENSE && d->C_layout != KS_COV_DIAG))
        return false;
    if (d->flags != 0) return false;
    return true;
}

bool make_layout(const ks_desc *d, const ks::KernelSet *ks_, Layout *lo) {
    const int64_t n = d->n;
    const int64_t rrec = n * (3 * n + 1);
    const int64_t srec = n * (3 * n + 2);
    std::memset(lo, 0, sizeof(*lo));
    int64_t N = d->k + 1;
    int l = 0;
    int64_t rec = 0, sys = 0, slots = 0;
    while (true) {
        if (l >= ks::kMaxLevels) return false;
        lo->Nl[l] = N;
        lo->rec_off[l] = rec;
        lo->slot_off[l] = slots;
        if (l >= 1) {
            lo->sys_off[l] = sys;
            sys += N * srec;
        }
        rec += (N + 1) / 2;
        const int64_t units = N == 1 ? 1 : N / 2;
        // per-block slots of the level kernel, plus one for the fold kernel of an odd level
        slots += N == 1 ? 1 : (units + ks_->upb_fwd - 1) / ks_->upb_fwd + (N & 1);
        if (N == 1) break;
        N /= 2;
        ++l;
    }
    lo->L = l;
    lo->nslots = slots;
    lo->spm_first = lo->L >= 1 ? lo->rec_off[1] : rec;
    lo->spm_records = rec - lo->spm_first;
    size_t off = 0;
    lo->off_rrows = off;
    off = align_up(off + sizeof(double) * (size_t)rec * rrec);
    lo->off_sys = off;
    off = align_up(off + sizeof(double) * (size_t)sys);
    lo->off_spm = off;
    off = align_up(off + sizeof(double) * (size_t)lo->spm_records * 2 * n * n);
    lo->off_slots = off;
    off = align_up(off + sizeof(double) * 2 * (size_t)slots);
    lo->off_flags = off;
    off = align_up(off + 64);
    lo->total = off;
    return true;
}

}  // namespace

struct ks_plan {
    ks_desc d;
    hipStream_t stream;
    char *ws;
    const ks::KernelSet *kset;
    Layout lo;
    bool smoothed;
    unsigned host_flags;   // status word copied back after each call
    int tail_passes;       // single-workgroup tail: levels needing <= this many passes
    int l_switch;          // FP32 form: levels below this one run in FP32 (0 = none)
    // instrumentation (ks_time_kernels)
    int time_kind;
    bool time_armed;       // events of the current call were recorded
    hipEvent_t ev[2];
    bool ev_made;
    double time_ms;
    int64_t time_count;
};

namespace {

ks_status hip_err(hipError_t e) { return e == hipSuccess ? KS_OK : KS_E_HIP; }

void mark(ks_plan *p, int kind, int which) {
    if (p->time_kind != kind || !p->ev_made) return;
    (void)hipEventRecord(p->ev[which], p->stream);
    if (which == 1) p->time_armed = true;
}

// add the elapsed time of the bracketed launches (after the stream sync)
void collect_time(ks_plan *p) {
    if (!p->time_armed) return;
    p->time_armed = false;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev[0], p->ev[1]) == hipSuccess) {
        p->time_ms += ms;
        p->time_count += 1;
    }
}

double *seg_d(ks_plan *p, size_t off) { return reinterpret_cast<double *>(p->ws + off); }

// first level whose units fit in `passes` passes of `per_pass` units
int tail_start(const Layout &lo, int per_pass, int passes, bool backward) {
    if (passes <= 0) return lo.L + 1;
    for (int l = 0; l <= lo.L; ++l) {
        const int64_t N = lo.Nl[l];
        const int64_t units = backward ? (N + 1) / 2 : (N == 1 ? 1 : N / 2);
        if (units <= (int64_t)per_pass * passes) return l;
    }
    return lo.L;
}

void enqueue_forward(ks_plan *p, const double *H, const double *F, const double *c,
                     const double *K, const double *G, const double *o, const double *C) {
    const Layout &lo = p->lo;
    const int64_t n = p->d.n;
    const int64_t rrec = n * (3 * n + 1);
    double *rrows = seg_d(p, lo.off_rrows);
    double *sys = seg_d(p, lo.off_sys);
    double *slots = seg_d(p, lo.off_slots);
    unsigned *flags = reinterpret_cast<unsigned *>(p->ws + lo.off_flags);
    ks::launch_clear_flags(flags, p->stream);
    mark(p, KS_TIME_FWD_ALL, 0);
    int l0 = tail_start(lo, p->kset->upb_fwd_tail, p->tail_passes, false);
    const int ls = p->l_switch;
    if (ls > 0 && l0 <= ls) l0 = ls + 1;  // the tail reads FP64 records only
    if (l0 > lo.L) l0 = lo.L;             // the base level always runs in the tail kernel
    ks::FwdArgs a{};
    a.k = p->d.k;
    a.m = p->d.m;
    a.K_diag = p->d.K_layout == KS_COV_DIAG;
    a.C_diag = p->d.C_layout == KS_COV_DIAG;
    a.H = H; a.F = F; a.c = c; a.K = K; a.G = G; a.o = o; a.C = C;
    a.flags = flags;
    for (int l = 0; l < l0; ++l) {
        a.Nl = lo.Nl[l];
        a.units = lo.Nl[l] / 2;
        a.level = l;
        a.sys_in = l >= 1 ? sys + lo.sys_off[l] : nullptr;
        a.sys_out = sys + lo.sys_off[l + 1];
        a.rrows = rrows + lo.rec_off[l] * rrec;
        a.slots = slots + 2 * lo.slot_off[l];
        const int64_t blocks = (a.units + p->kset->upb_fwd - 1) / p->kset->upb_fwd;
        a.fold_slot = a.slots + 2 * blocks;
        // precision of this level: FP32 below the switch, FP64 from it on
        const int v = l < ls ? ks::FV_F32 : (l == ls && l > 0 ? ks::FV_F64_FROM_F32 : ks::FV_F64);
        if (l == 0) mark(p, KS_TIME_FWD_LEVEL0, 0);
        if (l == 0) {
            p->kset->fwd_raw[v == ks::FV_F32](a, p->stream);
            if (lo.Nl[l] & 1) p->kset->fold_raw[v == ks::FV_F32](a, p->stream);
        } else {
            p->kset->fwd[v](a, p->stream);
            if (lo.Nl[l] & 1) p->kset->fold[v](a, p->stream);
        }
        if (l == 0) mark(p, KS_TIME_FWD_LEVEL0, 1);
    }
    ks::FwdTailArgs ta{};
    ta.a = a;
    ta.l0 = l0;
    ta.L = lo.L;
    ta.sys = sys;
    ta.rrows = rrows;
    ta.slots = slots;
    ta.nprev = lo.slot_off[l0];
    ta.rank_tol = 64.0 * (p->l_switch > 0 ? 1.1920928955078125e-07 : 2.220446049250313e-16);
    for (int l = 0; l <= lo.L; ++l) {
        ta.sys_off[l] = lo.sys_off[l];
        ta.rec_off[l] = lo.rec_off[l];
        ta.Nl[l] = lo.Nl[l];
    }
    if (l0 == 0) mark(p, KS_TIME_FWD_LEVEL0, 0);
    (l0 == 0 ? p->kset->fwd_tail_raw : p->kset->fwd_tail)(ta, p->stream);
    if (l0 == 0) mark(p, KS_TIME_FWD_LEVEL0, 1);
    mark(p, KS_TIME_FWD_ALL, 1);
}

void enqueue_backward(ks_plan *p, double *u_out, double *cov_out) {
    const Layout &lo = p->lo;
    const int mode = (u_out && cov_out) ? ks::BWD_BOTH : (u_out ? ks::BWD_Y : ks::BWD_COV);
    ks::BwdArgs b{};
    b.k = p->d.k;
    b.rrows_all = seg_d(p, lo.off_rrows);
    b.u_in = u_out;
    b.u_out = u_out;
    b.cov = cov_out;
    b.spm = seg_d(p, lo.off_spm);
    b.spm_first = lo.spm_first;
    b.store_s = cov_out != nullptr;
    for (int l = 0; l <= lo.L; ++l) {
        b.rec_off[l] = lo.rec_off[l];
        b.Nl[l] = lo.Nl[l];
    }
    int l1 = tail_start(lo, p->kset->upb_bwd_tail[mode], p->tail_passes, true);
    if (l1 < p->l_switch) l1 = p->l_switch;  // the tail reads FP64 records only
    mark(p, KS_TIME_BWD_ALL, 0);
    if (l1 <= lo.L) {
        b.level = lo.L;
        b.l_lo = l1;
        if (l1 == 0) mark(p, KS_TIME_BWD_LEVEL0, 0);
        p->kset->bwd_tail[mode](b, p->stream);
        if (l1 == 0) mark(p, KS_TIME_BWD_LEVEL0, 1);
    }
    for (int l = (l1 <= lo.L ? l1 : lo.L + 1) - 1; l >= 0; --l) {
        b.level = l;
        b.l_lo = l;
        if (l == 0) mark(p, KS_TIME_BWD_LEVEL0, 0);
        p->kset->bwd[mode][l < p->l_switch ? 1 : 0](b, p->stream);
        if (l == 0) mark(p, KS_TIME_BWD_LEVEL0, 1);
    }
    mark(p, KS_TIME_BWD_ALL, 1);
}

ks_status finish(ks_plan *p) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return KS_E_HIP;
    const unsigned *flags = reinterpret_cast<const unsigned *>(p->ws + p->lo.off_flags);
    e = hipMemcpyAsync(&p->host_flags, flags, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream);
    if (e != hipSuccess) return KS_E_HIP;
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return KS_E_HIP;
    collect_time(p);
    const unsigned f = p->host_flags;
    if (f & ks::FLAG_NOT_SPD) return KS_E_NOT_SPD;
    if (f & ks::FLAG_NONFINITE) return KS_E_NONFINITE;
    if (f & ks::FLAG_RANK) return KS_E_RANK;
    return KS_OK;
}

bool inputs_ok(const ks_plan *p, const double *F, const double *c, const double *K,
               const double *G, const double *o, const double *C) {
    if (p->d.k > 0 && (!F || !c || !K)) return false;
    if (p->d.m > 0 && (!G || !o || !C)) return false;
    return true;
}

}  // namespace

extern "C" {

size_t ks_workspace_bytes(const ks_desc *desc) {
    if (!valid_desc(desc)) return 0;
    const ks::KernelSet *kset = ks::find_kernels(desc->n, desc->m);
    if (!kset) return 0;
    Layout lo;
    if (!make_layout(desc, kset, &lo)) return 0;
    return lo.total;
}

int ks_supported(int32_t n, int32_t m) { return ks::find_kernels(n, m) != nullptr; }

ks_status ks_create(const ks_desc *desc, void *workspace, size_t ws_bytes, void *hip_stream,
                    ks_plan **out) {
    if (!out) return KS_E_ARG;
    *out = nullptr;
    if (!valid_desc(desc)) return KS_E_ARG;
    const ks::KernelSet *kset = ks::find_kernels(desc->n, desc->m);
    if (!kset) return KS_E_ARG;
    Layout lo;
    if (!make_layout(desc, kset, &lo)) return KS_E_ARG;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 || ws_bytes < lo.total)
        return KS_E_WORKSPACE;
    ks_plan *p = new (std::nothrow) ks_plan;
    if (!p) return KS_E_ARG;
    p->d = *desc;
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->ws = static_cast<char *>(workspace);
    p->kset = kset;
    p->lo = lo;
    p->smoothed = false;
    p->host_flags = 0;
    p->time_kind = KS_TIME_OFF;
    p->time_armed = false;
    p->ev_made = false;
    p->time_ms = 0.0;
    p->time_count = 0;
    p->tail_passes = 2;
    if (const char *e = std::getenv("KS_TAIL_PASSES")) p->tail_passes = std::atoi(e);
    // FP32 form: levels with more than switch_cols columns run in FP32
    int64_t switch_cols = 1024;
    if (const char *e = std::getenv("KS_FP32_SWITCH")) switch_cols = std::atoll(e);
    p->l_switch = 0;
    if (desc->precision == KS_FP32_FORM)
        while (p->l_switch < lo.L && lo.Nl[p->l_switch] > switch_cols) ++p->l_switch;
    *out = p;
    return KS_OK;
}

ks_status ks_smooth(ks_plan *p, const double *H, const double *F, const double *c,
                    const double *K, const double *G, const double *o, const double *C,
                    double *u_out) {
    if (!p || !u_out || !inputs_ok(p, F, c, K, G, o, C)) return KS_E_ARG;
    p->smoothed = false;
    enqueue_forward(p, H, F, c, K, G, o, C);
    enqueue_backward(p, u_out, nullptr);
    ks_status s = finish(p);
    p->smoothed = s == KS_OK;
    return s;
}

ks_status ks_smooth_cov(ks_plan *p, const double *H, const double *F, const double *c,
                        const double *K, const double *G, const double *o, const double *C,
                        double *u_out, double *cov_out) {
    if (!p || !u_out || !cov_out || !inputs_ok(p, F, c, K, G, o, C)) return KS_E_ARG;
    p->smoothed = false;
    enqueue_forward(p, H, F, c, K, G, o, C);
    enqueue_backward(p, u_out, cov_out);
    ks_status s = finish(p);
    p->smoothed = s == KS_OK;
    return s;
}

ks_status ks_covariances(ks_plan *p, double *cov_out) {
    if (!p || !cov_out) return KS_E_ARG;
    if (!p->smoothed) return KS_E_ORDER;
    enqueue_backward(p, nullptr, cov_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return KS_E_HIP;
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return KS_E_HIP;
    collect_time(p);
    return KS_OK;
}

ks_status ks_destroy(ks_plan *p) {
    if (!p) return KS_E_ARG;
    if (p->ev_made) {
        (void)hipEventDestroy(p->ev[0]);
        (void)hipEventDestroy(p->ev[1]);
    }
    delete p;
    return KS_OK;
}

const char *ks_status_string(ks_status s) {
    switch (s) {
    case KS_OK: return "ok";
    case KS_E_ARG: return "invalid argument or unsupported dimensions";
    case KS_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case KS_E_NOT_SPD: return "a covariance matrix is not symmetric positive definite";
    case KS_E_RANK: return "U A lacks full column rank";
    case KS_E_NONFINITE: return "non-finite value in the R factor";
    case KS_E_HIP: return "HIP runtime error";
    case KS_E_ORDER: return "ks_covariances called before a successful ks_smooth";
    }
    return "unknown status";
}

ks_status ks_plan_layout(const ks_plan *p, ks_layout *out) {
    if (!p || !out) return KS_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->levels = p->lo.L + 1;
    out->rrow_offset = (int64_t)(p->lo.off_rrows / sizeof(double));
    out->rrow_stride = (int64_t)p->d.n * (3 * p->d.n + 1);
    for (int l = 0; l <= p->lo.L; ++l) {
        out->level_rec_offset[l] = p->lo.rec_off[l];
        out->level_columns[l] = p->lo.Nl[l];
    }
    return KS_OK;
}

ks_status ks_time_kernels(ks_plan *p, int32_t kind) {
    if (!p || kind < KS_TIME_OFF || kind > KS_TIME_BWD_ALL) return KS_E_ARG;
    if (kind != KS_TIME_OFF && !p->ev_made) {
        if (hipEventCreate(&p->ev[0]) != hipSuccess) return KS_E_HIP;
        if (hipEventCreate(&p->ev[1]) != hipSuccess) {
            (void)hipEventDestroy(p->ev[0]);
            return KS_E_HIP;
        }
        p->ev_made = true;
    }
    p->time_kind = kind;
    p->time_armed = false;
    p->time_ms = 0.0;
    p->time_count = 0;
    return KS_OK;
}

ks_status ks_kernel_time(const ks_plan *p, double *total_ms, int64_t *count) {
    if (!p || !total_ms || !count) return KS_E_ARG;
    *total_ms = p->time_ms;
    *count = p->time_count;
    return KS_OK;
}

}  // extern "C"
