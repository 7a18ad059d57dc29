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

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ks.h"
#include "ks_internal.h"
#include "ks_objective.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxSideStreams = 8;

// Side streams (default priority) that independent launch sequences are forked
// onto from the caller's stream and joined back from, by events; under stream
// capture each side stream becomes one branch of the graph.  KS_SIDE_STREAMS
// sets their number (0: everything stays on the caller's stream).
struct SideStreams {
    int n = 0;
    hipStream_t s[kMaxSideStreams];
    hipEvent_t fork_ev, join_ev[kMaxSideStreams];

    void create() {
        int want = 4;
        if (const char *e = std::getenv("KS_SIDE_STREAMS")) want = std::atoi(e);
        want = std::max(0, std::min(want, kMaxSideStreams));
        n = 0;
        if (want > 0 && hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming) == hipSuccess) {
            for (int c = 0; c < want; ++c) {
                if (hipStreamCreateWithFlags(&s[c], hipStreamNonBlocking) != hipSuccess) break;
                if (hipEventCreateWithFlags(&join_ev[c], hipEventDisableTiming) != hipSuccess) {
                    (void)hipStreamDestroy(s[c]);
                    break;
                }
                n = c + 1;
            }
            if (n == 0) (void)hipEventDestroy(fork_ev);
        }
        (void)hipGetLastError();
    }
    void destroy(hipStream_t origin) {
        if (n == 0) return;
        (void)hipStreamSynchronize(origin);
        for (int c = 0; c < n; ++c) {
            (void)hipStreamDestroy(s[c]);
            (void)hipEventDestroy(join_ev[c]);
        }
        (void)hipEventDestroy(fork_ev);
        n = 0;
    }
    void fork(hipStream_t origin) {
        (void)hipEventRecord(fork_ev, origin);
        for (int c = 0; c < n; ++c) (void)hipStreamWaitEvent(s[c], fork_ev, 0);
    }
    void join(hipStream_t origin) {
        for (int c = 0; c < n; ++c) {
            (void)hipEventRecord(join_ev[c], s[c]);
            (void)hipStreamWaitEvent(origin, join_ev[c], 0);
        }
    }
};

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
    size_t off_rrows, off_sys, off_spm, off_slots, off_obj, off_flags, off_foldz, total;
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
    lo->off_obj = off;
    off = align_up(off + sizeof(double) * (size_t)(ks::kObjBlocks + 1));
    lo->off_flags = off;
    off = align_up(off + 64);
    lo->off_foldz = off;
    off = align_up(off + sizeof(double) * (size_t)(n * (n + 1)));
    lo->total = off;
    return true;
}

}  // namespace

// A captured launch sequence, keyed by the pointers it was captured with
// (the pointer set also fixes the mode).  KS_NO_GRAPH=1 in the environment
// turns capture off.
struct PassGraph {
    bool enabled = false, have = false;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *key[12] = {};
    int nkey = 0;

    void create() {
        const char *e = std::getenv("KS_NO_GRAPH");
        enabled = !(e && std::atoi(e) != 0) &&
                  hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
        (void)hipGetLastError();
    }
    void drop() {
        if (have) (void)hipGraphExecDestroy(exec);
        have = false;
    }
    void destroy() {
        drop();
        if (cap) (void)hipStreamDestroy(cap);
        cap = nullptr;
        enabled = false;
    }
    bool same_key(const void *const *k, int n) const {
        if (n != nkey) return false;
        for (int i = 0; i < n; ++i)
            if (k[i] != key[i]) return false;
        return true;
    }
    // Runs enqueue(stream) for `origin`.  A key seen for the first time runs
    // eagerly (callers whose pointers change every call never pay a capture);
    // the second consecutive call with the same key captures the sequence on
    // the private stream, and later ones replay it.
    template <class F>
    void run(hipStream_t origin, const void *const *k, int n, F &&enqueue) {
        if (!enabled) {
            enqueue(origin);
            return;
        }
        if (!same_key(k, n)) {
            drop();
            nkey = n;
            for (int i = 0; i < n; ++i) key[i] = k[i];
            enqueue(origin);
            return;
        }
        if (!have) {
            hipGraph_t g;
            if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                enqueue(cap);
                if (hipStreamEndCapture(cap, &g) == hipSuccess) {
                    if (hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess) have = true;
                    (void)hipGraphDestroy(g);
                }
            }
            (void)hipGetLastError();
            if (!have) enabled = false;  // capture unavailable: stay eager from now on
        }
        if (have) {
            (void)hipGraphLaunch(exec, origin);
        } else {
            enqueue(origin);
        }
    }
};

struct ks_plan {
    ks_desc d;
    hipStream_t stream;
    char *ws;
    const ks::KernelSet *kset;
    Layout lo;
    bool smoothed;
    unsigned host_flags;   // status word copied back after each call
    unsigned *pinned_flags;  // the same in pinned host memory (plans from ks_create; nullptr otherwise):
                             // a copy into it completes without the pageable staging round trip
    int l_switch;          // FP32 form: levels below this one run in FP32 (0 = none)
    int l0;                // first level of the forward tail launch
    int l1[3];             // lowest level of the backward tail launch, per backward mode
    double rank_tol;
    int fg, fg_from, bg, bg_from;  // level groups: levels per launch and first grouped level
    // instrumentation (ks_time_kernels)
    int time_kind;
    bool time_armed;       // events of the current call were recorded
    hipEvent_t ev[2];
    bool ev_made;
    double time_ms;
    int64_t time_count;
    // the last call's launch sequence as a graph, replayed while its pointers
    // and mode repeat (captured on a private stream: capture is not possible
    // on the legacy default stream a caller may pass)
    PassGraph graph;
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

// Schedule choices per (state dimension, precision form): how many unit passes
// of the single-workgroup forward / backward tail kernels the top levels may
// take, and (FP32 form) above how many columns a level runs in FP32.  Set by
// ks_set_tuning (an autotuned table); KS_TAIL_PASSES and KS_FP32_SWITCH in the
// environment override every entry.
struct Tuning {
    int32_t fwd_passes, bwd_passes;
    int64_t switch_cols;
    int32_t fwd_group, fwd_group_from, bwd_group, bwd_group_from;
    int32_t fwd_variant, bwd_variant;
};
constexpr int kTuneMaxN = 64;
std::mutex g_tune_mu;
Tuning g_tune[kTuneMaxN + 1][2];
bool g_tune_set[kTuneMaxN + 1][2];

Tuning tuning_for(int n, int precision) {
    Tuning t{2, 2, 1024, 1, 1, 1, 1, 0, 0};
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        if (n >= 0 && n <= kTuneMaxN && precision >= 0 && precision < 2 && g_tune_set[n][precision])
            t = g_tune[n][precision];
    }
    if (const char *e = std::getenv("KS_TAIL_PASSES")) t.fwd_passes = t.bwd_passes = std::atoi(e);
    if (const char *e = std::getenv("KS_FP32_SWITCH")) t.switch_cols = std::atoll(e);
    if (const char *e = std::getenv("KS_FWD_GROUP")) t.fwd_group = std::atoi(e);
    if (const char *e = std::getenv("KS_FWD_GROUP_FROM")) t.fwd_group_from = std::atoi(e);
    if (const char *e = std::getenv("KS_BWD_GROUP")) t.bwd_group = std::atoi(e);
    if (const char *e = std::getenv("KS_BWD_GROUP_FROM")) t.bwd_group_from = std::atoi(e);
    if (const char *e = std::getenv("KS_FWD_VARIANT")) t.fwd_variant = std::atoi(e);
    if (const char *e = std::getenv("KS_BWD_VARIANT")) t.bwd_variant = std::atoi(e);
    return t;
}

// the kernel set of a problem under the tuning of its (n, form): the tuned
// forward and backward variants, or the defaults where a variant does not exist
const ks::KernelSet *tuned_kernels(const ks_desc &d) {
    const Tuning tu = tuning_for(d.n, d.precision);
    const ks::KernelSet *k = ks::find_kernels(d.n, d.m, tu.fwd_variant, tu.bwd_variant);
    // a forward variant that whitens diagonal covariances only stands back for dense ones
    if (k && k->raw_diag_only && (d.K_layout != KS_COV_DIAG || d.C_layout != KS_COV_DIAG))
        k = ks::find_kernels(d.n, d.m, 0, tu.bwd_variant);
    return k ? k : ks::find_kernels(d.n, d.m);
}

// the level schedule of one problem: FP32 levels, first forward tail level,
// lowest backward tail level (identical for a plan, a batch and the engine)
struct Schedule {
    int l_switch, l0, l1;
    double rank_tol;
    int fg, fg_from, bg, bg_from;  // level groups (single plans)
};

Schedule make_schedule(const ks_desc &d, const ks::KernelSet *kset, const Layout &lo, int bwd_mode) {
    const Tuning tu = tuning_for(d.n, d.precision);
    Schedule sc{};
    sc.l_switch = 0;
    if (d.precision == KS_FP32_FORM)
        while (sc.l_switch < lo.L && lo.Nl[sc.l_switch] > tu.switch_cols) ++sc.l_switch;
    int l0 = tail_start(lo, kset->upb_fwd_tail, tu.fwd_passes, false);
    if (sc.l_switch > 0 && l0 <= sc.l_switch) l0 = sc.l_switch + 1;  // the tail reads FP64 records only
    if (kset->narrow_units > 0) {
        // the tail kernels do the arithmetic of the narrow-level kernels, so a
        // level whose own launch would run the wide-level forward stays out of
        // the tail: the tail passes never change results
        for (int l = 0; l <= lo.L; ++l) {
            const bool wide = l == 0 ? sc.l_switch == 0
                                     : ks::level_variant(kset, l, sc.l_switch, lo.Nl[l]) == ks::FV_F64;
            if (wide && l0 <= l) l0 = l + 1;
        }
    }
    sc.l0 = l0 > lo.L ? lo.L : l0;                                    // the base always runs in the tail
    int l1 = tail_start(lo, kset->upb_bwd_tail[bwd_mode], tu.bwd_passes, true);
    sc.l1 = l1 < sc.l_switch ? sc.l_switch : l1;
    sc.rank_tol = 64.0 * (sc.l_switch > 0 ? 1.1920928955078125e-07 : 2.220446049250313e-16);
    sc.fg = std::max(1, std::min(tu.fwd_group, 8));
    sc.fg_from = std::max(0, tu.fwd_group_from);
    sc.bg = std::max(1, std::min(tu.bwd_group, 8));
    sc.bg_from = std::max(0, tu.bwd_group_from);
    return sc;
}

// End (exclusive) of the forward launch that starts at level l: a group of
// fg levels from fg_from on, where the kernel family has group kernels; a
// group never reaches the tail and never crosses the FP32 switch.
int fwd_launch_end(const ks_plan *p, int l) {
    if (p->fg < 2 || l < p->fg_from || !p->kset->fwd_multi[0]) return l + 1;
    int end = std::min(l + p->fg, p->l0);
    if (l < p->l_switch) end = std::min(end, p->l_switch);
    return std::max(end, l + 1);
}

int64_t lcm64(int64_t a, int64_t b) {
    int64_t x = a, y = b;
    while (y) {
        const int64_t r = x % y;
        x = y;
        y = r;
    }
    return a / x * b;
}

// part 0: the whole forward sweep; 1: its head (status clear and the launch
// holding level 0); 2: the rest (needs a head that ends before the tail).
void enqueue_forward(ks_plan *p, const double *H, const double *F, const double *c,
                     const double *K, const double *G, const double *o, const double *C, int part = 0) {
    const Layout &lo = p->lo;
    const int64_t n = p->d.n;
    const int64_t rrec = n * (3 * n + 1);
    double *rrows = seg_d(p, lo.off_rrows);
    double *sys = seg_d(p, lo.off_sys);
    double *slots = seg_d(p, lo.off_slots);
    unsigned *flags = reinterpret_cast<unsigned *>(p->ws + lo.off_flags);
    if (part != 2) {
        ks::launch_clear_flags(flags, p->stream);
        mark(p, KS_TIME_FWD_ALL, 0);
    }
    const int l0 = p->l0;
    const int ls = p->l_switch;
    ks::FwdArgs a{};
    a.k = p->d.k;
    a.m = p->d.m;
    a.K_diag = p->d.K_layout == KS_COV_DIAG;
    a.C_diag = p->d.C_layout == KS_COV_DIAG;
    a.H = H; a.F = F; a.c = c; a.K = K; a.G = G; a.o = o; a.C = C;
    a.flags = flags;
    a.fold_z = seg_d(p, lo.off_foldz);
    a.fold_cnt = flags + ks::kFoldCounter;
    const int head_end = l0 >= 1 ? fwd_launch_end(p, 0) : 0;
    const int l_first = part == 2 ? head_end : 0, l_end = part == 1 ? head_end : l0;
    for (int l = l_first; l < l_end;) {
        const int end = fwd_launch_end(p, l);
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
        const int v = ks::level_variant(p->kset, l, ls, lo.Nl[l]);
        if (end - l >= 2) {
            // levels l .. end-1 in one launch: each workgroup an aligned subtree
            ks::FwdMultiArgs ma{};
            ma.a = a;
            ma.l_first = l;
            ma.nlev = end - l;
            ma.U = lcm64(p->kset->upb_multi, (int64_t)1 << (ma.nlev - 1));
            ma.groups = std::max<int64_t>(1, a.units / ma.U);
            ma.sys = sys;
            ma.rrows = rrows;
            ma.slots = a.slots;
            ma.slot_pairs = lo.slot_off[end] - lo.slot_off[l];
            for (int q = 0; q <= lo.L; ++q) {
                ma.sys_off[q] = lo.sys_off[q];
                ma.rec_off[q] = lo.rec_off[q];
                ma.Nl[q] = lo.Nl[q];
            }
            if (l == 0) mark(p, KS_TIME_FWD_LEVEL0, 0);
            (l == 0 ? p->kset->fwd_multi_raw[v == ks::FV_F32] : p->kset->fwd_multi[v])(ma, p->stream);
            if (l == 0) mark(p, KS_TIME_FWD_LEVEL0, 1);
        } else if (l == 0) {
            const int f32 = v == ks::FV_F32;
            mark(p, KS_TIME_FWD_LEVEL0, 0);
            if ((lo.Nl[l] & 1) && p->kset->fwd_fold_raw[f32]) {
                p->kset->fwd_fold_raw[f32](a, p->stream);  // the level kernel folds the last column itself
                mark(p, KS_TIME_FWD_LEVEL0, 1);
            } else {
                // the level-0 bracket holds the level kernel alone (not the fold)
                p->kset->fwd_raw[f32](a, p->stream);
                mark(p, KS_TIME_FWD_LEVEL0, 1);
                if (lo.Nl[l] & 1) p->kset->fold_raw[f32](a, p->stream);
            }
        } else if ((lo.Nl[l] & 1) && p->kset->fwd_fold[v]) {
            p->kset->fwd_fold[v](a, p->stream);  // the level kernel folds the last column itself
        } else {
            p->kset->fwd[v](a, p->stream);
            if (lo.Nl[l] & 1) p->kset->fold[v](a, p->stream);
        }
        l = end;
    }
    if (part == 1) return;
    ks::FwdTailArgs ta{};
    ta.a = a;
    ta.l0 = l0;
    ta.L = lo.L;
    ta.sys = sys;
    ta.rrows = rrows;
    ta.slots = slots;
    ta.nprev = lo.slot_off[l0];
    ta.rank_tol = p->rank_tol;
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

void enqueue_backward(ks_plan *p, double *u_out, double *cov_out, double *lag1_out = nullptr) {
    const Layout &lo = p->lo;
    const int mode = (u_out && cov_out) ? ks::BWD_BOTH : (u_out ? ks::BWD_Y : ks::BWD_COV);
    ks::BwdArgs b{};
    b.k = p->d.k;
    b.rrows_all = seg_d(p, lo.off_rrows);
    b.u_in = u_out;
    b.u_out = u_out;
    b.cov = cov_out;
    b.spm = seg_d(p, lo.off_spm);
    b.lag1 = cov_out ? lag1_out : nullptr;
    b.spm_first = lo.spm_first;
    b.store_s = cov_out != nullptr;
    for (int l = 0; l <= lo.L; ++l) {
        b.rec_off[l] = lo.rec_off[l];
        b.Nl[l] = lo.Nl[l];
    }
    const int l1 = p->l1[mode];
    mark(p, KS_TIME_BWD_ALL, 0);
    if (l1 <= lo.L) {
        b.level = lo.L;
        b.l_lo = l1;
        if (l1 == 0) mark(p, KS_TIME_BWD_LEVEL0, 0);
        p->kset->bwd_tail[mode](b, p->stream);
        if (l1 == 0) mark(p, KS_TIME_BWD_LEVEL0, 1);
    }
    // below the tail: groups of bg levels from bg_from on (highest group
    // first; a group never crosses the FP32 switch), one launch per level
    // elsewhere
    const int top0 = (l1 <= lo.L ? l1 : lo.L + 1) - 1;
    for (int top = top0; top >= 0;) {
        int low = top;
        if (p->bg >= 2 && top >= p->bg_from && p->kset->bwd_multi[mode][0]) {
            // the group holding `top` in the partition bg_from + q bg of the levels
            low = p->bg_from + (top - p->bg_from) / p->bg * p->bg;
            if (top >= p->l_switch && low < p->l_switch) low = p->l_switch;
        }
        b.level = top;
        b.l_lo = low;
        const int tr = top < p->l_switch ? 1 : 0;
        if (low == 0) mark(p, KS_TIME_BWD_LEVEL0, 0);
        if (low < top)
            p->kset->bwd_multi[mode][tr](b, p->stream);
        else
            p->kset->bwd[mode][tr](b, p->stream);
        if (low == 0) mark(p, KS_TIME_BWD_LEVEL0, 1);
        top = low - 1;
    }
    mark(p, KS_TIME_BWD_ALL, 1);
}

ks_status finish(ks_plan *p) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return KS_E_HIP;
    const unsigned *flags = reinterpret_cast<const unsigned *>(p->ws + p->lo.off_flags);
    unsigned *dst = p->pinned_flags ? p->pinned_flags : &p->host_flags;
    e = hipMemcpyAsync(dst, flags, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream);
    if (e != hipSuccess) return KS_E_HIP;
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return KS_E_HIP;
    collect_time(p);
    const unsigned f = *dst;
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

// One smoothing pass (forward, then the backward for the given outputs) on
// the plan's stream, as a replayed graph when possible.  Timed calls run
// eagerly (their event marks bracket individual launches), except that a call
// timing the level-0 launch replays everything after level 0.
void run_pass(ks_plan *p, const double *H, const double *F, const double *c, const double *K,
              const double *G, const double *o, const double *C, double *u_out, double *cov_out,
              double *lag1_out) {
    auto enqueue = [&](hipStream_t st) {
        hipStream_t keep = p->stream;
        p->stream = st;
        enqueue_forward(p, H, F, c, K, G, o, C);
        enqueue_backward(p, u_out, cov_out, lag1_out);
        p->stream = keep;
    };
    if (p->time_kind == KS_TIME_FWD_LEVEL0 && p->l0 >= 1 && fwd_launch_end(p, 0) < p->l0) {
        // the bracketed level-0 launch stays eager (events captured inside a
        // graph would lengthen it); the rest of the pass replays as a graph
        enqueue_forward(p, H, F, c, K, G, o, C, 1);
        auto rest = [&](hipStream_t st) {
            hipStream_t keep = p->stream;
            p->stream = st;
            enqueue_forward(p, H, F, c, K, G, o, C, 2);
            enqueue_backward(p, u_out, cov_out, lag1_out);
            p->stream = keep;
        };
        const void *key[11] = {H, F, c, K, G, o, C, u_out, cov_out, lag1_out, &p->l0};
        p->graph.run(p->stream, key, 11, rest);
        return;
    }
    if (p->time_kind != KS_TIME_OFF) {
        enqueue(p->stream);
        return;
    }
    const void *key[10] = {H, F, c, K, G, o, C, u_out, cov_out, lag1_out};
    p->graph.run(p->stream, key, 10, enqueue);
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
    if (!ks::find_kernels(desc->n, desc->m)) return KS_E_ARG;
    const ks::KernelSet *kset = tuned_kernels(*desc);
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
    p->pinned_flags = nullptr;
    if (hipHostMalloc(reinterpret_cast<void **>(&p->pinned_flags), sizeof(unsigned), hipHostMallocDefault) !=
        hipSuccess)
        p->pinned_flags = nullptr;  // the pageable word serves
    p->time_kind = KS_TIME_OFF;
    p->time_armed = false;
    p->ev_made = false;
    p->graph.create();
    p->time_ms = 0.0;
    p->time_count = 0;
    for (int mode = 0; mode < 3; ++mode) {
        const Schedule sc = make_schedule(*desc, kset, lo, mode);
        p->l_switch = sc.l_switch;
        p->l0 = sc.l0;
        p->l1[mode] = sc.l1;
        p->rank_tol = sc.rank_tol;
        p->fg = sc.fg;
        p->fg_from = sc.fg_from;
        p->bg = sc.bg;
        p->bg_from = sc.bg_from;
    }
    *out = p;
    return KS_OK;
}

ks_status ks_smooth(ks_plan *p, const double *H, const double *F, const double *c,
                    const double *K, const double *G, const double *o, const double *C,
                    double *u_out) {
    if (!p || !u_out || !inputs_ok(p, F, c, K, G, o, C)) return KS_E_ARG;
    p->smoothed = false;
    run_pass(p, H, F, c, K, G, o, C, u_out, nullptr, nullptr);
    ks_status s = finish(p);
    p->smoothed = s == KS_OK;
    return s;
}

ks_status ks_smooth_cov(ks_plan *p, const double *H, const double *F, const double *c,
                        const double *K, const double *G, const double *o, const double *C,
                        double *u_out, double *cov_out) {
    if (!p || !u_out || !cov_out || !inputs_ok(p, F, c, K, G, o, C)) return KS_E_ARG;
    p->smoothed = false;
    run_pass(p, H, F, c, K, G, o, C, u_out, cov_out, nullptr);
    ks_status s = finish(p);
    p->smoothed = s == KS_OK;
    return s;
}

ks_status ks_smooth_cov_lag1(ks_plan *p, const double *H, const double *F, const double *c,
                             const double *K, const double *G, const double *o, const double *C,
                             double *u_out, double *cov_out, double *lag1_out) {
    if (!p || !u_out || !cov_out || (!lag1_out && p->d.k > 0) || !inputs_ok(p, F, c, K, G, o, C))
        return KS_E_ARG;
    p->smoothed = false;
    run_pass(p, H, F, c, K, G, o, C, u_out, cov_out, lag1_out);
    ks_status s = finish(p);
    p->smoothed = s == KS_OK;
    return s;
}

ks_status ks_objective(ks_plan *p, const double *H, const double *F, const double *c,
                       const double *K, const double *G, const double *o, const double *C,
                       const double *u, double *terms_out, double *total) {
    if (!p || !total) return KS_E_ARG;
    const ks_desc &d = p->d;
    if (d.n > 64 || d.m > 64) return KS_E_ARG;
    if (d.k > 0 && (!c || !K || (u && !F))) return KS_E_ARG;
    if (d.m > 0 && (!o || !C || (u && !G))) return KS_E_ARG;
    ks::ObjArgs a{};
    a.k = d.k;
    a.n = d.n;
    a.m = d.m;
    a.K_diag = d.K_layout == KS_COV_DIAG;
    a.C_diag = d.C_layout == KS_COV_DIAG;
    a.H = u ? H : nullptr;
    a.F = F; a.c = c; a.K = K; a.G = G; a.o = o; a.C = C;
    a.u = u;
    a.terms = terms_out;
    a.partial = reinterpret_cast<double *>(p->ws + p->lo.off_obj);
    a.flags = reinterpret_cast<unsigned *>(p->ws + p->lo.off_flags);
    ks::launch_clear_flags(a.flags, p->stream);
    ks::launch_objective(a, p->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return KS_E_HIP;
    double v = 0.0;
    unsigned f = 0;
    e = hipMemcpyAsync(&v, a.partial + ks::objective_blocks(d.k), sizeof(double), hipMemcpyDeviceToHost,
                       p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&f, a.flags, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return KS_E_HIP;
    *total = v;
    if (f & ks::FLAG_NOT_SPD) return KS_E_NOT_SPD;
    if (!std::isfinite(v)) return KS_E_NONFINITE;
    return KS_OK;
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
    p->graph.destroy();
    if (p->pinned_flags) (void)hipHostFree(p->pinned_flags);
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
    case KS_E_BUSY: return "the engine cannot admit the request now (workspace, tables or status words in use)";
    }
    return "unknown status";
}

ks_status ks_set_tuning(int32_t n, int32_t precision, const ks_tuning *t) {
    if (n < 1 || n > kTuneMaxN || (precision != KS_FP64 && precision != KS_FP32_FORM) || !t ||
        t->fwd_tail_passes < 0 || t->bwd_tail_passes < 0 || t->fp32_switch_columns < 1 || t->fwd_group < 1 ||
        t->fwd_group > 8 || t->fwd_group_from < 0 || t->bwd_group < 1 || t->bwd_group > 8 ||
        t->bwd_group_from < 0 || t->fwd_variant < 0 || t->bwd_variant < 0)
        return KS_E_ARG;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[n][precision] = Tuning{t->fwd_tail_passes, t->bwd_tail_passes, t->fp32_switch_columns, t->fwd_group,
                                  t->fwd_group_from, t->bwd_group, t->bwd_group_from, t->fwd_variant,
                                  t->bwd_variant};
    g_tune_set[n][precision] = true;
    return KS_OK;
}

ks_status ks_get_tuning(int32_t n, int32_t precision, ks_tuning *out) {
    if (n < 1 || n > kTuneMaxN || (precision != KS_FP64 && precision != KS_FP32_FORM) || !out)
        return KS_E_ARG;
    const Tuning t = tuning_for(n, precision);
    std::memset(out, 0, sizeof(*out));
    out->fwd_tail_passes = t.fwd_passes;
    out->bwd_tail_passes = t.bwd_passes;
    out->fp32_switch_columns = t.switch_cols;
    out->fwd_group = t.fwd_group;
    out->fwd_group_from = t.fwd_group_from;
    out->bwd_group = t.bwd_group;
    out->bwd_group_from = t.bwd_group_from;
    out->fwd_variant = t.fwd_variant;
    out->bwd_variant = t.bwd_variant;
    return KS_OK;
}

int32_t ks_kernel_variants(int32_t n, int32_t m, int32_t backward) {
    return ks::kernel_variants(n, m, backward != 0);
}

ks_status ks_plan_schedule(const ks_plan *p, int32_t *fp32_levels, int32_t *fwd_tail_level,
                           int32_t *bwd_tail_level) {
    if (!p || !fp32_levels || !fwd_tail_level || !bwd_tail_level) return KS_E_ARG;
    *fp32_levels = p->l_switch;
    *fwd_tail_level = p->l0;
    *bwd_tail_level = p->l1[ks::BWD_BOTH];
    return KS_OK;
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

namespace ks {

ks_status smooth_cov_on(const ks_desc *desc, void *workspace, size_t ws_bytes, hipStream_t stream,
                        const double *H, const double *F, const double *c, const double *K,
                        const double *G, const double *o, const double *C, double *u_out,
                        double *cov_out) {
    if (!valid_desc(desc) || !u_out || !cov_out) return KS_E_ARG;
    if (!find_kernels(desc->n, desc->m)) return KS_E_ARG;
    const KernelSet *kset = tuned_kernels(*desc);
    ks_plan p;  // host state on the stack: no graph, no timing events
    if (!make_layout(desc, kset, &p.lo)) return KS_E_ARG;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 || ws_bytes < p.lo.total)
        return KS_E_WORKSPACE;
    p.d = *desc;
    p.stream = stream;
    p.ws = static_cast<char *>(workspace);
    p.kset = kset;
    p.smoothed = false;
    p.host_flags = 0;
    p.pinned_flags = nullptr;  // allocates nothing
    p.time_kind = KS_TIME_OFF;
    p.time_armed = false;
    p.ev_made = false;
    p.time_ms = 0.0;
    p.time_count = 0;
    for (int mode = 0; mode < 3; ++mode) {  // as ks_create
        const Schedule sc = make_schedule(*desc, kset, p.lo, mode);
        p.l_switch = sc.l_switch;
        p.l0 = sc.l0;
        p.l1[mode] = sc.l1;
        p.rank_tol = sc.rank_tol;
        p.fg = sc.fg;
        p.fg_from = sc.fg_from;
        p.bg = sc.bg;
        p.bg_from = sc.bg_from;
    }
    if (!inputs_ok(&p, F, c, K, G, o, C)) return KS_E_ARG;
    run_pass(&p, H, F, c, K, G, o, C, u_out, cov_out, nullptr);
    return finish(&p);
}

}  // namespace ks

// ====================================================================== batch
//
// Many problems (any mix of n, m, k, covariance layouts and precision forms)
// advanced together: every forward level step is one launch per kernel class
// (n, observation class) and precision variant covering the units of that
// level of every problem still above its tail; each problem's top levels run
// as one workgroup of a single tail launch; the backward mirrors it.  The
// schedule of each problem is exactly that of a single plan, so its results
// are bitwise those of ks_smooth_cov on it alone.  Launch arguments live in
// device tables (one upload per set of input/output pointers) and the launch
// sequence is captured once in a hipGraph and replayed.

namespace {

struct BatchProblem {
    ks_desc d;
    const ks::KernelSet *kset;
    Layout lo;
    size_t ws_off;  // of the problem's region in the workspace
    int l_switch;   // levels below run in FP32 (FP32 form)
    int l0;         // first forward level in the tail launch
    int l1;         // lowest backward level in the tail launch
    double rank_tol;
};

// one batched launch: a kernel and its block map (ranges in the table arrays)
struct BLaunch {
    enum Kind { FWD, FOLD, FTAIL, BWD, BTAIL } kind;
    const ks::KernelSet *kset;
    int variant;    // forward: FwdVariant (raw: 0/1); backward: record type
    bool raw;       // level-0 forward / tail starting at level 0
    int64_t map0, blocks;
};

template <class T>
size_t tab_bytes(size_t n) { return align_up(sizeof(T) * n); }

}  // namespace

struct ks_batch {
    hipStream_t stream;
    char *ws;
    int32_t count;
    int mode_cov;  // mode the cached tables/graph were built for (-1 none)
    std::vector<BatchProblem> probs;
    std::vector<BLaunch> launches[2];  // [want_cov]
    // host tables
    std::vector<ks::FwdArgs> fwd_tab;
    std::vector<ks::FwdTailArgs> tail_tab;
    std::vector<ks::BwdArgs> bwd_tab;
    std::vector<int32_t> map_item, map_level;
    std::vector<int64_t> map_blk;
    // device tables
    size_t off_fwd, off_tail, off_bwd, off_item, off_blk, off_level, off_flags, total;
    std::vector<ks_io> cached_io;
    hipGraphExec_t exec;
    bool have_exec;
    bool use_graph;
    std::vector<unsigned> host_flags;
    hipStream_t cap;  // private capture stream (capture is impossible on the legacy default stream)
    // kernel classes share no data, so their launch sequences run
    // concurrently, one side stream per class (a captured graph gets one
    // branch per class)
    SideStreams side;
};

namespace {

template <class T>
T *dptr(ks_batch *b, size_t off) { return reinterpret_cast<T *>(b->ws + off); }

// Build the schedule: table entries with placeholder pointers (filled per call
// by fill_tables) and the launch list, for want_cov = 0 and 1.
void plan_batch(ks_batch *b) {
    const int P = b->count;
    b->fwd_tab.clear();
    b->tail_tab.clear();
    b->bwd_tab.assign(P, ks::BwdArgs{});
    b->map_item.clear();
    b->map_blk.clear();
    b->map_level.clear();
    auto add_map = [&](int32_t item, int64_t blk, int32_t lvl) {
        b->map_item.push_back(item);
        b->map_blk.push_back(blk);
        b->map_level.push_back(lvl);
    };
    // distinct kernel sets in first-seen order
    std::vector<const ks::KernelSet *> classes;
    for (auto &pr : b->probs)
        if (std::find(classes.begin(), classes.end(), pr.kset) == classes.end())
            classes.push_back(pr.kset);
    int maxL0 = 0, maxL1 = 0;
    for (auto &pr : b->probs) {
        maxL0 = std::max(maxL0, pr.l0);
        maxL1 = std::max(maxL1, pr.l1);
    }
    // forward entries: one FwdArgs per (problem, level < l0)
    std::vector<std::vector<int32_t>> fwd_index(P);
    for (int i = 0; i < P; ++i) {
        fwd_index[i].assign(b->probs[i].l0, -1);
        for (int l = 0; l < b->probs[i].l0; ++l) {
            fwd_index[i][l] = (int32_t)b->fwd_tab.size();
            b->fwd_tab.push_back(ks::FwdArgs{});
        }
    }
    for (int i = 0; i < P; ++i) b->tail_tab.push_back(ks::FwdTailArgs{});

    for (int cov = 0; cov < 2; ++cov) {
        auto &L = b->launches[cov];
        L.clear();
        const int mode = cov ? ks::BWD_BOTH : ks::BWD_Y;
        for (int s = 0; s < maxL0; ++s) {
            for (auto *cls : classes) {
                for (int v = 0; v < ks::kFwdVariants; ++v) {
                    BLaunch fl{BLaunch::FWD, cls, v, s == 0, (int64_t)b->map_item.size(), 0};
                    for (int i = 0; i < P; ++i) {
                        const BatchProblem &pr = b->probs[i];
                        if (pr.kset != cls || s >= pr.l0) continue;
                        const int vi = ks::level_variant(pr.kset, s, pr.l_switch, pr.lo.Nl[s]);
                        if (vi != v) continue;
                        const int64_t units = pr.lo.Nl[s] / 2;
                        const int64_t blocks = (units + cls->upb_fwd - 1) / cls->upb_fwd;
                        for (int64_t k = 0; k < blocks; ++k) add_map(fwd_index[i][s], k, s);
                        fl.blocks += blocks;
                    }
                    if (fl.blocks) L.push_back(fl);
                    BLaunch fo{BLaunch::FOLD, cls, v, s == 0, (int64_t)b->map_item.size(), 0};
                    for (int i = 0; i < P; ++i) {
                        const BatchProblem &pr = b->probs[i];
                        if (pr.kset != cls || s >= pr.l0 || !(pr.lo.Nl[s] & 1)) continue;
                        const int vi = ks::level_variant(pr.kset, s, pr.l_switch, pr.lo.Nl[s]);
                        if (vi != v) continue;
                        add_map(fwd_index[i][s], 0, s);
                        fo.blocks += 1;
                    }
                    if (fo.blocks) L.push_back(fo);
                }
            }
        }
        for (auto *cls : classes) {
            for (int raw = 1; raw >= 0; --raw) {
                BLaunch t{BLaunch::FTAIL, cls, 0, raw == 1, (int64_t)b->map_item.size(), 0};
                for (int i = 0; i < P; ++i) {
                    const BatchProblem &pr = b->probs[i];
                    if (pr.kset != cls || (pr.l0 == 0) != (raw == 1)) continue;
                    add_map(i, 0, pr.l0);
                    t.blocks += 1;
                }
                if (t.blocks) L.push_back(t);
            }
        }
        for (auto *cls : classes) {
            BLaunch t{BLaunch::BTAIL, cls, mode, false, (int64_t)b->map_item.size(), 0};
            for (int i = 0; i < P; ++i) {
                if (b->probs[i].kset != cls || b->probs[i].l1 > b->probs[i].lo.L) continue;
                add_map(i, 0, b->probs[i].lo.L);
                t.blocks += 1;
            }
            if (t.blocks) L.push_back(t);
        }
        for (int s = maxL1 - 1; s >= 0; --s) {
            for (auto *cls : classes) {
                for (int tr = 0; tr < 2; ++tr) {
                    BLaunch bl{BLaunch::BWD, cls, tr, false, (int64_t)b->map_item.size(), 0};
                    for (int i = 0; i < P; ++i) {
                        const BatchProblem &pr = b->probs[i];
                        if (pr.kset != cls || s >= std::min(pr.l1, pr.lo.L + 1)) continue;
                        if ((s < pr.l_switch ? 1 : 0) != tr) continue;
                        const int64_t units = (pr.lo.Nl[s] + 1) / 2;
                        const int64_t blocks = (units + cls->upb_bwd[mode] - 1) / cls->upb_bwd[mode];
                        for (int64_t k = 0; k < blocks; ++k) add_map(i, k, s);
                        bl.blocks += blocks;
                    }
                    if (bl.blocks) L.push_back(bl);
                }
            }
        }
    }
}

// per-call contents of the tables (pointers of the io arrays)
void fill_tables(ks_batch *b, const ks_io *io, bool cov) {
    const int P = b->count;
    int64_t fi = 0;
    for (int i = 0; i < P; ++i) {
        const BatchProblem &pr = b->probs[i];
        const Layout &lo = pr.lo;
        char *base = b->ws + pr.ws_off;
        const int64_t n = pr.d.n, rrec = n * (3 * n + 1);
        double *rrows = reinterpret_cast<double *>(base + lo.off_rrows);
        double *sys = reinterpret_cast<double *>(base + lo.off_sys);
        double *slots = reinterpret_cast<double *>(base + lo.off_slots);
        unsigned *flags = dptr<unsigned>(b, b->off_flags) + i;
        ks::FwdArgs a{};
        a.k = pr.d.k;
        a.m = pr.d.m;
        a.K_diag = pr.d.K_layout == KS_COV_DIAG;
        a.C_diag = pr.d.C_layout == KS_COV_DIAG;
        a.H = io[i].H; a.F = io[i].F; a.c = io[i].c; a.K = io[i].K;
        a.G = io[i].G; a.o = io[i].o; a.C = io[i].C;
        a.flags = flags;
        for (int l = 0; l < pr.l0; ++l) {
            a.Nl = lo.Nl[l];
            a.units = lo.Nl[l] / 2;
            a.level = l;
            a.sys_in = l >= 1 ? sys + lo.sys_off[l] : nullptr;
            a.sys_out = sys + lo.sys_off[l + 1];
            a.rrows = rrows + lo.rec_off[l] * rrec;
            a.slots = slots + 2 * lo.slot_off[l];
            const int64_t blocks = (a.units + pr.kset->upb_fwd - 1) / pr.kset->upb_fwd;
            a.fold_slot = a.slots + 2 * blocks;
            b->fwd_tab[fi++] = a;
        }
        ks::FwdTailArgs &ta = b->tail_tab[i];
        ta = ks::FwdTailArgs{};
        ta.a = a;
        ta.l0 = pr.l0;
        ta.L = lo.L;
        ta.sys = sys;
        ta.rrows = rrows;
        ta.slots = slots;
        ta.nprev = lo.slot_off[pr.l0];
        ta.rank_tol = pr.rank_tol;
        for (int l = 0; l <= lo.L; ++l) {
            ta.sys_off[l] = lo.sys_off[l];
            ta.rec_off[l] = lo.rec_off[l];
            ta.Nl[l] = lo.Nl[l];
        }
        ks::BwdArgs &bw = b->bwd_tab[i];
        bw = ks::BwdArgs{};
        bw.k = pr.d.k;
        bw.level = lo.L;
        bw.l_lo = pr.l1;
        bw.store_s = cov;
        bw.rrows_all = rrows;
        bw.u_in = io[i].u_out;
        bw.u_out = io[i].u_out;
        bw.cov = cov ? io[i].cov_out : nullptr;
        bw.spm = reinterpret_cast<double *>(base + lo.off_spm);
        bw.spm_first = lo.spm_first;
        for (int l = 0; l <= lo.L; ++l) {
            bw.rec_off[l] = lo.rec_off[l];
            bw.Nl[l] = lo.Nl[l];
        }
    }
}

hipError_t upload_tables(ks_batch *b) {
    hipError_t e;
    if ((e = hipMemcpyAsync(dptr<char>(b, b->off_fwd), b->fwd_tab.data(), sizeof(ks::FwdArgs) * b->fwd_tab.size(),
                            hipMemcpyHostToDevice, b->stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(dptr<char>(b, b->off_tail), b->tail_tab.data(), sizeof(ks::FwdTailArgs) * b->tail_tab.size(),
                            hipMemcpyHostToDevice, b->stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(dptr<char>(b, b->off_bwd), b->bwd_tab.data(), sizeof(ks::BwdArgs) * b->bwd_tab.size(),
                            hipMemcpyHostToDevice, b->stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(dptr<char>(b, b->off_item), b->map_item.data(), sizeof(int32_t) * b->map_item.size(),
                            hipMemcpyHostToDevice, b->stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(dptr<char>(b, b->off_blk), b->map_blk.data(), sizeof(int64_t) * b->map_blk.size(),
                            hipMemcpyHostToDevice, b->stream)) != hipSuccess) return e;
    return hipMemcpyAsync(dptr<char>(b, b->off_level), b->map_level.data(), sizeof(int32_t) * b->map_level.size(),
                          hipMemcpyHostToDevice, b->stream);
}

void enqueue_batch(ks_batch *b, bool cov) {
    const int mode = cov ? ks::BWD_BOTH : ks::BWD_Y;
    ks::launch_clear_flags_n(dptr<unsigned>(b, b->off_flags), b->count, b->stream);
    const ks::FwdArgs *ft = dptr<ks::FwdArgs>(b, b->off_fwd);
    const ks::FwdTailArgs *tt = dptr<ks::FwdTailArgs>(b, b->off_tail);
    const ks::BwdArgs *bt = dptr<ks::BwdArgs>(b, b->off_bwd);
    const int32_t *mi = dptr<int32_t>(b, b->off_item);
    const int64_t *mb = dptr<int64_t>(b, b->off_blk);
    const int32_t *ml = dptr<int32_t>(b, b->off_level);
    // kernel classes in order of first appearance, each on its own side stream
    std::vector<const ks::KernelSet *> classes;
    for (const BLaunch &L : b->launches[cov])
        if (std::find(classes.begin(), classes.end(), L.kset) == classes.end()) classes.push_back(L.kset);
    const bool fork = b->side.n > 0 && classes.size() > 1;
    if (fork) b->side.fork(b->stream);
    for (const BLaunch &L : b->launches[cov]) {
        const ks::BlockMap bm{mi + L.map0, mb + L.map0, ml + L.map0};
        const int cls = (int)(std::find(classes.begin(), classes.end(), L.kset) - classes.begin());
        hipStream_t st = fork ? b->side.s[cls % b->side.n] : b->stream;
        switch (L.kind) {
        case BLaunch::FWD:
            if (L.raw) L.kset->fwd_raw_b[L.variant == ks::FV_F32](ft, bm, L.blocks, st);
            else L.kset->fwd_b[L.variant](ft, bm, L.blocks, st);
            break;
        case BLaunch::FOLD:
            if (L.raw) L.kset->fold_raw_b[L.variant == ks::FV_F32](ft, bm, L.blocks, st);
            else L.kset->fold_b[L.variant](ft, bm, L.blocks, st);
            break;
        case BLaunch::FTAIL:
            (L.raw ? L.kset->fwd_tail_raw_b : L.kset->fwd_tail_b)(tt, bm, L.blocks, st);
            break;
        case BLaunch::BTAIL:
            L.kset->bwd_tail_b[mode](bt, bm, L.blocks, st);
            break;
        case BLaunch::BWD:
            L.kset->bwd_b[mode][L.variant](bt, bm, L.blocks, st);
            break;
        }
    }
    if (fork) b->side.join(b->stream);
}

bool same_io(const std::vector<ks_io> &a, const ks_io *io, int n) {
    if ((int)a.size() != n) return false;
    return std::memcmp(a.data(), io, sizeof(ks_io) * n) == 0;
}

}  // namespace

extern "C" {

static ks_status batch_setup(int32_t count, const ks_desc *descs, ks_batch *b, size_t *total) {
    if (count <= 0 || !descs) return KS_E_ARG;
    size_t off = 0;
    b->count = count;
    b->probs.resize(count);
    for (int i = 0; i < count; ++i) {
        BatchProblem &pr = b->probs[i];
        pr.d = descs[i];
        if (!valid_desc(&pr.d)) return KS_E_ARG;
        pr.kset = ks::find_kernels(pr.d.n, pr.d.m) ? tuned_kernels(pr.d) : nullptr;
        if (!pr.kset) return KS_E_ARG;
        if (!make_layout(&pr.d, pr.kset, &pr.lo)) return KS_E_ARG;
        pr.ws_off = off;
        off = align_up(off + pr.lo.total);
        const Schedule sc = make_schedule(pr.d, pr.kset, pr.lo, ks::BWD_BOTH);
        pr.l_switch = sc.l_switch;
        pr.l0 = sc.l0;
        pr.l1 = sc.l1;
        pr.rank_tol = sc.rank_tol;
    }
    plan_batch(b);
    b->off_fwd = off;
    off += tab_bytes<ks::FwdArgs>(b->fwd_tab.size());
    b->off_tail = off;
    off += tab_bytes<ks::FwdTailArgs>(b->tail_tab.size());
    b->off_bwd = off;
    off += tab_bytes<ks::BwdArgs>(b->bwd_tab.size());
    b->off_item = off;
    off += tab_bytes<int32_t>(b->map_item.size());
    b->off_blk = off;
    off += tab_bytes<int64_t>(b->map_blk.size());
    b->off_level = off;
    off += tab_bytes<int32_t>(b->map_level.size());
    b->off_flags = off;
    off += tab_bytes<unsigned>(count);
    b->total = off;
    *total = off;
    return KS_OK;
}

size_t ks_batch_workspace_bytes(int32_t count, const ks_desc *descs) {
    ks_batch tmp;
    size_t total = 0;
    if (batch_setup(count, descs, &tmp, &total) != KS_OK) return 0;
    return total;
}

ks_status ks_batch_create(int32_t count, const ks_desc *descs, void *workspace, size_t ws_bytes,
                          void *hip_stream, ks_batch **out) {
    if (!out) return KS_E_ARG;
    *out = nullptr;
    ks_batch *b = new (std::nothrow) ks_batch;
    if (!b) return KS_E_ARG;
    size_t total = 0;
    ks_status st = batch_setup(count, descs, b, &total);
    if (st != KS_OK) {
        delete b;
        return st;
    }
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 || ws_bytes < total) {
        delete b;
        return KS_E_WORKSPACE;
    }
    b->ws = static_cast<char *>(workspace);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->mode_cov = -1;
    b->have_exec = false;
    b->use_graph = !(std::getenv("KS_NO_GRAPH") && std::atoi(std::getenv("KS_NO_GRAPH")) != 0);
    b->host_flags.assign(count, 0u);
    b->cap = nullptr;
    if (b->use_graph && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) b->cap = nullptr;
    (void)hipGetLastError();
    b->side.create();
    *out = b;
    return KS_OK;
}

ks_status ks_batch_smooth(ks_batch *b, const ks_io *io, int32_t want_cov, ks_status *statuses) {
    if (!b || !io) return KS_E_ARG;
    const bool cov = want_cov != 0;
    for (int i = 0; i < b->count; ++i) {
        const ks_desc &d = b->probs[i].d;
        if (!io[i].u_out || (cov && !io[i].cov_out)) return KS_E_ARG;
        if (d.k > 0 && (!io[i].F || !io[i].c || !io[i].K)) return KS_E_ARG;
        if (d.m > 0 && (!io[i].G || !io[i].o || !io[i].C)) return KS_E_ARG;
    }
    hipError_t e;
    const bool fresh = !(b->mode_cov == (int)cov && same_io(b->cached_io, io, b->count));
    if (fresh) {
        fill_tables(b, io, cov);
        if ((e = upload_tables(b)) != hipSuccess) return KS_E_HIP;
        b->cached_io.assign(io, io + b->count);
        b->mode_cov = (int)cov;
        if (b->have_exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->have_exec = false;
        }
        if (b->use_graph && b->cap) {
            hipGraph_t g;
            hipStream_t origin = b->stream;
            b->stream = b->cap;
            if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                enqueue_batch(b, cov);
                if (hipStreamEndCapture(b->cap, &g) == hipSuccess) {
                    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess) b->have_exec = true;
                    (void)hipGraphDestroy(g);
                }
            }
            b->stream = origin;
            (void)hipGetLastError();
        }
    }
    if (b->have_exec) {
        if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return KS_E_HIP;
    } else {
        enqueue_batch(b, cov);
    }
    if (hipGetLastError() != hipSuccess) return KS_E_HIP;
    e = hipMemcpyAsync(b->host_flags.data(), dptr<unsigned>(b, b->off_flags), sizeof(unsigned) * b->count,
                       hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return KS_E_HIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return KS_E_HIP;
    ks_status worst = KS_OK;
    for (int i = 0; i < b->count; ++i) {
        const unsigned f = b->host_flags[i];
        const ks_status s = (f & ks::FLAG_NOT_SPD) ? KS_E_NOT_SPD
                          : (f & ks::FLAG_NONFINITE) ? KS_E_NONFINITE
                          : (f & ks::FLAG_RANK) ? KS_E_RANK : KS_OK;
        if (statuses) statuses[i] = s;
        if (worst == KS_OK && s != KS_OK) worst = s;
    }
    return worst;
}

ks_status ks_batch_destroy(ks_batch *b) {
    if (!b) return KS_E_ARG;
    if (b->have_exec) (void)hipGraphExecDestroy(b->exec);
    b->side.destroy(b->stream);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return KS_OK;
}

}  // extern "C"


// ===================================================================== engine
//
// Continuous batching of served requests.  The engine sub-allocates one
// region per admitted request from a caller-owned workspace (first fit over a
// coalescing free list) and refuses a request whose region or launch-table
// share does not fit right now (KS_E_BUSY: the caller keeps it queued).  Each
// tick advances every in-flight request by one step of its schedule -- one
// forward level with its fold, the forward tail, the backward tail or one
// backward level -- with one launch per kernel class, step kind and variant
// over all requests at that kind of step, so requests admitted while others
// are deep in their recursion start level 0 in the same launches.  Every
// request follows exactly the schedule of a single plan, so its results are
// bitwise those of ks_smooth_cov (or ks_smooth) on it alone.

#include <map>
#include <set>

namespace {

struct EngReq {
    uint64_t ticket;
    BatchProblem pr;
    ks_io io;
    bool cov;
    int32_t slot;      // status word
    int phase;         // 0 forward levels, 1 forward tail, 2 backward tail, 3 backward levels
    int level;         // current level of phases 0 and 3
    bool fresh;        // status word not yet cleared
    size_t tab_need;   // bound on this request's share of a tick's tables
};

constexpr int32_t kEngSlots = 4096;

// A tick that was enqueued and may still run: its event, the requests whose
// last step it holds (retired once it completes), and the pinned copy of the
// status words it reads back.
struct EngTick {
    bool busy = false;
    uint64_t seq = 0;
    hipEvent_t ev = nullptr;
    unsigned *hflags = nullptr;  // pinned host memory, kEngSlots words
    std::vector<EngReq> finishing;
};

}  // namespace

struct ks_engine {
    char *ws;
    size_t region_bytes;   // [0, region_bytes): request regions
    size_t tab_off, tab_bytes;  // two table buffers of tab_bytes each (ticks alternate)
    unsigned *dflags;      // kEngSlots status words
    hipStream_t stream;
    std::map<size_t, size_t> free_list;  // offset -> bytes
    std::set<int32_t> free_slots;
    std::vector<EngReq> inflight;        // requests with steps still to launch
    std::vector<std::pair<uint64_t, ks_status>> retired;
    size_t tab_used;       // sum of tab_need over requests with steps still to launch
    uint64_t next_ticket, ticks;
    std::vector<char> staging;
    EngTick tick[2];       // the tick using table buffer b
    int next_buf;          // table buffer of the next tick
    SideStreams side;      // the launch groups of one tick are independent
};

namespace {

constexpr size_t kEngTabFixed = 8 * kAlign;  // per-array alignment of one tick's tables

bool eng_alloc(ks_engine *e, size_t bytes, size_t *off) {
    for (auto it = e->free_list.begin(); it != e->free_list.end(); ++it) {
        if (it->second < bytes) continue;
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        e->free_list.erase(it);
        if (rest) e->free_list[at] = rest;
        return true;
    }
    return false;
}

void eng_free(ks_engine *e, size_t off, size_t bytes) {
    auto it = e->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != e->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        e->free_list.erase(nx);
    }
    if (it != e->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            e->free_list.erase(it);
        }
    }
}

int fwd_variant(const BatchProblem &pr, int s) { return ks::level_variant(pr.kset, s, pr.l_switch, pr.lo.Nl[s]); }

int64_t fwd_blocks(const BatchProblem &pr, int l) {
    return (pr.lo.Nl[l] / 2 + pr.kset->upb_fwd - 1) / pr.kset->upb_fwd;
}

int64_t bwd_blocks(const BatchProblem &pr, int l, int mode) {
    const int upb = pr.kset->upb_bwd[mode];
    return ((pr.lo.Nl[l] + 1) / 2 + upb - 1) / upb;
}

// the request's arguments (as fill_tables builds them for a batch)
ks::FwdArgs eng_fwd_args(const ks_engine *e, const EngReq &r, int l) {
    const BatchProblem &pr = r.pr;
    const Layout &lo = pr.lo;
    char *base = e->ws + pr.ws_off;
    const int64_t n = pr.d.n, rrec = n * (3 * n + 1);
    ks::FwdArgs a{};
    a.k = pr.d.k;
    a.m = pr.d.m;
    a.K_diag = pr.d.K_layout == KS_COV_DIAG;
    a.C_diag = pr.d.C_layout == KS_COV_DIAG;
    a.H = r.io.H; a.F = r.io.F; a.c = r.io.c; a.K = r.io.K;
    a.G = r.io.G; a.o = r.io.o; a.C = r.io.C;
    a.flags = e->dflags + r.slot;
    if (l >= 0) {
        double *sys = reinterpret_cast<double *>(base + lo.off_sys);
        double *slots = reinterpret_cast<double *>(base + lo.off_slots);
        a.Nl = lo.Nl[l];
        a.units = lo.Nl[l] / 2;
        a.level = l;
        a.sys_in = l >= 1 ? sys + lo.sys_off[l] : nullptr;
        a.sys_out = sys + lo.sys_off[l + 1];
        a.rrows = reinterpret_cast<double *>(base + lo.off_rrows) + lo.rec_off[l] * rrec;
        a.slots = slots + 2 * lo.slot_off[l];
        a.fold_slot = a.slots + 2 * fwd_blocks(pr, l);
    }
    return a;
}

ks::FwdTailArgs eng_tail_args(const ks_engine *e, const EngReq &r) {
    const BatchProblem &pr = r.pr;
    const Layout &lo = pr.lo;
    char *base = e->ws + pr.ws_off;
    ks::FwdTailArgs ta{};
    ta.a = eng_fwd_args(e, r, -1);
    ta.l0 = pr.l0;
    ta.L = lo.L;
    ta.sys = reinterpret_cast<double *>(base + lo.off_sys);
    ta.rrows = reinterpret_cast<double *>(base + lo.off_rrows);
    ta.slots = reinterpret_cast<double *>(base + lo.off_slots);
    ta.nprev = lo.slot_off[pr.l0];
    ta.rank_tol = pr.rank_tol;
    for (int l = 0; l <= lo.L; ++l) {
        ta.sys_off[l] = lo.sys_off[l];
        ta.rec_off[l] = lo.rec_off[l];
        ta.Nl[l] = lo.Nl[l];
    }
    return ta;
}

ks::BwdArgs eng_bwd_args(const ks_engine *e, const EngReq &r) {
    const BatchProblem &pr = r.pr;
    const Layout &lo = pr.lo;
    char *base = e->ws + pr.ws_off;
    ks::BwdArgs bw{};
    bw.k = pr.d.k;
    bw.level = lo.L;
    bw.l_lo = pr.l1;
    bw.store_s = r.cov;
    bw.rrows_all = reinterpret_cast<double *>(base + lo.off_rrows);
    bw.u_in = r.io.u_out;
    bw.u_out = r.io.u_out;
    bw.cov = r.cov ? r.io.cov_out : nullptr;
    bw.spm = reinterpret_cast<double *>(base + lo.off_spm);
    bw.spm_first = lo.spm_first;
    for (int l = 0; l <= lo.L; ++l) {
        bw.rec_off[l] = lo.rec_off[l];
        bw.Nl[l] = lo.Nl[l];
    }
    return bw;
}

// next step after the one just run; false when the request is finished
bool eng_advance(EngReq &r) {
    const BatchProblem &pr = r.pr;
    const int top = std::min(pr.l1, pr.lo.L + 1);  // backward levels below run one per step
    switch (r.phase) {
    case 0:
        if (++r.level < pr.l0) return true;
        r.phase = 1;
        return true;
    case 1:
        if (pr.l1 <= pr.lo.L) { r.phase = 2; return true; }
        r.phase = 3;
        r.level = top - 1;
        return true;
    case 2:
        if (top == 0) return false;
        r.phase = 3;
        r.level = top - 1;
        return true;
    default:
        return --r.level >= 0;
    }
}

ks_status status_of(unsigned f) {
    return (f & ks::FLAG_NOT_SPD) ? KS_E_NOT_SPD
         : (f & ks::FLAG_NONFINITE) ? KS_E_NONFINITE
         : (f & ks::FLAG_RANK) ? KS_E_RANK : KS_OK;
}

// Retire the requests of completed ticks, oldest tick first: status from the
// tick's copy of the status words; region and status word free again.  With
// wait, blocks until every enqueued tick has completed.  Returns how many
// requests were retired, or -1 on a HIP error.
int32_t eng_reap(ks_engine *e, bool wait) {
    int32_t nfin = 0;
    while (true) {
        EngTick *T = nullptr;
        for (auto &t : e->tick)
            if (t.busy && (!T || t.seq < T->seq)) T = &t;
        if (!T) return nfin;
        if (wait) {
            if (hipEventSynchronize(T->ev) != hipSuccess) return -1;
        } else {
            const hipError_t q = hipEventQuery(T->ev);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();
                return nfin;
            }
            if (q != hipSuccess) return -1;
        }
        for (const EngReq &r : T->finishing) {
            e->retired.emplace_back(r.ticket, status_of(T->hflags[r.slot]));
            eng_free(e, r.pr.ws_off, align_up(r.pr.lo.total));
            e->free_slots.insert(r.slot);
            ++nfin;
        }
        T->finishing.clear();
        T->busy = false;
    }
}

size_t eng_finishing(const ks_engine *e) {
    return e->tick[0].finishing.size() + e->tick[1].finishing.size();
}

}  // namespace

extern "C" {

ks_status ks_engine_create(void *workspace, size_t ws_bytes, void *hip_stream, ks_engine **out) {
    if (!out) return KS_E_ARG;
    *out = nullptr;
    const size_t flags_bytes = align_up(sizeof(unsigned) * kEngSlots);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 || ws_bytes < ((size_t)1 << 20))
        return KS_E_WORKSPACE;
    ks_engine *e = new (std::nothrow) ks_engine;
    if (!e) return KS_E_ARG;
    e->ws = static_cast<char *>(workspace);
    e->stream = static_cast<hipStream_t>(hip_stream);
    // 1/16 of the workspace (at least 256 KiB) for two launch-table buffers,
    // the status words after them, the rest for request regions
    size_t tab = std::max<size_t>((size_t)256 << 10, ws_bytes / 16) / (2 * kAlign) * (2 * kAlign);
    e->region_bytes = (ws_bytes - tab - flags_bytes) / kAlign * kAlign;
    e->tab_off = e->region_bytes;
    e->tab_bytes = tab / 2;
    e->dflags = reinterpret_cast<unsigned *>(e->ws + e->tab_off + tab);
    e->next_buf = 0;
    e->free_list[0] = e->region_bytes;
    for (int32_t s = 0; s < kEngSlots; ++s) e->free_slots.insert(s);
    e->tab_used = kEngTabFixed;
    e->next_ticket = 1;
    e->ticks = 0;
    e->side.create();
    *out = e;
    return KS_OK;
}

ks_status ks_engine_submit(ks_engine *e, const ks_desc *desc, const ks_io *io, int32_t want_cov,
                           uint64_t *ticket) {
    if (!e || !desc || !io || !ticket || !valid_desc(desc)) return KS_E_ARG;
    EngReq r{};
    BatchProblem &pr = r.pr;
    pr.d = *desc;
    pr.kset = ks::find_kernels(desc->n, desc->m) ? tuned_kernels(*desc) : nullptr;
    if (!pr.kset || !make_layout(desc, pr.kset, &pr.lo)) return KS_E_ARG;
    if (!io->u_out || (want_cov && !io->cov_out)) return KS_E_ARG;
    if (desc->k > 0 && (!io->F || !io->c || !io->K)) return KS_E_ARG;
    if (desc->m > 0 && (!io->G || !io->o || !io->C)) return KS_E_ARG;
    // schedule, exactly as a single plan derives it
    const int mode = want_cov ? ks::BWD_BOTH : ks::BWD_Y;
    const Schedule sc = make_schedule(*desc, pr.kset, pr.lo, mode);
    pr.l_switch = sc.l_switch;
    pr.l0 = sc.l0;
    pr.l1 = sc.l1;
    pr.rank_tol = sc.rank_tol;
    // bound on the request's share of one tick's tables
    int64_t maxb = 1;
    for (int l = 0; l < pr.l0; ++l) maxb = std::max(maxb, fwd_blocks(pr, l));
    for (int l = 0; l < std::min(pr.l1, pr.lo.L + 1); ++l) maxb = std::max(maxb, bwd_blocks(pr, l, mode));
    r.tab_need = std::max({sizeof(ks::FwdArgs), sizeof(ks::FwdTailArgs), sizeof(ks::BwdArgs)})
               + (size_t)(maxb + 1) * (sizeof(int32_t) * 2 + sizeof(int64_t)) + sizeof(int32_t);
    const size_t region = align_up(pr.lo.total);
    if (region > e->region_bytes || kEngTabFixed + r.tab_need > e->tab_bytes) return KS_E_WORKSPACE;
    if (e->free_slots.empty() || e->tab_used + r.tab_need > e->tab_bytes) return KS_E_BUSY;
    size_t off;
    if (!eng_alloc(e, region, &off)) return KS_E_BUSY;
    pr.ws_off = off;
    r.io = *io;
    r.cov = want_cov != 0;
    r.slot = *e->free_slots.begin();
    e->free_slots.erase(e->free_slots.begin());
    r.phase = pr.l0 > 0 ? 0 : 1;
    r.level = 0;
    r.fresh = true;
    r.ticket = e->next_ticket++;
    e->tab_used += r.tab_need;
    *ticket = r.ticket;
    e->inflight.push_back(r);
    return KS_OK;
}

ks_status ks_engine_step(ks_engine *e, int32_t *finished) {
    if (!e) return KS_E_ARG;
    if (finished) *finished = 0;
    int32_t nfin = eng_reap(e, false);
    if (nfin < 0) return KS_E_HIP;
    if (e->inflight.empty()) {
        if (finished) *finished = nfin;
        return KS_OK;
    }
    if (!e->tick[0].ev) {  // first tick: events and pinned status copies
        for (auto &t : e->tick) {
            if (hipEventCreateWithFlags(&t.ev, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc(reinterpret_cast<void **>(&t.hflags), sizeof(unsigned) * kEngSlots,
                              hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                for (auto &u : e->tick) {
                    if (u.ev) (void)hipEventDestroy(u.ev);
                    if (u.hflags) (void)hipHostFree(u.hflags);
                    u.ev = nullptr;
                    u.hflags = nullptr;
                }
                return KS_E_HIP;
            }
        }
    }
    EngTick &T = e->tick[e->next_buf];
    if (T.busy) {  // both table buffers in use: wait for the older tick (this one)
        if (hipEventSynchronize(T.ev) != hipSuccess) return KS_E_HIP;
        const int32_t more = eng_reap(e, false);
        if (more < 0) return KS_E_HIP;
        nfin += more;
    }
    const size_t R = e->inflight.size();
    std::vector<ks::FwdArgs> ftab;
    std::vector<ks::FwdTailArgs> ttab;
    std::vector<ks::BwdArgs> btab;
    std::vector<int32_t> item, level, clear, idx(R, -1);
    std::vector<int64_t> blk;
    std::vector<BLaunch> launches;
    std::vector<const ks::KernelSet *> classes;
    for (size_t q = 0; q < R; ++q) {
        EngReq &r = e->inflight[q];
        if (std::find(classes.begin(), classes.end(), r.pr.kset) == classes.end()) classes.push_back(r.pr.kset);
        if (r.fresh) clear.push_back(r.slot);
        if (r.phase == 0) { idx[q] = (int32_t)ftab.size(); ftab.push_back(eng_fwd_args(e, r, r.level)); }
        else if (r.phase == 1) { idx[q] = (int32_t)ttab.size(); ttab.push_back(eng_tail_args(e, r)); }
        else { idx[q] = (int32_t)btab.size(); btab.push_back(eng_bwd_args(e, r)); }
    }
    auto add = [&](int32_t it, int64_t b, int32_t lv) {
        item.push_back(it);
        blk.push_back(b);
        level.push_back(lv);
    };
    // launch list; a request's fold follows its level's launch
    for (auto *cls : classes) {
        for (int raw = 1; raw >= 0; --raw)
            for (int v = 0; v < ks::kFwdVariants; ++v) {
                BLaunch fl{BLaunch::FWD, cls, v, raw == 1, (int64_t)item.size(), 0};
                std::vector<size_t> folds;
                for (size_t q = 0; q < R; ++q) {
                    const EngReq &r = e->inflight[q];
                    if (r.pr.kset != cls || r.phase != 0 || (r.level == 0) != (raw == 1)) continue;
                    if (fwd_variant(r.pr, r.level) != v) continue;
                    const int64_t nb = fwd_blocks(r.pr, r.level);
                    for (int64_t k = 0; k < nb; ++k) add(idx[q], k, r.level);
                    fl.blocks += nb;
                    if (r.pr.lo.Nl[r.level] & 1) folds.push_back(q);
                }
                if (fl.blocks) launches.push_back(fl);
                BLaunch fo{BLaunch::FOLD, cls, v, raw == 1, (int64_t)item.size(), (int64_t)folds.size()};
                for (size_t q : folds) add(idx[q], 0, e->inflight[q].level);
                if (fo.blocks) launches.push_back(fo);
            }
        for (int raw = 1; raw >= 0; --raw) {
            BLaunch t{BLaunch::FTAIL, cls, 0, raw == 1, (int64_t)item.size(), 0};
            for (size_t q = 0; q < R; ++q) {
                const EngReq &r = e->inflight[q];
                if (r.pr.kset != cls || r.phase != 1 || (r.pr.l0 == 0) != (raw == 1)) continue;
                add(idx[q], 0, r.pr.l0);
                t.blocks += 1;
            }
            if (t.blocks) launches.push_back(t);
        }
        for (int mode : {(int)ks::BWD_Y, (int)ks::BWD_BOTH}) {
            BLaunch t{BLaunch::BTAIL, cls, mode, false, (int64_t)item.size(), 0};
            for (size_t q = 0; q < R; ++q) {
                const EngReq &r = e->inflight[q];
                if (r.pr.kset != cls || r.phase != 2 || (r.cov ? ks::BWD_BOTH : ks::BWD_Y) != mode) continue;
                add(idx[q], 0, r.pr.lo.L);
                t.blocks += 1;
            }
            if (t.blocks) launches.push_back(t);
            for (int tr = 0; tr < 2; ++tr) {
                // variant = mode * 2 + record type
                BLaunch bl{BLaunch::BWD, cls, mode * 2 + tr, false, (int64_t)item.size(), 0};
                for (size_t q = 0; q < R; ++q) {
                    const EngReq &r = e->inflight[q];
                    if (r.pr.kset != cls || r.phase != 3 || (r.cov ? ks::BWD_BOTH : ks::BWD_Y) != mode) continue;
                    if ((r.level < r.pr.l_switch ? 1 : 0) != tr) continue;
                    const int64_t nb = bwd_blocks(r.pr, r.level, mode);
                    for (int64_t k = 0; k < nb; ++k) add(idx[q], k, r.level);
                    bl.blocks += nb;
                }
                if (bl.blocks) launches.push_back(bl);
            }
        }
    }
    // one upload: argument tables, block maps, status words to clear
    size_t off = 0;
    const size_t o_f = off; off += tab_bytes<ks::FwdArgs>(ftab.size());
    const size_t o_t = off; off += tab_bytes<ks::FwdTailArgs>(ttab.size());
    const size_t o_b = off; off += tab_bytes<ks::BwdArgs>(btab.size());
    const size_t o_i = off; off += tab_bytes<int32_t>(item.size());
    const size_t o_k = off; off += tab_bytes<int64_t>(blk.size());
    const size_t o_l = off; off += tab_bytes<int32_t>(level.size());
    const size_t o_c = off; off += tab_bytes<int32_t>(clear.size());
    if (off > e->tab_bytes) return KS_E_WORKSPACE;  // excluded by admission
    e->staging.resize(off);
    char *st = e->staging.data();
    auto put = [&](size_t o, const void *src, size_t bytes) { if (bytes) std::memcpy(st + o, src, bytes); };
    put(o_f, ftab.data(), sizeof(ks::FwdArgs) * ftab.size());
    put(o_t, ttab.data(), sizeof(ks::FwdTailArgs) * ttab.size());
    put(o_b, btab.data(), sizeof(ks::BwdArgs) * btab.size());
    put(o_i, item.data(), sizeof(int32_t) * item.size());
    put(o_k, blk.data(), sizeof(int64_t) * blk.size());
    put(o_l, level.data(), sizeof(int32_t) * level.size());
    put(o_c, clear.data(), sizeof(int32_t) * clear.size());
    char *dt = e->ws + e->tab_off + (size_t)e->next_buf * e->tab_bytes;
    if (hipMemcpyAsync(dt, st, off, hipMemcpyHostToDevice, e->stream) != hipSuccess) return KS_E_HIP;
    if (!clear.empty())
        ks::launch_clear_flags_list(e->dflags, reinterpret_cast<const int32_t *>(dt + o_c), (int32_t)clear.size(),
                                    e->stream);
    const ks::FwdArgs *ft = reinterpret_cast<const ks::FwdArgs *>(dt + o_f);
    const ks::FwdTailArgs *tt = reinterpret_cast<const ks::FwdTailArgs *>(dt + o_t);
    const ks::BwdArgs *bt = reinterpret_cast<const ks::BwdArgs *>(dt + o_b);
    const int32_t *mi = reinterpret_cast<const int32_t *>(dt + o_i);
    const int64_t *mb = reinterpret_cast<const int64_t *>(dt + o_k);
    const int32_t *ml = reinterpret_cast<const int32_t *>(dt + o_l);
    // every launch of a tick covers its own requests, so the launches run
    // concurrently on the side streams, round robin; a fold stays on the
    // stream of the level launch it follows
    const bool fork = e->side.n > 0 && launches.size() > 1;
    if (fork) e->side.fork(e->stream);
    int group = -1;
    for (const BLaunch &L : launches) {
        const ks::BlockMap bm{mi + L.map0, mb + L.map0, ml + L.map0};
        if (L.kind != BLaunch::FOLD) ++group;
        hipStream_t sm = fork ? e->side.s[group % e->side.n] : e->stream;
        switch (L.kind) {
        case BLaunch::FWD:
            if (L.raw) L.kset->fwd_raw_b[L.variant == ks::FV_F32](ft, bm, L.blocks, sm);
            else L.kset->fwd_b[L.variant](ft, bm, L.blocks, sm);
            break;
        case BLaunch::FOLD:
            if (L.raw) L.kset->fold_raw_b[L.variant == ks::FV_F32](ft, bm, L.blocks, sm);
            else L.kset->fold_b[L.variant](ft, bm, L.blocks, sm);
            break;
        case BLaunch::FTAIL:
            (L.raw ? L.kset->fwd_tail_raw_b : L.kset->fwd_tail_b)(tt, bm, L.blocks, sm);
            break;
        case BLaunch::BTAIL:
            L.kset->bwd_tail_b[L.variant](bt, bm, L.blocks, sm);
            break;
        case BLaunch::BWD:
            L.kset->bwd_b[L.variant / 2][L.variant % 2](bt, bm, L.blocks, sm);
            break;
        }
    }
    if (fork) e->side.join(e->stream);
    if (hipGetLastError() != hipSuccess) return KS_E_HIP;
    // advance; the requests whose last step this tick holds wait (in the
    // tick) for its completion, with a copy of the status words
    int32_t hi = -1;
    std::vector<EngReq> keep;
    keep.reserve(R);
    for (size_t q = 0; q < R; ++q) {
        EngReq &r = e->inflight[q];
        r.fresh = false;
        if (eng_advance(r)) {
            keep.push_back(r);
            continue;
        }
        hi = std::max(hi, r.slot);
        e->tab_used -= r.tab_need;  // no later tick holds it
        T.finishing.push_back(r);
    }
    e->inflight.swap(keep);
    if (hi >= 0 && hipMemcpyAsync(T.hflags, e->dflags, sizeof(unsigned) * (hi + 1), hipMemcpyDeviceToHost,
                                  e->stream) != hipSuccess)
        return KS_E_HIP;
    if (hipEventRecord(T.ev, e->stream) != hipSuccess) return KS_E_HIP;
    T.busy = true;
    T.seq = ++e->ticks;
    e->next_buf ^= 1;
    if (finished) *finished = nfin;
    return KS_OK;
}

ks_status ks_engine_wait(ks_engine *e, int32_t *finished) {
    if (!e) return KS_E_ARG;
    const int32_t nfin = eng_reap(e, true);
    if (finished) *finished = nfin < 0 ? 0 : nfin;
    return nfin < 0 ? KS_E_HIP : KS_OK;
}

ks_status ks_engine_retired(ks_engine *e, int32_t capacity, uint64_t *tickets, ks_status *statuses,
                            int32_t *count) {
    if (!e || !count || capacity < 0 || (capacity > 0 && (!tickets || !statuses))) return KS_E_ARG;
    if (eng_reap(e, false) < 0) return KS_E_HIP;
    const int32_t c = (int32_t)std::min<size_t>((size_t)capacity, e->retired.size());
    for (int32_t i = 0; i < c; ++i) {
        tickets[i] = e->retired[i].first;
        statuses[i] = e->retired[i].second;
    }
    e->retired.erase(e->retired.begin(), e->retired.begin() + c);
    *count = c;
    return KS_OK;
}

ks_status ks_engine_poll(ks_engine *e, uint64_t ticket, ks_status *result) {
    if (!e || !result) return KS_E_ARG;
    if (eng_reap(e, false) < 0) return KS_E_HIP;
    for (size_t i = 0; i < e->retired.size(); ++i) {
        if (e->retired[i].first != ticket) continue;
        *result = e->retired[i].second;
        e->retired.erase(e->retired.begin() + i);
        return KS_OK;
    }
    for (const EngReq &r : e->inflight)
        if (r.ticket == ticket) return KS_E_BUSY;
    for (const auto &t : e->tick)
        for (const EngReq &r : t.finishing)
            if (r.ticket == ticket) return KS_E_BUSY;
    return KS_E_ARG;
}

ks_status ks_engine_query(const ks_engine *e, ks_engine_stats *out) {
    if (!e || !out) return KS_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->inflight = (int64_t)(e->inflight.size() + eng_finishing(e));
    out->retired_pending = (int64_t)e->retired.size();
    out->ticks = (int64_t)e->ticks;
    out->ticks_pending = (int64_t)e->tick[0].busy + (int64_t)e->tick[1].busy;
    out->region_bytes = e->region_bytes;
    for (auto &f : e->free_list) {
        out->free_bytes += f.second;
        out->largest_free = std::max(out->largest_free, f.second);
    }
    return KS_OK;
}

ks_status ks_engine_destroy(ks_engine *e) {
    if (!e) return KS_E_ARG;
    if (e->tick[0].ev) (void)hipStreamSynchronize(e->stream);  // no tick reads the tables or pinned words
    e->side.destroy(e->stream);
    for (auto &t : e->tick) {
        if (t.ev) (void)hipEventDestroy(t.ev);
        if (t.hflags) (void)hipHostFree(t.hflags);
    }
    delete e;
    return KS_OK;
}

}  // extern "C"
