// ks_dispatch.hip -- registry of the instantiated kernel sets and the small
// status kernel.
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "ks_internal.h"

namespace ks {

const KernelSetList &list_n1_3();
const KernelSetList &list_n4();
const KernelSetList &list_n5();
const KernelSetList &list_n6();
const KernelSetList &list_n8();
const KernelSetList &list_n12();
const KernelSetList &list_n16();
const KernelSetList &list_blk_n24();
const KernelSetList &list_blk_n32();
const KernelSetList &list_blk_n48();

static const KernelSetList &list_at(int i) {
    using F = const KernelSetList &(*)();
    static const F fns[] = {&list_n1_3, &list_n4, &list_n5, &list_n6, &list_n8, &list_n12, &list_n16,
                              &list_blk_n24, &list_blk_n32, &list_blk_n48};
    return fns[i]();
}
static constexpr int kNumLists = 10;

// the entry of (n, observation class mm) with variants (fv, bv), or nullptr
static const KernelSet *entry(int n, int mm, int fv, int bv) {
    for (int li = 0; li < kNumLists; ++li) {
        const KernelSetList &L = list_at(li);
        for (int64_t i = 0; i < L.count; ++i) {
            const KernelSet &s = L.sets[i];
            if (s.n == n && s.mm == mm && s.fv == fv && s.bv == bv) return &s;
        }
    }
    return nullptr;
}

const KernelSet *find_kernels(int n, int m) {
    const KernelSet *best = nullptr;
    for (int li = 0; li < kNumLists; ++li) {
        const KernelSetList &L = list_at(li);
        for (int64_t i = 0; i < L.count; ++i) {
            const KernelSet &s = L.sets[i];
            if (s.n != n || s.mm < (m > 0 ? m : 1) || s.fv != 0 || s.bv != 0) continue;
            if (!best || s.mm < best->mm) best = &s;
        }
    }
    return best;
}

int kernel_variants(int n, int m, bool backward) {
    const KernelSet *d = find_kernels(n, m);
    if (!d) return 0;
    int count = 0;
    while (backward ? entry(n, d->mm, 0, count) : entry(n, d->mm, count, 0)) ++count;
    return count;
}

// The forward half of one set and the backward half of another: the
// compositions made so far live here (stable addresses: batches and the
// engine group launches by kernel-set pointer).
static std::mutex g_compose_mu;
static std::map<std::tuple<int, int, int, int>, KernelSet> g_composed;

const KernelSet *find_kernels(int n, int m, int fv, int bv) {
    const KernelSet *d = find_kernels(n, m);
    if (!d) return nullptr;
    if (fv == 0 && bv == 0) return d;
    const KernelSet *f = entry(n, d->mm, fv, 0), *b = entry(n, d->mm, 0, bv);
    if (!f || !b) return nullptr;
    if (fv == 0) return b;  // a backward variant's set carries the default forward
    // a forward variant's set need not carry the default backward (n = 4..12:
    // the unstaged level-0 set keeps the wavefront family's backward, the
    // default is the MFMA one), so the backward half always comes from b
    std::lock_guard<std::mutex> lock(g_compose_mu);
    auto key = std::make_tuple(n, d->mm, fv, bv);
    auto it = g_composed.find(key);
    if (it != g_composed.end()) return &it->second;
    KernelSet s = *b;  // backward half, forward half from f
    std::memcpy(s.fwd_raw, f->fwd_raw, sizeof(s.fwd_raw));
    std::memcpy(s.fwd, f->fwd, sizeof(s.fwd));
    std::memcpy(s.fold_raw, f->fold_raw, sizeof(s.fold_raw));
    std::memcpy(s.fold, f->fold, sizeof(s.fold));
    s.fwd_tail_raw = f->fwd_tail_raw;
    s.fwd_tail = f->fwd_tail;
    std::memcpy(s.fwd_raw_b, f->fwd_raw_b, sizeof(s.fwd_raw_b));
    std::memcpy(s.fwd_b, f->fwd_b, sizeof(s.fwd_b));
    std::memcpy(s.fold_raw_b, f->fold_raw_b, sizeof(s.fold_raw_b));
    std::memcpy(s.fold_b, f->fold_b, sizeof(s.fold_b));
    s.fwd_tail_raw_b = f->fwd_tail_raw_b;
    s.fwd_tail_b = f->fwd_tail_b;
    s.upb_fwd = f->upb_fwd;
    s.upb_fwd_tail = f->upb_fwd_tail;
    std::memcpy(s.fwd_fold, f->fwd_fold, sizeof(s.fwd_fold));
    std::memcpy(s.fwd_fold_raw, f->fwd_fold_raw, sizeof(s.fwd_fold_raw));
    s.raw_diag_only = f->raw_diag_only;
    s.narrow_units = f->narrow_units;
    std::memcpy(s.fwd_multi_raw, f->fwd_multi_raw, sizeof(s.fwd_multi_raw));
    std::memcpy(s.fwd_multi, f->fwd_multi, sizeof(s.fwd_multi));
    s.upb_multi = f->upb_multi;
    s.fv = fv;
    s.bv = bv;
    return &g_composed.emplace(key, s).first->second;
}

__global__ void k_clear_flags(unsigned *flags) {
    if (threadIdx.x < kStatusWords) flags[threadIdx.x] = 0u;
}

void launch_clear_flags(unsigned *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, flags);
}

__global__ void k_clear_flags_n(unsigned *flags, int32_t count) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) flags[i] = 0u;
}

void launch_clear_flags_n(unsigned *flags, int32_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flags_n, dim3((count + 255) / 256), dim3(256), 0, s, flags, count);
}

__global__ void k_clear_flags_list(unsigned *flags, const int32_t *idx, int32_t count) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) flags[idx[i]] = 0u;
}

void launch_clear_flags_list(unsigned *flags, const int32_t *idx, int32_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flags_list, dim3((count + 255) / 256), dim3(256), 0, s, flags, idx, count);
}

}  // namespace ks
