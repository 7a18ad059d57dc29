// ks_dispatch.hip -- registry of the instantiated kernel sets and the small
// status kernel.
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

const KernelSet *find_kernels(int n, int m) {
    const KernelSet *best = nullptr;
    for (int li = 0; li < kNumLists; ++li) {
        const KernelSetList &L = list_at(li);
        for (int64_t i = 0; i < L.count; ++i) {
            const KernelSet &s = L.sets[i];
            if (s.n != n || s.mm < (m > 0 ? m : 1)) continue;
            if (!best || s.mm < best->mm) best = &s;
        }
    }
    return best;
}

__global__ void k_clear_flags(unsigned *flags) {
    if (threadIdx.x == 0) flags[0] = 0u;
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
