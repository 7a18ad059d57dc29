// ks_static.hip -- ks_smooth_cov_static: the states + covariances pass of
// ks_smooth_cov with the plan's working data in a static device array, for
// callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ks.h"
#include "ks_internal.h"

namespace {

// Working data of one pass (R rows, reduced systems, stored S blocks, per-block
// statistics, status word).  One copy per GPU, held until the process ends.
// Host code never passes this name to a kernel or a copy: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[KS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device (null until looked up)

// address of the current device's array, looked up once per device with that
// device current; null on failure
void *scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" ks_status ks_smooth_cov_static(const ks_desc *desc, const double *H, const double *F,
                                          const double *c, const double *K, const double *G,
                                          const double *o, const double *C, double *u_out,
                                          double *cov_out, void *hip_stream) {
    const size_t need = ks_workspace_bytes(desc);  // 0 for a null, invalid or unsupported desc
    if (need == 0) return KS_E_ARG;
    if (need > KS_STATIC_SCRATCH_BYTES) return KS_E_WORKSPACE;  // checked before any HIP call
    if (!u_out || !cov_out) return KS_E_ARG;
    void *ws = scratch_ptr();
    if (!ws) return KS_E_HIP;
    return ks::smooth_cov_on(desc, ws, KS_STATIC_SCRATCH_BYTES, static_cast<hipStream_t>(hip_stream), H, F, c,
                             K, G, o, C, u_out, cov_out);
}
