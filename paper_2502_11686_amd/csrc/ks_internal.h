// ks_internal.h -- interface between the libks host runtime and its gfx950
// kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ks {

// status bits written by kernels into the workspace's flag word
enum : unsigned {
    FLAG_NOT_SPD = 1u,
    FLAG_NONFINITE = 2u,
    FLAG_RANK = 4u,
};

constexpr int kBlock = 256;   // threads per workgroup for every level kernel
constexpr int kMaxLevels = 64;

// Arguments of one forward level (odd-even elimination of the even block
// columns of the level-l system, Section III).
struct FwdArgs {
    int64_t k;        // evolution steps of the problem
    int64_t Nl;       // block columns in this level's system
    int64_t units;    // units launched (one per even column pair)
    int32_t level;
    int32_t m;        // observation rows (level 0 only)
    int32_t K_diag, C_diag;
    // raw inputs (level 0)
    const double *H, *F, *c, *K, *G, *o, *C;
    // reduced systems (levels >= 1 read sys_in; every level < L writes sys_out)
    const double *sys_in;
    double *sys_out;
    double *rrows;    // first R-row record of this level
    double *slots;    // per-block [min |R_pp|, max |R_pp|]
    unsigned *flags;
};

// Arguments of one backward level (back-substitution and/or Algorithm 2).
struct BwdArgs {
    int64_t k;
    int64_t units;    // R-row records at this level
    int32_t level;
    int32_t store_s;  // write S_{i,I} blocks for lower levels
    const double *rrows_all;  // record 0
    const double *u_in;       // u_out (neighbour states)
    double *u_out;
    double *cov;              // cov_out (neighbour blocks are read from it too)
    double *spm;              // S_{i,i-2^l}, S_{i,i+2^l} of records >= spm_first
    int64_t spm_first;
    int64_t rec_off[kMaxLevels];
};

// kernels launched by the runtime for state dimension n, observation class mm
struct KernelSet {
    int n, mm;
    void (*fwd_raw)(const FwdArgs &, hipStream_t);
    void (*fwd)(const FwdArgs &, hipStream_t);
    void (*base_raw)(const FwdArgs &, hipStream_t);
    void (*base)(const FwdArgs &, hipStream_t);
    void (*bwd_y)(const BwdArgs &, hipStream_t);
    void (*bwd_cov)(const BwdArgs &, hipStream_t);
    void (*bwd_both)(const BwdArgs &, hipStream_t);
    int units_per_block_fwd;
    int units_per_block_bwd;
};

// nullptr when (n, m) has no instantiation
const KernelSet *find_kernels(int n, int m);

void launch_clear_flags(unsigned *flags, hipStream_t s);
void launch_status(const double *slots, int64_t nslots, unsigned *flags, hipStream_t s);

}  // namespace ks
