// ks_internal.h -- interface between the libks host runtime and its gfx950
// kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ks.h"

namespace ks {

// status bits written by kernels into the workspace's flag word
enum : unsigned {
    FLAG_NOT_SPD = 1u,
    FLAG_NONFINITE = 2u,
    FLAG_RANK = 4u,
};

constexpr int kBlock = 256;      // threads per workgroup of the per-level kernels
constexpr int kTailBlock = 512;  // threads of the single-workgroup forward tail
constexpr int kMaxLevels = 64;

// Arguments of one forward level (odd-even elimination of the even block
// columns of the level-l system, Section III).
// a plan's status words (64 bytes): [0] the flags, [kFoldCounter] the fold
// arrival counter; all cleared at the start of every pass
constexpr int kStatusWords = 16;
constexpr int kFoldCounter = 8;

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
    double *fold_slot;  // [min, max] of the level's fold kernel
    unsigned *flags;
    // the fold split across two workgroups of a level launch (single plans):
    // Z rows of the last column (n x (n+1) of the level's record type) and
    // the arrival counter of the two workgroups (zero between launches)
    double *fold_z;
    unsigned *fold_cnt;
    // first column (observation step, reduced-system record) and first
    // evolution entry that the input pointers above start at: 0 for the
    // caller's arrays; nonzero when a kernel reads a staged copy of a slice
    int64_t col0, ent0;
};

// Forward levels l0..L in one workgroup, then the rank test.
struct FwdTailArgs {
    FwdArgs a;        // shared fields (k, m, layouts, raw inputs, flags)
    int32_t l0, L;
    double *sys;      // reduced-system segment
    double *rrows;    // R-row record 0
    double rank_tol;  // KS_E_RANK when min |R_pp| <= rank_tol * max |R_pp|
    const double *slots;  // per-block slots of the launches before the tail
    int64_t nprev;
    int64_t sys_off[kMaxLevels];
    int64_t rec_off[kMaxLevels];
    int64_t Nl[kMaxLevels];
};

// A group of consecutive forward levels l_first .. l_first + nlev - 1 in one
// launch (subtree fusion): workgroup w owns the level-l_first units
// [w U, (w+1) U) (the last workgroup up to the level's end) and every unit
// they feed at the later levels of the group.  U is a multiple of 2^(nlev-1).
struct FwdMultiArgs {
    FwdArgs a;        // shared fields (k, m, layouts, raw inputs, flags)
    int32_t l_first, nlev;
    int64_t U;        // level-l_first units per workgroup
    int64_t groups;   // workgroups
    double *sys;      // reduced-system segment
    double *rrows;    // R-row record 0
    double *slots;    // one [min |R_pp|, max |R_pp|] pair per workgroup, then
    int64_t slot_pairs;   // ... neutral pairs up to here (the per-level slots the group replaces)
    int64_t sys_off[kMaxLevels];
    int64_t rec_off[kMaxLevels];
    int64_t Nl[kMaxLevels];
};

// Arguments of a backward level// Arguments of a backward level (back-substitution and/or Algorithm 2); the
// tail kernel runs levels `level` down to `l_lo`.
struct BwdArgs {
    int64_t k;
    int32_t level;
    int32_t l_lo;
    int32_t store_s;  // write S_{i,I} blocks for lower levels
    const double *rrows_all;  // record 0
    const double *u_in;       // u_out (neighbour states)
    double *u_out;
    double *cov;              // cov_out (neighbour blocks are read from it too)
    double *spm;              // S_{i,i-2^l}, S_{i,i+2^l} of records >= spm_first
    double *lag1;             // level 0 writes S_{i,i+1} = cov(u_i, u_{i+1}) here when non-null
    int64_t spm_first;
    int64_t rec_off[kMaxLevels];
    int64_t Nl[kMaxLevels];
};

enum BwdMode { BWD_Y = 0, BWD_COV = 1, BWD_BOTH = 2 };

// precision variant of a forward launch: compute/storage type and the type of
// the records it reads
enum FwdVariant { FV_F64 = 0, FV_F32 = 1, FV_F64_FROM_F32 = 2, FV_F64_NARROW = 3, kFwdVariants = 4 };

using FwdFn = void (*)(const FwdArgs &, hipStream_t);
using BwdFn = void (*)(const BwdArgs &, hipStream_t);
using TailFn = void (*)(const FwdTailArgs &, hipStream_t);
using FwdMFn = void (*)(const FwdMultiArgs &, hipStream_t);

// Batched launches: workgroup b of a launch takes its arguments from table
// entry item[b]; blk[b] is its block (or record-pass) index within that
// problem's level and level[b] the level (backward launches).
struct BlockMap {
    const int32_t *item;
    const int64_t *blk;
    const int32_t *level;
};
using FwdBFn = void (*)(const FwdArgs *, BlockMap, int64_t blocks, hipStream_t);
using BwdBFn = void (*)(const BwdArgs *, BlockMap, int64_t blocks, hipStream_t);
using TailBFn = void (*)(const FwdTailArgs *, BlockMap, int64_t blocks, hipStream_t);

// kernels launched by the runtime for state dimension n, observation class mm
struct KernelSet {
    int n, mm;
    FwdFn fwd_raw[2];       // level 0 from the FP64 inputs: [FP64 | FP32]
    FwdFn fwd[kFwdVariants];  // levels >= 1, indexed by FwdVariant
    FwdFn fold_raw[2];      // last column of an odd level
    FwdFn fold[kFwdVariants];
    TailFn fwd_tail_raw;    // single-workgroup tail starting at level 0 (FP64)
    TailFn fwd_tail;        // tail starting above level 0 (FP64 records in and out)
    BwdFn bwd[3][2];        // [BwdMode][records FP64 | FP32]; arithmetic in FP64
    BwdFn bwd_tail[3];      // FP64 records
    // the same kernels driven by work tables (one launch for many problems)
    FwdBFn fwd_raw_b[2];
    FwdBFn fwd_b[kFwdVariants];
    FwdBFn fold_raw_b[2];
    FwdBFn fold_b[kFwdVariants];
    TailBFn fwd_tail_raw_b;
    TailBFn fwd_tail_b;
    BwdBFn bwd_b[3][2];
    BwdBFn bwd_tail_b[3];
    int upb_fwd;            // units per workgroup, per-level forward kernel
    int upb_fwd_tail;       // units per pass of the forward tail
    int upb_bwd[3];
    int upb_bwd_tail[3];
    // levels >= 1 with the odd level's fold done by the level kernel's last
    // unit (no separate fold launch); null where the family has none
    FwdFn fwd_fold[kFwdVariants];
    // groups of consecutive levels in one launch (subtree fusion), null where
    // the family has none: forward groups starting at level 0 ([FP64 | FP32])
    // and above it (indexed by the FwdVariant of the group's first level);
    // backward groups (BwdArgs: levels `level` down to `l_lo`, workgroup c owns
    // the records of columns i with c 2^(level+1) < i+1 < (c+1) 2^(level+1)),
    // [BwdMode][records FP64 | FP32]
    FwdMFn fwd_multi_raw[2];
    FwdMFn fwd_multi[kFwdVariants];
    BwdFn bwd_multi[3][2];
    int upb_multi;    // units per pass of a forward group workgroup
    int rpp_multi;    // records per pass of a backward group workgroup
    // which compiled variant of the (n, observation class) this set is: its
    // forward half (fv) and backward half (bv); 0 = the default of n
    int fv, bv;
    // level 0 of an odd-N_0 problem with the last column folded in by the
    // level kernel ([FP64 | FP32]); null where the family has none
    FwdFn fwd_fold_raw[2];
    // nonzero: the level-0 forward whitens diagonal covariances only, so
    // problems with a dense covariance take forward variant 0 instead
    int raw_diag_only;
    // nonzero: FP64 levels >= 1 with fewer units than this run the kernels
    // of FV_F64_NARROW (a family whose units finish sooner, for levels too
    // narrow to fill the device)
    int narrow_units;
};

// The forward variant of level l: FP32 below the FP32-form switch l_switch,
// FP64 reading FP32 records at it, FP64 above; FP64 levels >= 1 narrower
// than the set's narrow_units take FV_F64_NARROW.  The same for a plan, a
// batch and the engine, so a problem's kernels never depend on its company.
inline int level_variant(const KernelSet *k, int l, int l_switch, int64_t Nl) {
    const int v = l < l_switch ? FV_F32 : (l == l_switch && l > 0 ? FV_F64_FROM_F32 : FV_F64);
    if (v == FV_F64 && l >= 1 && k->narrow_units > 0 && Nl / 2 < k->narrow_units) return FV_F64_NARROW;
    return v;
}

struct KernelSetList {
    const KernelSet *sets;
    int64_t count;
};

// nullptr when (n, m) has no instantiation (the default variants)
const KernelSet *find_kernels(int n, int m);
// the set of (n, m) with forward variant fv and backward variant bv (a
// composed set with a stable address), or nullptr when either variant does
// not exist
const KernelSet *find_kernels(int n, int m, int fv, int bv);
// number of forward / backward variants compiled for (n, m) (0 if none)
int kernel_variants(int n, int m, bool backward);

// One states + covariances pass (ks_smooth_cov's kernels and schedule) on a
// workspace the caller provides, without a plan object kept or any stream,
// event or graph created; synchronizes on the stream.  Validates everything
// ks_create and ks_smooth_cov validate.
ks_status smooth_cov_on(const ks_desc *desc, void *workspace, size_t ws_bytes, hipStream_t stream,
                        const double *H, const double *F, const double *c, const double *K,
                        const double *G, const double *o, const double *C, double *u_out,
                        double *cov_out);

void launch_clear_flags(unsigned *flags, hipStream_t s);
void launch_clear_flags_n(unsigned *flags, int32_t count, hipStream_t s);
// flags[idx[i]] = 0 for i < count (idx in device memory)
void launch_clear_flags_list(unsigned *flags, const int32_t *idx, int32_t count, hipStream_t s);

}  // namespace ks
