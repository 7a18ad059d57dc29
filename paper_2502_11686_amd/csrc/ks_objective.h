// ks_objective.h -- the least-squares objective kernel (device side of
// ks_objective).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ks {

// Per-block partial sums of the objective; one more slot holds the total.
constexpr int kObjBlocks = 2048;

struct ObjArgs {
    int64_t k;
    int32_t n, m;
    bool K_diag, C_diag;
    const double *H, *F, *c, *K, *G, *o, *C;
    const double *u;   // [k+1][n], or NULL for u = 0
    double *terms;     // [k+1] per-step terms, or NULL
    double *partial;   // kObjBlocks + 1 doubles of workspace
    unsigned *flags;   // FLAG_NOT_SPD when some K_i or C_i is not positive definite
};

// Enqueues the objective kernel and the reduction of its partial sums; the
// total lands in partial[objective_blocks(k)].
void launch_objective(const ObjArgs &a, hipStream_t s);
int objective_blocks(int64_t k);

}  // namespace ks
