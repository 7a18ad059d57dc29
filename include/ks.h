/*
 * ks.h -- C ABI of libks, the MI355X (gfx950) odd-even Kalman smoother.
 *
 * Method: Gargir & Toledo, "Parallel-in-Time Kalman Smoothing Using Orthogonal
 * Transformations" (IPDPS 2025).  The smoother solves the generalized linear
 * least-squares problem of Section II-A,
 *
 *     u_hat = argmin_u || U (A u - b) ||_2^2,     U^T U = cov(e)^{-1},
 *
 * for the evolution equations H_i u_i = F_i u_{i-1} + c_i + eps_i (i = 1..k,
 * cov(eps_i) = K_i) and observation equations o_i = G_i u_i + delta_i
 * (i = 0..k, cov(delta_i) = C_i; the paper calls C_i "L_i"), by the odd-even
 * QR factorization U A P = Q R of Section III (recursive elimination of the
 * even block columns with Householder transformations, one GPU launch per
 * level), back-substitution up the levels (Section III-A), and the odd-even
 * block SelInv of Algorithm 2 (Section IV) for the covariance blocks
 * Sigma_i = [(R^T R)^{-1}]_{ii} = cov(u_hat_i).
 *
 * Layouts.  Every array argument is a DEVICE pointer to row-major, packed,
 * step-major FP64 data (no strides, no padding):
 *
 *     H, F  [k][n][n]   entry t belongs to evolution step i = t + 1
 *     c     [k][n]
 *     K     [k][n][n] (KS_COV_DENSE) or [k][n] variances (KS_COV_DIAG)
 *     G     [k+1][m][n]
 *     o     [k+1][m]
 *     C     [k+1][m][m] (KS_COV_DENSE) or [k+1][m] variances (KS_COV_DIAG)
 *     u_out [k+1][n]         smoothed states u_hat_i
 *     cov_out [k+1][n][n]    Sigma_i, exactly symmetric
 *
 * H may be NULL, meaning H_i = I.  Dense K_i and C_i are read in full (both
 * triangles) and must be symmetric positive definite; their Cholesky factors
 * whiten the rows (any factor V with V^T V = K^{-1} gives the same u_hat).
 *
 * Ownership.  The caller owns every buffer, including the device workspace
 * given to ks_create, and the HIP stream.  The library never allocates or
 * frees device memory.  A plan keeps the R factor in its workspace between
 * ks_smooth and ks_covariances, so the workspace must outlive the plan.
 *
 * Synchrony.  ks_smooth, ks_smooth_cov and ks_covariances enqueue their
 * kernels on the plan's stream and then synchronize on that stream before
 * returning, so errors detected on the device come back as a status.
 *
 * Errors.  Functions return a ks_status and never abort, throw or print.
 * Output contents are unspecified when the status is not KS_OK.  Argument
 * checks run before any launch.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KS_OK = 0,
    KS_E_ARG = -1,          /* bad dimension, flag, NULL pointer or unsupported n / m     */
    KS_E_WORKSPACE = -2,    /* workspace NULL, misaligned (256 B) or smaller than needed  */
    KS_E_NOT_SPD = -3,      /* some K_i or C_i is not symmetric positive definite          */
    KS_E_RANK = -4,         /* U A lacks numerically full column rank (some |R_jj(p,p)|
                               <= 64 eps max |R(q,q)|), e.g. k = 0 with m < n              */
    KS_E_NONFINITE = -5,    /* a NaN or Inf reached the R factor                           */
    KS_E_HIP = -6,          /* a HIP runtime call failed                                   */
    KS_E_ORDER = -7,        /* ks_covariances before a successful ks_smooth                */
    KS_E_BUSY = -8          /* engine: request does not fit in the free workspace now      */
} ks_status;

/* KS_FP64: every level in FP64.
 * KS_FP32_FORM: the elimination levels with more than 1024 block columns
 * (the wide bottom of the recursion, where almost all the work and traffic
 * is) run in FP32 with FP32 accumulation -- column norms of the Householder
 * vectors scaled by the column's largest entry, reflector coefficients from
 * refined reciprocals -- and keep their R rows and reduced systems in FP32;
 * the top levels run in FP64, and back-substitution and every SelInv product
 * (R^{-1} R^{-T}, T S T^T) run in FP64 on the FP32 rows.  Inputs and outputs
 * stay FP64.  The rank test uses 64 FLT_EPSILON.  (The switch point can be
 * moved with the environment variable KS_FP32_SWITCH read at ks_create.) */
typedef enum { KS_FP64 = 0, KS_FP32_FORM = 1 } ks_precision;
typedef enum { KS_COV_DENSE = 0, KS_COV_DIAG = 1 } ks_cov_layout;

/* Problem description.  k >= 0 evolution steps (k + 1 states), state
 * dimension n >= 1, observation dimension m >= 0 (uniform over steps). */
typedef struct {
    int64_t k;
    int32_t n, m;
    int32_t precision;   /* ks_precision                          */
    int32_t K_layout;    /* ks_cov_layout of K                    */
    int32_t C_layout;    /* ks_cov_layout of C                    */
    uint32_t flags;      /* reserved, must be 0                   */
} ks_desc;

typedef struct ks_plan ks_plan;

/* Exact number of device-workspace bytes a plan for *desc needs, or 0 when
 * the description is invalid or unsupported.  Host-only; no GPU needed. */
size_t ks_workspace_bytes(const ks_desc *desc);

/* Whether the library has kernels for state dimension n and observation
 * dimension m (1 = yes, 0 = no).  Host-only. */
int ks_supported(int32_t n, int32_t m);

/* Create a plan on a caller-owned device workspace (256-byte aligned, at
 * least ks_workspace_bytes(desc) bytes) and a caller-owned hipStream_t
 * (NULL = the default stream).  On success *out receives the plan. */
ks_status ks_create(const ks_desc *desc, void *workspace, size_t ws_bytes,
                    void *hip_stream, ks_plan **out);

/* Smoothed states only (the paper's "NC" mode, Section V-D): whitening,
 * odd-even QR (all levels) and back-substitution.  Keeps R for a later
 * ks_covariances. */
ks_status ks_smooth(ks_plan *plan, const double *H, const double *F,
                    const double *c, const double *K, const double *G,
                    const double *o, const double *C, double *u_out);

/* Covariance blocks Sigma_i from the R factor of the last successful
 * ks_smooth / ks_smooth_cov on this plan (Algorithm 2). */
ks_status ks_covariances(ks_plan *plan, double *cov_out);

/* States and covariances in one pass: the backward sweep fuses
 * back-substitution with the SelInv level of Algorithm 2. */
ks_status ks_smooth_cov(ks_plan *plan, const double *H, const double *F,
                        const double *c, const double *K, const double *G,
                        const double *o, const double *C, double *u_out,
                        double *cov_out);

/* As ks_smooth_cov, and also the lag-one blocks lag1_out[i] =
 * cov(u_i, u_{i+1}) = S_{i,i+1}, i = 0..k-1 ([k][n][n], row index over u_i;
 * may be NULL when k = 0).  Algorithm 2 already forms them at level 0, where
 * every adjacent pair has its even member: S_{i,i+1} = -P_b and
 * S_{i-1,i} = -P_a^T for even i (P = R_ii^{-1} R_iI S_II), so exporting them
 * costs one extra store per block.  Off-diagonal covariance blocks of
 * Section IV; useful for EM. */
ks_status ks_smooth_cov_lag1(ks_plan *plan, const double *H, const double *F,
                             const double *c, const double *K, const double *G,
                             const double *o, const double *C, double *u_out,
                             double *cov_out, double *lag1_out);

/* Value of the objective of Section II-A at u: *total = || U (A u - b) ||^2
 * = sum over i >= 1 of r_i^T K_i^{-1} r_i with r_i = H_i u_i - F_i u_{i-1} - c_i,
 * plus sum over i >= 0 of s_i^T C_i^{-1} s_i with s_i = G_i u_i - o_i
 * (dense covariances through their Cholesky factors, read from the lower
 * triangle).  u is a device array [k+1][n], or NULL for u = 0: then H, F and
 * G are not read and the value is ||U b||^2, which is the objective at the
 * current iterate of a Gauss-Newton or Levenberg-Marquardt iteration
 * (Section II-B) once c and o hold its nonlinear residuals.  terms_out
 * (device [k+1], may be NULL) receives the per-step terms, evolution and
 * observation of step i added together.  total is a HOST pointer.  Uses a
 * small region of the plan's workspace and leaves the R factor of the last
 * smooth intact.  Synchronizes on the plan's stream.  KS_E_NOT_SPD when some
 * K_i or C_i has a non-positive pivot; KS_E_NONFINITE when the total is not
 * finite. */
ks_status ks_objective(ks_plan *plan, const double *H, const double *F,
                       const double *c, const double *K, const double *G,
                       const double *o, const double *C, const double *u,
                       double *terms_out, double *total);

/* ------------------------------------------------ allocation-free variant
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc) and cannot
 * hand in a workspace either: ks_smooth_cov_static computes what ks_create +
 * ks_smooth_cov + ks_destroy would (same kernels, same schedule, bitwise the
 * same states and covariances), but keeps the plan's working data (R rows,
 * reduced systems, stored S blocks, status word) in a static device array of
 * KS_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on until
 * the process ends.  It creates no plan, stream, event or graph and calls no
 * device allocation routine.  desc, the inputs and the outputs are as for
 * ks_create / ks_smooth_cov (device pointers; H may be NULL); hip_stream is
 * the caller's stream (NULL = default stream), and the call synchronizes on
 * it before returning.  Errors: KS_E_ARG for an invalid or unsupported
 * description or a NULL required pointer; KS_E_WORKSPACE when
 * ks_workspace_bytes(desc) exceeds KS_STATIC_SCRATCH_BYTES (nothing is
 * launched); KS_E_HIP when the array's device address cannot be obtained;
 * otherwise the statuses of ks_smooth_cov.  Every call on one GPU uses that
 * GPU's array: calls that overlap on one GPU (other threads, other streams)
 * race and must be serialized by the caller. */
#define KS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

ks_status ks_smooth_cov_static(const ks_desc *desc, const double *H, const double *F,
                               const double *c, const double *K, const double *G,
                               const double *o, const double *C, double *u_out,
                               double *cov_out, void *hip_stream);

/* Release the plan's host state (the workspace stays the caller's). */
ks_status ks_destroy(ks_plan *plan);

/* Static description of a status code. */
const char *ks_status_string(ks_status s);

/* Where the plan keeps the R factor inside its workspace, for inspection:
 * block row of original column i (eliminated at level l = ctz(i+1), level
 * column j = (i+1)/2^l - 1, even) is the record
 *     rrow_offset + (level_rec_offset[l] + j/2) * rrow_stride    (in doubles)
 * holding n rows of [R_ii | R_i,i+2^l | rho_i | R_i,i-2^l] (3n+1 doubles
 * each); missing neighbour blocks are zero.  levels = L + 1 with
 * L = floor(log2(k+1)). */
typedef struct {
    int32_t levels;
    int64_t rrow_offset;          /* doubles from the workspace start */
    int64_t rrow_stride;          /* doubles per record, n (3n + 1)   */
    int64_t level_rec_offset[64];
    int64_t level_columns[64];    /* N_l = floor((k+1) / 2^l)          */
} ks_layout;

ks_status ks_plan_layout(const ks_plan *plan, ks_layout *out);

/* Kernel timing (instrumentation).  ks_time_kernels(plan, kind) resets the
 * plan's accumulators and, for kind != KS_TIME_OFF, makes every later
 * ks_smooth / ks_smooth_cov / ks_covariances on the plan bracket the selected
 * launches with a pair of hipEvents recorded on the plan's stream.  After each
 * call the elapsed time is added up; ks_kernel_time reports the total in
 * milliseconds and the number of bracketed launches (or sequences). */
typedef enum {
    KS_TIME_OFF = 0,
    KS_TIME_FWD_LEVEL0 = 1,   /* the level-0 forward launch (load, whiten, eliminate) */
    KS_TIME_BWD_LEVEL0 = 2,   /* the level-0 backward launch                          */
    KS_TIME_FWD_ALL = 3,      /* all forward launches of a call, as one interval     */
    KS_TIME_BWD_ALL = 4       /* all backward launches of a call, as one interval    */
} ks_time_kind;

ks_status ks_time_kernels(ks_plan *plan, int32_t kind);
ks_status ks_kernel_time(const ks_plan *plan, double *total_ms, int64_t *count);

/* ---------------------------------------------------------------- tuning
 *
 * The schedule's free choices, per state dimension n (1..64) and precision
 * form.  None of them changes what is computed: with the same kernel
 * variants every unit and block row does the same arithmetic whichever
 * launch runs it, so FP64 results are bitwise independent of the tail passes
 * and level groups (a level that runs the matrix-core forward of forward
 * variant 1, n = 32, 48, always has a launch of its own, so the tail, which
 * has the arithmetic of the narrow-level kernels, never takes it over; the
 * FP32 switch changes which levels run in FP32, hence
 * FP32-form results; another kernel variant is another compiled kernel and
 * may round differently).  Plans, batches and the engine read the same
 * table, so a problem's results are the same through all three.
 *   fwd_tail_passes, bwd_tail_passes: the top levels that need at most that
 *     many passes of the single-workgroup forward (backward) tail kernel run
 *     inside it instead of one launch each (0: the base level only);
 *   fp32_switch_columns: in the FP32 form, the levels with more block columns
 *     than this run in FP32;
 *   fwd_group, fwd_group_from: from level fwd_group_from on, fwd_group
 *     consecutive forward levels run in one launch whose workgroups each own
 *     an aligned subtree of units (units read only what their own workgroup
 *     wrote one level down, so levels are separated by workgroup barriers);
 *     1 = one launch per level;
 *   bwd_group, bwd_group_from: the same for the backward levels below the
 *     backward tail (groups bwd_group_from + q bwd_group .. + bwd_group - 1);
 *   fwd_variant, bwd_variant: which compiled shape variant of the forward and
 *     backward kernels runs (ks_kernel_variants), for plans, batches and the
 *     engine alike; a variant that does not exist means the default.
 * Groups apply to single plans (ks_smooth*, ks_covariances,
 * ks_smooth_cov_static) where the kernel family has group kernels, never
 * cross the FP32 switch and stay below the tails.  Defaults 2, 2, 1024,
 * 1, 1, 1, 1, 0, 0; an autotuned table is applied by the Python binding; the
 * environment variables KS_TAIL_PASSES (both pass counts), KS_FP32_SWITCH,
 * KS_FWD_GROUP, KS_FWD_GROUP_FROM, KS_BWD_GROUP, KS_BWD_GROUP_FROM,
 * KS_FWD_VARIANT and KS_BWD_VARIANT override every entry.  Plans, batches and engine requests read the table
 * when they are created; not safe to call concurrently with those. */
typedef struct {
    int32_t fwd_tail_passes;
    int32_t bwd_tail_passes;
    int64_t fp32_switch_columns;   /* >= 1 */
    int32_t fwd_group;             /* 1..8 */
    int32_t fwd_group_from;        /* >= 0 */
    int32_t bwd_group;             /* 1..8 */
    int32_t bwd_group_from;        /* >= 0 */
    int32_t fwd_variant;           /* compiled forward variant (0 = default) */
    int32_t bwd_variant;           /* compiled backward variant (0 = default) */
} ks_tuning;

ks_status ks_set_tuning(int32_t n, int32_t precision, const ks_tuning *t);
/* effective values (environment overrides applied) */
ks_status ks_get_tuning(int32_t n, int32_t precision, ks_tuning *out);
/* Number of compiled forward (backward = 0) or backward (backward != 0)
 * variants for state dimension n and observation dimension m, 0 when (n, m)
 * is unsupported.  Variants compute the same quantities with different
 * kernels, so results may differ by rounding: forward variant 1 of n <= 12
 * runs level 0 without staging a workgroup's inputs in LDS; forward variant 1
 * of n = 32, 48 runs the FP64 forward levels with at least 512 units on the
 * FP64 matrix cores (blocked Householder QR, compact-WY updates; narrower
 * levels and the FP32-form levels keep the default kernels) and applies to
 * problems with diagonal K and C only -- a problem with a dense covariance
 * takes variant 0 instead; forward variant 2 of n = 32, 48 is the default
 * 2-D tiled forward compiled for another occupancy target (n = 32 without
 * the four-wavefronts-per-SIMD register cap, n = 48 with it); backward
 * variants of the MFMA family take 4, 2 or
 * 1 records per workgroup (n <= 12; n = 16, 24: 2 or 1; n = 32: 1 or 2;
 * n = 32 and 48 run the blocked form of that backward), and
 * for n = 1, 2, 3, 5 backward variant 1 is the MFMA family instead of the
 * wavefront family.  Host-only. */
int32_t ks_kernel_variants(int32_t n, int32_t m, int32_t backward);
/* the plan's schedule: number of FP32 levels, first level of the forward tail
 * launch, lowest level of the backward tail launch (states + covariances) */
ks_status ks_plan_schedule(const ks_plan *plan, int32_t *fp32_levels, int32_t *fwd_tail_level,
                           int32_t *bwd_tail_level);

/* ---------------------------------------------------------------- batches
 *
 * Many independent problems (any mix of k, n, m, layouts and precision forms)
 * smoothed together.  Every forward and backward level step is one launch per
 * kernel class (state dimension n, observation class) and precision variant,
 * covering that level of every problem that has it; each problem's top levels
 * run as one workgroup of a single launch.  Each problem follows exactly the
 * schedule a single plan would, so its results are bitwise those of
 * ks_smooth_cov / ks_smooth on it alone.  The launch sequence is captured in a
 * hipGraph on the first call with a given set of pointers and replayed while
 * the pointers stay the same (set KS_NO_GRAPH=1 before ks_batch_create to
 * launch eagerly). */
typedef struct ks_batch ks_batch;

/* device pointers of one problem, layouts as for ks_smooth_cov */
typedef struct {
    const double *H, *F, *c, *K, *G, *o, *C;
    double *u_out;
    double *cov_out;   /* may be NULL when want_cov == 0 */
} ks_io;

/* Exact device-workspace bytes for the batch, or 0 if any description is
 * invalid or unsupported.  Host-only. */
size_t ks_batch_workspace_bytes(int32_t count, const ks_desc *descs);

/* Create a batch over caller-owned workspace (256-byte aligned) and stream. */
ks_status ks_batch_create(int32_t count, const ks_desc *descs, void *workspace, size_t ws_bytes,
                          void *hip_stream, ks_batch **out);

/* Smooth every problem (states, plus covariances when want_cov != 0);
 * synchronous.  statuses (count entries, may be NULL) receives each
 * problem's status; the return value is KS_OK or the first error. */
ks_status ks_batch_smooth(ks_batch *batch, const ks_io *io, int32_t want_cov,
                          ks_status *statuses);

ks_status ks_batch_destroy(ks_batch *batch);

/* ---------------------------------------------------------------- engine
 *
 * Continuous batching for a stream of requests (one smoothing problem each,
 * Section III's forward elimination, the back-substitution, and optionally
 * Algorithm 2's covariances).  The engine owns a caller-given device
 * workspace: 1/16 of it (at least 256 KiB) holds two buffers of per-tick
 * launch tables and 4096 status words, the rest is handed out as one region
 * per admitted request, of exactly ks_workspace_bytes(desc) rounded up to 256
 * bytes (first fit over a free list that merges neighbours on release).  Each
 * tick advances every request that still has steps to launch by one step of
 * its schedule -- one forward level (with its fold), the forward tail, the
 * backward tail or one backward level -- with one launch per kernel class,
 * step kind and precision variant covering all requests at that step, so a
 * request admitted between ticks starts its level 0 in the same launches that
 * carry older requests through their top levels.  A request's schedule is
 * that of a single plan: its results are bitwise those of ks_smooth_cov
 * (want_cov != 0) or ks_smooth on it alone.
 *
 * Engine calls are asynchronous: ks_engine_step enqueues a tick on the
 * engine's stream and returns; at most two ticks are in flight (their launch
 * tables alternate between the two buffers), so a step that finds both in
 * flight first waits for the older one.  Requests may be submitted while ticks
 * run.  A request is finished once the tick holding its last step has
 * completed; ks_engine_step, ks_engine_retired and ks_engine_poll notice
 * completed ticks without blocking, ks_engine_wait blocks until every
 * enqueued tick has completed.  Only then are a finished request's outputs
 * final and its region and status word free.  Host-side state is not
 * thread-safe: one thread drives an engine.
 *
 * Deliberate differences from a flat "inputs[7]" interface: a request's
 * device pointers come in the batch API's ks_io struct, covariances
 * are asked for by want_cov (ks_desc.flags stays reserved; H = NULL means
 * H_i = I), and tuning is the process-wide table of ks_set_tuning rather than
 * a per-engine JSON string. */
typedef struct ks_engine ks_engine;

typedef struct {
    int64_t inflight;         /* admitted, not yet retired                       */
    int64_t retired_pending;  /* retired, not yet collected by ks_engine_retired  */
    int64_t ticks;            /* ticks enqueued                                   */
    size_t region_bytes;      /* workspace bytes for request regions             */
    size_t free_bytes;        /* of which free                                   */
    size_t largest_free;      /* largest free extent (bounds the next admission) */
    int64_t ticks_pending;    /* enqueued ticks not yet seen complete (0..2)     */
} ks_engine_stats;

/* workspace: device memory, 256-byte aligned, at least 1 MiB, caller-owned
 * and kept alive until ks_engine_destroy; all work goes to hip_stream.
 * Host-only: the first step creates two events and 32 KiB of pinned host
 * memory (KS_E_HIP from that step if it fails). */
ks_status ks_engine_create(void *workspace, size_t ws_bytes, void *hip_stream, ks_engine **out);

/* Admit one request; host-only (launches nothing), also while ticks run.  io
 * points to device arrays laid out as for ks_smooth_cov, which must stay
 * valid and unchanged (outputs: untouched by the caller) until the request is
 * retired.  KS_E_BUSY: no free region, table share or status word right now
 * -- retry after a step; KS_E_WORKSPACE: the request can never fit this
 * engine; KS_E_ARG: bad description or pointer.  *ticket identifies the
 * request. */
ks_status ks_engine_submit(ks_engine *engine, const ks_desc *desc, const ks_io *io, int32_t want_cov,
                           uint64_t *ticket);

/* Retire the requests of completed ticks, then enqueue one tick (nothing when
 * no request has steps left to launch) and return without waiting for it.
 * *finished (may be NULL) receives the number of requests retired by this
 * call. */
ks_status ks_engine_step(ks_engine *engine, int32_t *finished);

/* Block until every enqueued tick has completed and retire their requests;
 * *finished (may be NULL) as for ks_engine_step. */
ks_status ks_engine_wait(ks_engine *engine, int32_t *finished);

/* Collect up to capacity retired requests, oldest first: ticket and status
 * (KS_OK, KS_E_NOT_SPD, KS_E_NONFINITE or KS_E_RANK, as ks_smooth_cov would
 * return).  *count receives how many were written. */
ks_status ks_engine_retired(ks_engine *engine, int32_t capacity, uint64_t *tickets,
                            ks_status *statuses, int32_t *count);

/* The status of one request: KS_OK with *result set once it is retired (it
 * is then removed from the retired list), KS_E_BUSY while it is not, KS_E_ARG
 * for a ticket that is neither (unknown or collected). */
ks_status ks_engine_poll(ks_engine *engine, uint64_t ticket, ks_status *result);

ks_status ks_engine_query(const ks_engine *engine, ks_engine_stats *out);

/* Waits for the engine's stream, then frees host state; requests not yet
 * retired are abandoned. */
ks_status ks_engine_destroy(ks_engine *engine);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
