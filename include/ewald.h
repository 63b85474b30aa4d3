/*
 * ewald.h -- C ABI of the MI355X (gfx950) classical Ewald summation library.
 *
 * The library evaluates the electrostatic energy, the forces and the
 * potentials (dE/dq) of N point charges in a periodic cube, split as in
 * Saunders, Grant & Mueller, "Long range forces in a performance portable
 * Molecular Dynamics framework" (section 3):
 *
 *   real space (section 3.1.1, truncated as in Eq. short_range_force):
 *       E_real = 1/2 sum_i sum_{(j,s) != (i,0), |d| < r_c} q_i q_j erfc(sqrt(alpha)|d|)/|d|,
 *       d = r_i - r_j + s, s in L Z^3 (every image closer than r_c, also when r_c > L/2)
 *   reciprocal space (section 3.1.2, factorised as in Eq. perf_mod1, Algorithms 1 and 2):
 *       S_k = sum_j q_j exp(i k.r_j),  k = 2 pi n / L,  n in K = {n != 0 : |n|^2 <= k_max^2}
 *       C_k = 4 pi / (V k^2) exp(-k^2 / (4 alpha)),  E_recip = 1/2 sum_K C_k |S_k|^2
 *       F_recip,i = q_i sum_K C_k k Im(exp(i k.r_i) conj(S_k))
 *   self term (section 3.2.2; formula not printed there):  E_self = -sqrt(alpha/pi) sum q_i^2
 *   neutralising background (the paper assumes Q = 0):     E_bg   = -pi Q^2 / (2 V alpha)
 *
 * Units are Gaussian (potential q/r, section 2.1).  alpha is the exponent of the
 * splitting Gaussian exp(-alpha r^2) (section 3.1.1): callers who write the
 * real-space kernel as erfc(beta r) pass alpha = beta^2.  The boundary at
 * infinity is conducting (no dipole term).
 *
 * Conventions shared by every entry point:
 *   - All pointers named "device" are HIP device pointers (e.g. torch CUDA/HIP
 *     tensors' data_ptr()) on the plan's device; "host" pointers are ordinary
 *     host memory.  All floating-point arrays are IEEE double, C-contiguous.
 *   - Positions may lie anywhere; they are reduced into [0, L)^3 internally.
 *     Results are returned in the caller's particle order.
 *   - Outputs are overwritten, never accumulated into.
 *   - Calls are stream-ordered and asynchronous on the plan's stream; they
 *     return after enqueueing the work.  Internally the reciprocal-space part
 *     runs on a second stream owned by the plan, forked from and joined back to
 *     the plan's stream with events, so that it overlaps the real-space part;
 *     work enqueued on the plan's stream after a call still sees all of that
 *     call's results and may overwrite its inputs.  Host-detectable errors
 *     return before anything is enqueued.  No call aborts the process.
 *   - Graph replay: the key of an evaluation is its n, buffers (pos, q and
 *     every output pointer) and kind (energy and forces, energy only, or
 *     backward with its grad_energy pointer).  The plan remembers the last 4
 *     distinct keys; the second evaluation with a remembered key captures the
 *     launch sequence into a HIP graph (on a plan-owned capture stream, so the
 *     plan's stream may be the null stream) and later ones launch that graph
 *     onto the plan's stream when that stream is idle (hipStreamQuery): the
 *     graph saves host launch time, which only a call on an idle stream waits
 *     for; behind queued work the kernels are launched one by one.  The graph
 *     runs the same kernels with the same arguments, so results are bitwise
 *     those of the kernel-by-kernel launch.  Any other call launches kernel by
 *     kernel; so do profiled calls and plans made with EWALD_FLAG_NO_GRAPH, and
 *     a plan whose capture failed once (it then never tries again).
 *   - A plan is not re-entrant: calls on one plan must not overlap.  Distinct
 *     plans may be used concurrently on distinct streams.
 *   - Results are bitwise reproducible for identical inputs, plan and device
 *     (fixed-order reductions, no floating-point atomics).
 */
#ifndef EWALD_MI355X_H
#define EWALD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque plan: one (L, alpha, r_c, k_max, n_max, precision, device, stream). */
typedef struct ewald_plan_s *ewald_plan_t;

/* Status codes.  ewald_status_string() gives a static English description. */
typedef enum {
    EWALD_OK = 0,
    EWALD_ERR_INVALID_ARG = -1,   /* a parameter or pointer is invalid            */
    EWALD_ERR_CAPACITY = -2,      /* n exceeds the plan's n_max                   */
    EWALD_ERR_OUT_OF_MEMORY = -3, /* device or host allocation failed             */
    EWALD_ERR_DEVICE = -4,        /* a HIP runtime call or kernel launch failed   */
    EWALD_ERR_NONFINITE = -5,     /* a position or charge was NaN or infinite     */
    EWALD_ERR_ADMISSION = -6,     /* workspace above a server's free HBM budget   */
    EWALD_ERR_SCRATCH = -7        /* buffers of an allocation-free evaluation
                                     exceed EWALD_SCRATCH_BYTES                   */
} ewald_status;

/* Arithmetic of the hot kernels. */
enum {
    EWALD_PRECISION_FP64 = 0,  /* every step in IEEE double                          */
    EWALD_PRECISION_MIXED = 1  /* FP32 pair functions (rsqrt, erfc, exp) and FP32
                                  phases, coefficients and products in the force
                                  gather; FP64 displacements, phase generation,
                                  the structure factor, per-particle sums and all
                                  energies                                         */
};

/* Plan parameters.
 *   n_max      largest N the plan will be called with, 1 <= n_max <= 2^25; all
 *              workspace is sized for it at plan time.
 *   box_L      side of the periodic cube (> 0).
 *   alpha      Gaussian splitting exponent (> 0), see above.
 *   r_c        real-space cutoff, 0 < r_c <= box_L; the test is |d|^2 < r_c^2.
 *   k_max      reciprocal cutoff on integer vectors, |n|^2 <= k_max^2,
 *              1 <= k_max <= EWALD_K_MAX_LIMIT.
 *   precision  EWALD_PRECISION_FP64 or EWALD_PRECISION_MIXED.
 *   device     HIP device ordinal the plan lives on.
 *   stream     hipStream_t the work is enqueued on; NULL means the device's
 *              null stream.  May be changed later with ewald_plan_set_stream().
 *   flags      0, or a combination of
 *                EWALD_FLAG_VALU_GATHER  reciprocal force gather on the vector ALUs,
 *                EWALD_FLAG_VALU_SK      structure factor on the vector ALUs,
 *              instead of the matrix cores (same results to rounding; used to
 *              compare the two), and
 *                EWALD_FLAG_NO_GRAPH     always launch kernel by kernel (see
 *                                        "Graph replay" below),
 *                EWALD_FLAG_ONE_STREAM   run the reciprocal-space chain on the plan's
 *                                        stream too, before the real-space one,
 *                                        instead of beside it on a second stream
 *                                        (same results; per-kernel timings then
 *                                        measure each kernel alone),
 *                EWALD_FLAG_NO_WORKSPACE allocate only the plan's constant tables
 *                                        (a few MB at most); such a plan is
 *                                        evaluated with ewald_energy_forces_noalloc(),
 *                                        or with ewald_energy_forces_ws() and
 *                                        ewald_energy_forces_batch() given a
 *                                        workspace (every other evaluation and
 *                                        debug call returns EWALD_ERR_INVALID_ARG).
 *              Other bits are invalid.  The vector kernels are
 *              also used where the matrix-core ones do not fit: the gather when a
 *              block's staged z powers would exceed 64 KB of LDS (FP64 with
 *              k_max > 83), the structure factor for k_max > 47. */
typedef struct {
    int64_t n_max;
    double box_L;
    double alpha;
    double r_c;
    int32_t k_max;
    int32_t precision;
    int32_t device;
    int32_t flags;
    void *stream;
} ewald_params;

#define EWALD_K_MAX_LIMIT 100
#define EWALD_FLAG_VALU_GATHER 1
#define EWALD_FLAG_VALU_SK 2
#define EWALD_FLAG_NO_GRAPH 4
#define EWALD_FLAG_NO_WORKSPACE 8
#define EWALD_FLAG_ONE_STREAM 16

/* Size of the per-device static scratch of ewald_energy_forces_noalloc(). */
#define EWALD_SCRATCH_BYTES ((size_t)64 << 20)

/* Static description of a status code (never NULL). */
const char *ewald_status_string(ewald_status status);

/* Validate parameters without touching the GPU: EWALD_OK or EWALD_ERR_INVALID_ARG. */
ewald_status ewald_params_validate(const ewald_params *params);

/* Device bytes a plan with these parameters allocates (0 if the parameters
 * are invalid).  Pure host arithmetic: usable for admission decisions. */
size_t ewald_plan_workspace_bytes(const ewald_params *params);

/* Number of k vectors in the half space K+ (n_x > 0, or n_x = 0 and n_y > 0,
 * or n_x = n_y = 0 and n_z > 0) for this k_max; |K| = 2 |K+|.  Host only. */
int64_t ewald_kset_size(int32_t k_max);

/* Create a plan: validates *params, builds the k-set tables and the cell grid
 * (n_c = floor(2 L / r_c) cells per axis) and allocates all device workspace for
 * n_max.  On success *out receives the plan; on failure *out is set to NULL and
 * nothing stays allocated.  Errors: INVALID_ARG (bad params or out == NULL),
 * OUT_OF_MEMORY, DEVICE. */
ewald_status ewald_plan(const ewald_params *params, ewald_plan_t *out);

/* Replace the stream the plan enqueues on (NULL: the null stream). */
ewald_status ewald_plan_set_stream(ewald_plan_t plan, void *stream);

/* Energy, forces and dE/dq for n charges (section 3, formulas above).
 *   pos     device, n x 3 row-major (x, y, z per particle); read only.
 *   q       device, n charges; read only.
 *   energy  device, 5 doubles written: {total, real, recip, self, background}.
 *   forces  device, n x 3 row-major F_i = -dE/dr_i, or NULL to skip.
 *   dEdq    device, n values dE/dq_i, or NULL to skip.
 * Errors returned immediately: INVALID_ARG (NULL plan/pos/q/energy, n < 1),
 * CAPACITY (n > n_max), DEVICE (launch failure).  Non-finite inputs are found
 * on the device: the energy is set to NaN and EWALD_ERR_NONFINITE is latched
 * for ewald_plan_status(). */
ewald_status ewald_energy_forces(ewald_plan_t plan, int64_t n, const double *pos, const double *q,
                                 double *energy, double *forces, double *dEdq);

/* Energy only (the forward of the adjoint pair below): same arguments and
 * errors as ewald_energy_forces without force / dE/dq outputs.  The force
 * gather is skipped; the reciprocal energy comes from the structure factor. */
ewald_status ewald_energy(ewald_plan_t plan, int64_t n, const double *pos, const double *q, double *energy);

/* Adjoint of E(pos, q) for an upstream gradient g = dL/dE:
 *   grad_energy  device, 1 double: g (read on the device, no host sync).
 *   energy       device, 5 doubles: the energy parts, recomputed.
 *   grad_pos     device, n x 3: dL/dr_i = -g F_i, or NULL to skip.
 *   grad_q       device, n: dL/dq_i = g dE/dq_i, or NULL to skip.
 * The phases and S(k) are recomputed from pos and q (nothing per particle and
 * k vector is stored between the forward and this call).  Errors as
 * ewald_energy_forces, plus INVALID_ARG for a NULL grad_energy. */
ewald_status ewald_energy_backward(ewald_plan_t plan, int64_t n, const double *pos, const double *q,
                                   const double *grad_energy, double *energy, double *grad_pos, double *grad_q);

/* Bytes of the per-evaluation buffers (cell list, neighbour lists, phase
 * tables, structure-factor partials, gather partials, counters) of one
 * evaluation of n particles on this plan: the workspace that
 * ewald_energy_forces_ws() takes.  Host only; 0 for a NULL plan or n outside
 * 1 .. n_max. */
size_t ewald_eval_workspace_bytes(ewald_plan_t plan, int64_t n);

/* ewald_energy_forces() with its per-evaluation buffers in caller memory.
 *   workspace        device, 256-byte aligned, at least
 *                    ewald_eval_workspace_bytes(plan, n) bytes; the call's
 *                    kernels use it until the call's work on the plan's stream
 *                    has completed (the caller may reuse it after that).
 *   workspace_bytes  its size.
 * Same results, bit for bit, as ewald_energy_forces() on the same plan (the
 * same kernels with the same launch shapes).  Allocates nothing; launches
 * kernel by kernel (no graph replay, no profiling); the counters that must
 * start at zero are cleared in the workspace by a fill kernel.  The plan may
 * have been made with EWALD_FLAG_NO_WORKSPACE.  Errors as
 * ewald_energy_forces(), plus INVALID_ARG for a NULL or misaligned workspace
 * and CAPACITY for one that is too small (nothing enqueued). */
ewald_status ewald_energy_forces_ws(ewald_plan_t plan, int64_t n, const double *pos, const double *q,
                                    double *energy, double *forces, double *dEdq, void *workspace,
                                    size_t workspace_bytes);

/* Most systems one ewald_energy_forces_batch() call takes. */
#define EWALD_BATCH_MAX 1024

/* ewald_energy_forces() of `count` independent systems in one launch
 * sequence: each kernel of the path (section 3.2.1 real space, Eq. perf_mod1
 * and Algorithms 1 and 2 reciprocal space, section 3.2.2 self and background
 * terms) is launched once for all the systems, over a ragged work list in
 * which every system owns a contiguous range of the launch's workgroups, in
 * place of count launches.  Systems may differ in n, box, alpha, r_c, k_max
 * and precision; those whose shapes select different kernel instances or
 * block sizes share the step's launch order but not a launch, and at most a
 * kernel's pack of argument structs (8 or more systems) goes into one launch.
 *   plans[i]             plan of system i; all on one device.
 *   n[i], pos[i], q[i], energy[i], forces[i], dEdq[i]
 *                        as for ewald_energy_forces() (forces and dEdq may be
 *                        NULL arrays, or hold NULL entries).
 *   workspace[i]         device, 256-byte aligned, at least
 *                        ewald_eval_workspace_bytes(plans[i], n[i]) bytes
 *                        (workspace_bytes[i] says how many): system i's
 *                        per-evaluation buffers.  May be a NULL array or hold
 *                        NULL: then the plan's own buffers are used, and that
 *                        plan (made without EWALD_FLAG_NO_WORKSPACE) is used
 *                        by no other NULL-workspace entry of the batch.
 *   stream               hipStream_t the batch is enqueued on (NULL: the null
 *                        stream).  As in a single evaluation, the
 *                        reciprocal-space launches run beside the real-space
 *                        ones on a second stream, that of plans[0], forked from
 *                        and joined back to `stream` with plans[0]'s events,
 *                        unless plans[0] was made with EWALD_FLAG_ONE_STREAM;
 *                        work enqueued on `stream` afterwards sees the whole
 *                        batch.  The plans' own streams are not used otherwise,
 *                        so no earlier call on a plan may still be running on
 *                        another stream, and ewald_plan_status() is read after
 *                        synchronising `stream`.
 * Each system's results are bitwise those of ewald_energy_forces_ws() on the
 * same inputs: every workgroup runs the same code on the same arguments.
 * Allocates nothing; the launch descriptors travel in the kernel arguments.
 * No graph replay and no profiling.  INVALID_ARG for count outside 1 ..
 * EWALD_BATCH_MAX, a NULL or mis-aligned pointer, plans on different devices,
 * or a plan's own buffers named twice; CAPACITY for n above a plan's n_max or
 * a workspace that is too small; nothing is enqueued on either. */
ewald_status ewald_energy_forces_batch(int32_t count, const ewald_plan_t *plans, const int64_t *n,
                                       const double *const *pos, const double *const *q, double *const *energy,
                                       double *const *forces, double *const *dEdq, void *const *workspace,
                                       const size_t *workspace_bytes, void *stream);

/* Allocation-free variant of ewald_energy_forces(), for callers that cannot
 * allocate device memory while they evaluate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * results (bitwise: the same kernels with the same launch shapes) and errors,
 * except that the per-evaluation buffers (cell list, neighbour lists, phase
 * tables, structure-factor partials, gather partials) are carved from a
 * static device array of EWALD_SCRATCH_BYTES that the library holds on every
 * device it runs on, until the process ends, instead of from the plan's
 * workspace.  The plan may have been made with EWALD_FLAG_NO_WORKSPACE.
 *   - Nothing is allocated: no hipMalloc, hipFree, event or graph creation; the
 *     kernels are launched one by one (no graph replay, no profiling).  The
 *     counters that must start at zero are cleared by a fill kernel.
 *   - Returns EWALD_ERR_SCRATCH, with nothing enqueued, when the buffers for n
 *     particles at the plan's k_max and cell grid exceed EWALD_SCRATCH_BYTES
 *     (about 12,000 ions at the density and cutoffs of the 32^3 rock salt).
 *   - All calls on one device share that device's array, which keeps the last
 *     call's contents: calls that may overlap on one device (any plans, any
 *     streams) race and give wrong results; the caller serialises them. */
ewald_status ewald_energy_forces_noalloc(ewald_plan_t plan, int64_t n, const double *pos, const double *q,
                                         double *energy, double *forces, double *dEdq);

/* Synchronise the plan's stream, then return and clear the status latched by
 * device-side checks (EWALD_OK if none). */
ewald_status ewald_plan_status(ewald_plan_t plan);

/* Synchronise the plan's stream and free everything the plan owns.
 * ewald_release(NULL) is a no-op; using a plan after release is undefined. */
void ewald_release(ewald_plan_t plan);

/* ---- inspection hooks (tests, profiling) ---- */

/* Number of k vectors in the plan's half space K+. */
int64_t ewald_plan_kcount(ewald_plan_t plan);

/* Host copy of the plan's K+ as integer triples (host, kcount x 3 int32), in
 * the order ewald_debug_copy_sk() uses. */
ewald_status ewald_debug_kset(ewald_plan_t plan, int32_t *n_xyz);

/* Host copy of S_k over K+ from the last completed evaluation (host arrays of
 * kcount doubles).  Synchronises the plan's stream. */
ewald_status ewald_debug_copy_sk(ewald_plan_t plan, double *re, double *im);

/* Which branches of the path the plan takes and took (host values).  Filled
 * from the plan's parameters and, after synchronising the plan's stream, from
 * the device state of its last completed evaluation of n particles (n must be
 * that evaluation's particle count).  For tests of the fallback paths, and
 * for the work the matrix-core kernels execute (their launch shapes for n
 * particles, counted on the host from the plan's tile layout). */
typedef struct {
    int64_t max_cell_count;      /* most particles in one real-space cell            */
    int64_t direct_particles;    /* particles whose neighbour list would have passed
                                    the capacity, evaluated by the direct loop        */
    int64_t listed_pairs;        /* ordered pairs (i, j, image) with |d| < r_c found
                                    by the neighbour lists (direct-loop particles'
                                    pairs are not counted)                            */
    int32_t cells_per_axis;      /* real-space cells per axis                         */
    int32_t list_capacity;       /* neighbour-list entries per particle               */
    int32_t sk_matrix_cores;     /* 1: structure factor on the matrix cores           */
    int32_t gather_matrix_cores; /* 1: force gather on the matrix cores               */
    int32_t phase_rows;          /* table rows per phase-kernel block                 */
    int32_t reserved;
    int64_t sk_mfma_flops;       /* flops the matrix-core instructions of one
                                    structure-factor launch for n particles execute
                                    (0 on the vector ALUs): 512 per FP64 4x4x4 MFMA   */
    int64_t gather_mfma_flops;   /* the same for one force-gather launch: 2048 per
                                    16x16x4 MFMA (FP32 mixed, FP64 plain)             */
} ewald_debug_stats;

ewald_status ewald_debug_stats_read(ewald_plan_t plan, int64_t n, ewald_debug_stats *out);

/* Kernel timing: when enabled, every launch of the plan is bracketed by HIP
 * events on the plan's stream and its duration accumulated per kernel class.
 * ewald_profile_read() synchronises, fills up to max_entries names (static
 * strings), total milliseconds and launch counts, and returns the number of
 * kernel classes; ewald_profile_reset() clears the totals. */
ewald_status ewald_profile_enable(ewald_plan_t plan, int32_t enable);
int32_t ewald_profile_read(ewald_plan_t plan, const char **names, double *total_ms,
                           int64_t *launches, int32_t max_entries);
ewald_status ewald_profile_reset(ewald_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* EWALD_MI355X_H */
