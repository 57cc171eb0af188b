/*
 * nbody.h - C ABI of libnbody.so: direct-summation gravitational N-body on
 * AMD Instinct MI355X (gfx950).
 *
 * What is computed. The force equation of Section 3 of Almerol et al.,
 * "Accelerating Gravitational N-Body Simulations Using the RISC-V-Based
 * Tenstorrent Wormhole" (SC'25 Workshops): the force on particle i is the
 * sum over every other particle j != i of G m_i m_j (r_j - r_i) / r_ij^3.
 * This library returns it per unit target mass, with Plummer softening eps:
 *
 *     a_i   =  G sum_{j != i} m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^(3/2)
 *     phi_i = -G sum_{j != i} m_j / (|x_j - x_i|^2 + eps^2)^(1/2)
 *
 * eps = 0 is the paper's unsoftened sum exactly. The pair arithmetic runs in
 * FP32 on the GPU, as the paper's device force does (Section 3,
 * mixed-precision paragraph); positions, velocities, the integrator and all
 * outputs are FP64.
 *
 * Conventions for every call below.
 *  - Array pointers are DEVICE pointers unless the name ends in _host. The
 *    caller owns every buffer; the calls in this header never allocate device
 *    memory, except nbody_plan_create, which owns what it allocates until
 *    nbody_plan_destroy.
 *  - Arrays are C-contiguous: pos, vel, acc are [n][3] float64 (x, y, z of a
 *    particle adjacent); mass and pot are [n] float64.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously on it; the call returns without
 *    synchronising. Device faults surface at the caller's next
 *    synchronisation, as for any HIP launch.
 *  - Validation is synchronous and host-side, before any launch. On any
 *    non-OK status nothing has been enqueued and outputs are untouched;
 *    nbody_last_error() then describes the problem.
 *  - Input and output arrays must not overlap, except where stated.
 *  - Results are deterministic: the same inputs and tuning give bitwise the
 *    same outputs on every run (no floating-point atomics).
 *  - Calls from several host threads are safe if they use distinct buffers;
 *    calls that share a workspace or a plan must be ordered by the caller.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nbody_status;
#define NBODY_OK 0
#define NBODY_EINVAL 1      /* a null pointer, size or scalar out of range   */
#define NBODY_ENOTSUP 2     /* a variant or size the library does not handle */
#define NBODY_EWORKSPACE 3  /* workspace missing or smaller than required    */
#define NBODY_EHIP 4        /* the HIP runtime returned an error             */

/* Pair-kernel forms. */
#define NBODY_FP32_PLAIN 0  /* FP32 coordinates and sums (two-level: per tile, then running) */
#define NBODY_FP32_COMP 1   /* FP32 pair arithmetic on double-single (hi, lo) coordinates
                               relative to a per-block FP64 frame, compensated (TwoSum)
                               accumulation, FP64 epilogue. For large systems the library
                               orders the particles spatially (internally; results stay at
                               the caller's indices) and source tiles far from a block
                               drop the lo parts, which keeps every separation within
                               6 ulps of its own size */

/* One diagnostics row (float64), written after every step by nbody_step. */
#define NBODY_DIAG_LEN 16
#define NBODY_DIAG_K 0        /* kinetic energy 1/2 sum m |v|^2                  */
#define NBODY_DIAG_W 1        /* potential energy 1/2 sum m phi                  */
#define NBODY_DIAG_E 2        /* K + W                                           */
#define NBODY_DIAG_P 3        /* [3] total momentum sum m v                      */
#define NBODY_DIAG_L 6        /* [3] total angular momentum sum m x cross v      */
#define NBODY_DIAG_COM 9      /* [3] centre of mass sum m x / sum m              */
#define NBODY_DIAG_M 12       /* total mass                                      */
#define NBODY_DIAG_NONFINITE 13 /* number of non-finite entries in pos and vel   */
#define NBODY_DIAG_STEP 14    /* step index within the call, starting at 1       */

/* Opaque batched plan: many independent clusters, their work list and tuning. */
typedef struct nbody_plan nbody_plan;

/* Bytes of device workspace the calls below need for a system of n_total
 * particles in n_clusters clusters (1 for a single system) with `variant`.
 * Pure host arithmetic; returns 0 for invalid arguments (n_total < 0,
 * n_clusters < 1, unknown variant). */
size_t nbody_workspace_bytes(int64_t n_total, int32_t n_clusters, int32_t variant);

/* Text of the last non-OK status on the calling thread ("" if none). The
 * pointer stays valid until the next call on that thread. */
const char *nbody_last_error(void);

/* Library version string. */
const char *nbody_version(void);

/* Accelerations (and potentials) of a single system (the force equation of
 * Section 3, softened by eps).
 *   pos   [n][3] f64 in; mass [n] f64 in (any finite values >= 0).
 *   n >= 0 (n = 0 is a no-op; n = 1 gives acc = pot = 0).
 *   eps >= 0 and finite; eps = 0 excludes j == i and any pair at zero
 *   separation (coincident distinct particles at eps = 0 are undefined).
 *   G finite.
 *   variant NBODY_FP32_PLAIN or NBODY_FP32_COMP.
 *   acc [n][3] f64 out; pot [n] f64 out or NULL.
 *   ws: device workspace of ws_bytes >= nbody_workspace_bytes(n, 1, variant),
 *   256-byte aligned; its contents need not be initialised and are scratch.
 * Errors: EINVAL (null pos/mass/acc with n > 0, n < 0, bad eps/G, overlap of
 * acc with pos), ENOTSUP (unknown variant), EWORKSPACE (missing, too small or
 * misaligned workspace), EHIP. */
nbody_status nbody_accel(const double *pos, const double *mass, int64_t n,
                         double eps, double G, int32_t variant,
                         double *acc, double *pot,
                         void *ws, size_t ws_bytes, void *stream);

/* Allocation-free nbody_accel, for callers that cannot allocate device
 * memory or hand the library a workspace: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and errors as nbody_accel, without ws/ws_bytes:
 * its workspace is a 64 MiB static device array inside the library, which
 * every GPU the library runs on holds until the process ends. The first call
 * on a device looks up that device's copy; no call allocates or frees.
 * Limits: n <= 1,676,064 (NBODY_FP32_PLAIN) and n <= 536,480
 * (NBODY_FP32_COMP); a larger n is EINVAL and names the limit. Where the
 * tuned grid j-split's partial sums do not fit, a smaller split is used, so
 * results are bitwise equal to nbody_accel's at most sizes and otherwise
 * differ only in summation order (within the same tolerances).
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (two streams, two host threads)
 * race and corrupt each other's results; the caller must order them. */
nbody_status nbody_accel_noalloc(const double *pos, const double *mass, int64_t n,
                                 double eps, double G, int32_t variant,
                                 double *acc, double *pot, void *stream);

/* n_steps kick-drift-kick leapfrog steps of a single system (all FP64 on the
 * GPU, forces by the chosen variant). Per step: v += dt/2 a; x += dt v;
 * a = A(x); v += dt/2 a.
 *   pos, vel [n][3] f64 in/out; acc [n][3] f64 in/out: on entry it must hold
 *   A(pos) (call nbody_accel once first), on return A(pos_final).
 *   pot [n] f64 out (potentials at the final positions) or NULL.
 *   mass [n] f64 in. eps, G, variant as for nbody_accel; dt finite;
 *   n_steps >= 0.
 *   plan: must be NULL. (Batched clusters are stepped by nbody_step_batched,
 *   which takes the per-cluster softenings; a non-NULL plan is EINVAL.)
 *   diag [n_steps][NBODY_DIAG_LEN] f64 out or NULL: one row after each step.
 *   ws as for nbody_accel (nbody_workspace_bytes(n, 1, variant)). */
nbody_status nbody_step(double *pos, double *vel, double *acc, double *pot,
                        const double *mass, int64_t n, double eps, double G,
                        double dt, int32_t n_steps, int32_t variant,
                        const nbody_plan *plan, double *diag,
                        void *ws, size_t ws_bytes, void *stream);

/* Build a plan for K independent clusters (the force equation of Section 3
 * applied within each cluster; clusters exert no force on one another).
 * Cluster k owns particles [offsets_host[k], offsets_host[k+1]).
 *   offsets_host [K+1] int64 host, offsets_host[0] = 0, non-decreasing;
 *   offsets_host[K] + 16 K < 2^31.
 *   variant as above; the batched calls made with the plan must use it.
 *   tune_path: a tuning file written by the autotuner (its "batched" lines
 *   pick the plan's kernel mode per cluster size class; other lines are
 *   checked and ignored), or NULL for the process-wide table (built-in, then
 *   NBODY_TUNE, then nbody_tune_load). The file affects this plan only.
 * The per-cluster softenings are not part of the plan: every batched call
 * takes them (eps_k), so one plan serves any softenings.
 * Allocates device memory for the work list and a capture stream on the
 * current device; the batched calls must be made with that device current
 * (EINVAL otherwise). Returns NULL on error (see nbody_last_error). */
nbody_plan *nbody_plan_create(const int64_t *offsets_host, int32_t K,
                              int32_t variant, const char *tune_path);

/* Free a plan (NULL is a no-op). The caller must ensure no enqueued work
 * still uses it. */
void nbody_plan_destroy(nbody_plan *plan);

/* Accelerations and potentials of every cluster of `plan`, each from its own
 * members only and softened by its own eps_k[k], in one persistent-kernel
 * launch per kernel mode.
 *   pos [n_total][3], mass [n_total] in; acc [n_total][3] out; pot [n_total]
 *   out or NULL; n_total = offsets_host[K] of the plan.
 *   eps_k [K] f64 in, DEVICE memory, 8-byte aligned, read by the kernel
 *   (its values are not checked on the host: each should be finite and
 *   >= 0; eps_k[k] = 0 is the unsoftened sum for cluster k, a NaN makes that
 *   cluster's outputs NaN). G finite. variant must equal the plan's.
 *   ws: ws_bytes >= nbody_workspace_bytes(n_total, K, variant).
 * Errors: EINVAL (NULL plan, NULL eps_k for a non-empty plan, misaligned
 * eps_k, variant differing from the plan's, a current device other than the
 * plan's, bad G, NULL or overlapping arrays), ENOTSUP (unknown variant),
 * EWORKSPACE, EHIP. */
nbody_status nbody_accel_batched(const double *pos, const double *mass,
                                 const nbody_plan *plan, const double *eps_k,
                                 double G, int32_t variant,
                                 double *acc, double *pot,
                                 void *ws, size_t ws_bytes, void *stream);

/* n_steps kick-drift-kick steps of every cluster of `plan` (the step of
 * nbody_step, the forces of nbody_accel_batched with eps_k).
 *   n must equal the plan's n_total; eps_k, variant as for
 *   nbody_accel_batched; other arguments as for nbody_step. The diagnostics
 *   rows sum over all clusters.
 * Each step is one replay of a HIP graph the plan captures on first use for
 * this set of pointers (eps_k included) and scalars; eps_k's contents are
 * read at every replay, so they may change between calls. */
nbody_status nbody_step_batched(double *pos, double *vel, double *acc, double *pot,
                                const double *mass, int64_t n, const nbody_plan *plan,
                                const double *eps_k, double G, double dt,
                                int32_t n_steps, int32_t variant, double *diag,
                                void *ws, size_t ws_bytes, void *stream);

/* Number of particles and clusters a plan covers, and its variant. */
int64_t nbody_plan_total(const nbody_plan *plan);
int32_t nbody_plan_clusters(const nbody_plan *plan);
int32_t nbody_plan_variant(const nbody_plan *plan);
/* Number of (cluster, i-block) work items and sum of their pair counts. */
int64_t nbody_plan_items(const nbody_plan *plan);
double nbody_plan_pairs(const nbody_plan *plan);

/* Tuning. A configuration is (block threads, i per thread, lanes per i,
 * waves per i-group, j-tile, grid j-split). nbody_tune_set forces one for a
 * variant and size class until reset (cfg = -1 restores the table entry);
 * nbody_tune_count and nbody_tune_describe enumerate the compiled set. Used
 * by the autotuner; size_class = floor(log2(n)). */
int32_t nbody_tune_count(int32_t variant);
nbody_status nbody_tune_describe(int32_t variant, int32_t cfg, int32_t *out6);
nbody_status nbody_tune_set(int32_t variant, int32_t size_class, int32_t cfg);
int32_t nbody_tune_get(int32_t variant, int64_t n);
nbody_status nbody_tune_load(const char *path);
/* Restore the built-in tuning table (then NBODY_TUNE, if set) and clear
 * every forced configuration. */
nbody_status nbody_tune_reset(void);

/* ---- acceleration + jerk and the Hermite integrator ----------------------
 * The paper's device computes the jerk (the time derivative of the
 * acceleration) beside the force (Section 3). With d = x_j - x_i,
 * w = v_j - v_i and q = |d|^2 + eps^2:
 *     jerk_i = G sum_{j != i} m_j [w q^{-3/2} - 3 (d.w) d q^{-5/2}].
 * Pair arithmetic is FP32 (the compensated form uses double-single
 * positions relative to particle 0 and velocities relative to particle 0's);
 * outputs are FP64. */

/* Workspace bytes for nbody_accel_jerk / nbody_step_hermite (0 for invalid
 * arguments). */
size_t nbody_workspace_bytes_jerk(int64_t n, int32_t variant);

/* Accelerations, jerks and potentials of one system.
 *   pos, vel [n][3] f64 in; mass [n] f64 in; acc, jerk [n][3] f64 out;
 *   pot [n] f64 out or NULL. Other arguments and errors as nbody_accel;
 *   ws_bytes >= nbody_workspace_bytes_jerk(n, variant). */
nbody_status nbody_accel_jerk(const double *pos, const double *vel, const double *mass, int64_t n,
                              double eps, double G, int32_t variant, double *acc, double *jerk,
                              double *pot, void *ws, size_t ws_bytes, void *stream);

/* n_steps of the fourth-order Hermite predictor-corrector with a shared
 * step, FP64 on the GPU (Makino and Aarseth 1992): predict
 * x_p = x + v dt + a dt^2/2 + j dt^3/6, v_p = v + a dt + j dt^2/2; evaluate
 * a_1, j_1 at (x_p, v_p); correct v_1 = v + (a + a_1) dt/2 + (j - j_1) dt^2/12,
 * x_1 = x + (v + v_1) dt/2 + (a - a_1) dt^2/12.
 *   acc, jerk must hold A(pos, vel) and J(pos, vel) on entry (call
 *   nbody_accel_jerk first) and hold a_1, j_1 of the last step on return.
 *   pot (nullable) and the diagnostics' W use the potentials evaluated at the
 *   predicted positions of the step. diag as for nbody_step.
 *   ws_bytes >= nbody_workspace_bytes_jerk(n, variant). */
nbody_status nbody_step_hermite(double *pos, double *vel, double *acc, double *jerk, double *pot,
                                const double *mass, int64_t n, double eps, double G, double dt,
                                int32_t n_steps, int32_t variant, double *diag, void *ws,
                                size_t ws_bytes, void *stream);

/* Shapes of the acceleration + jerk kernel, for the autotuner.
 * nbody_tune_jerk_count: number of compiled shapes valid for a variant (0 for
 * an unknown variant); shapes 10 and 11 (compensated form only) run the
 * near/far kernel on the spatial order. nbody_tune_jerk_describe
 * writes {K targets per lane, SW waves splitting the sources, targets per
 * block} to out3 (host memory); shapes 8 and 9 repeat shapes 2 and 1 with
 * eight sources per scalar-load group in the plain form. nbody_tune_jerk_set forces cfg + 1000 * split
 * (split 0 = the built-in rule) for every size of a variant; -1 returns to
 * the built-in table. nbody_tune_jerk_get returns cfg + 1000 * split as used
 * for n particles (-1 for invalid arguments). A forced split larger than the
 * one a workspace was sized for makes the next call fail with
 * NBODY_EWORKSPACE: size workspaces after forcing. nbody_tune_reset also
 * clears the forced jerk shape. */
int32_t nbody_tune_jerk_count(int32_t variant);
nbody_status nbody_tune_jerk_describe(int32_t cfg, int32_t *out3);
nbody_status nbody_tune_jerk_set(int32_t variant, int32_t cfg);
int32_t nbody_tune_jerk_get(int32_t variant, int64_t n);

/* Kernel timing, for measurement. While enabled (on != 0), every
 * force-kernel launch made outside graph capture by nbody_accel, nbody_step,
 * nbody_accel_batched, nbody_accel_jerk and nbody_step_hermite is bracketed by HIP events recorded on the stream
 * it runs on (the bracket covers the pair kernel alone, not the pack before it
 * nor the split combine after it). nbody_timing_read waits for those events, returns the
 * number of bracketed launches and their summed duration in milliseconds, and
 * clears the record. Enabling or disabling also clears it. Not thread-safe:
 * meant for one measuring thread. */
nbody_status nbody_timing_enable(int32_t on);
nbody_status nbody_timing_read(int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
