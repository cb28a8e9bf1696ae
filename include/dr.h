/*
 * dr.h -- C ABI of libdr: batched dynamic relaxation (DR) of many small,
 * independent pin-jointed fiber networks on one AMD Instinct MI355X (gfx950).
 *
 * Method: Merson & Shephard, "Using Hierarchical Parallelism to Accelerate
 * the Solution of Many Small Partial Differential Equations".  Section II
 * states the sub-problem (a fiber network at a macroscale material point,
 * relaxed to static equilibrium by damped explicit pseudo-dynamics whose
 * force residual is monitored); section III, Fig. 1, gives the loop; section
 * I says each sub-problem hands constitutive information (here the volume
 * averaged Cauchy stress) back to the macroscale.
 *
 * Readings where the paper is silent, applied by every entry point below:
 *   fiber law    T = EA (lambda^2 - 1) / 2 along the current fiber direction;
 *   lumped mass  m_i = 1/2 sum of the lengths of the fibers at node i;
 *   time step    dt = dt_safety * 2 / w, w^2 = max over free nodes of
 *                (2 / m_i) sum_{f at i} 1.1 EA_f / L_f, constant per solve;
 *   damping      f_d = -c m v with c = damping * w;
 *   start        prescribed nodes u = (F - I) X; free nodes from the affine
 *                field (F - I) X, from zero, or warm (u_prev + (F - F_prev) X);
 *   residual     rho = |g_free| / max(|g_prescribed|, 1e-4 mean(EA)
 *                sqrt(3 max(N_B, 1))), tested after every pass of the
 *                repeat-until loop (so at least one pass is made);
 *   stress       sigma = 1/det(F) sum_{b prescribed} (-g_b) (x) (x_b - F c0),
 *                c0 = (1/2, 1/2, 1/2), reference volume 1 (the unit cube),
 *                row-major sigma[3 p + q] = sum r_p y_q; the fiber (virial)
 *                form sum_f T_f d_f (x) d_f / l_f / det(F) is returned too.
 *
 * Conventions shared by all entry points
 *   - Every call returns a dr_status; on error a message is available from
 *     dr_last_error() (thread-local, valid until the next libdr call on the
 *     same thread).  No C++ exception crosses this interface.
 *   - Pointers are host pointers unless the name says "_device".
 *   - Inputs are copied before the call returns; the caller keeps ownership
 *     of every array it passes and libdr never frees caller memory.
 *   - A dr_batch owns all device memory it allocates; dr_batch_destroy
 *     releases it (a batch made by dr_batch_create_in allocates none: its
 *     device arrays live in the caller's workspace).  A handle is used by one
 *     host thread at a time; all of its device work is ordered on the HIP
 *     stream given at creation.
 *   - F is a 3x3 deformation gradient, row-major, F[3 i + j] = dx_i / dX_j.
 *   - Node ids are the caller's (problem-local, 0-based) ids; u is always
 *     returned in the caller's node order.
 *   - Non-convergence is not a call error: it is reported per problem in
 *     `result` (dr_result).
 */
#ifndef DR_H
#define DR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dr_batch dr_batch; /* opaque handle, owned by libdr */

typedef enum {
    DR_OK = 0,
    DR_E_INVALID = -1, /* bad argument or network; message names it */
    DR_E_NOMEM = -2,   /* host or device allocation failed */
    DR_E_DEVICE = -3,  /* HIP runtime error (no device, launch failure, ...) */
    DR_E_STATE = -4    /* call out of order (e.g. dr_stress before dr_solve) */
} dr_status;

typedef enum {
    DR_CONVERGED = 0, /* rho <= tol */
    DR_MAX_ITER = 1,  /* max_iter passes made without reaching tol */
    DR_NONFINITE = 2, /* a residual or energy became NaN / Inf */
    DR_RUNNING = 3,   /* started by dr_advance and not finished yet */
    DR_IDLE = 4,      /* no solve has been started for this problem */
    DR_STALLED = 5,   /* rho made no 0.1 % progress for stall_window passes */
    DR_ENERGY = 6,    /* the energy balance check failed (energy_tol) */
    DR_ABORTED = 7    /* a group's barrier wait timed out (tail hand-off); the
                         problem's state is lost: start it again */
} dr_result;

typedef enum { DR_FP64 = 0, DR_FP32 = 1 } dr_precision;

typedef enum {
    DR_PLACE_AUTO = 0,   /* LDS when the largest problem fits, else global */
    DR_PLACE_LDS = 1,    /* positions in LDS, node state in registers */
    DR_PLACE_GLOBAL = 2  /* positions and velocities in device memory */
} dr_placement;

typedef enum {
    DR_RESUME = -1,      /* dr_advance only: continue the problem's running solve */
    DR_START_AFFINE = 0, /* free nodes start at (F - I) X (cold start) */
    DR_START_ZERO = 1,   /* free nodes start at u = 0 (Fig. 1, commented init) */
    DR_START_WARM = 2    /* u_prev + (F - F_prev) X from the problem's last solve */
} dr_start;

/*
 * A packed batch of networks (the paper's PackedView idea, section III:
 * one row-offset array plus one value array holding every sub-problem).
 *   n_problems          >= 1
 *   node_offsets        [n_problems + 1], non-decreasing, node_offsets[0] = 0
 *   fiber_offsets       [n_problems + 1], non-decreasing, fiber_offsets[0] = 0
 *   X                   [total_nodes * 3] reference coordinates, xyz
 *                       interleaved, finite; the network lives in the unit cube
 *   fiber_nodes         [total_fibers * 2] problem-local node ids (a, b), a != b
 *   EA                  [total_fibers] finite and > 0
 *   fixed               [total_nodes] 1 = prescribed node, 0 = free; or NULL:
 *                       then the band rule below decides
 *   band                used when fixed is NULL (finite, >= 0): a node is
 *                       prescribed iff it lies within `band` of a face of the
 *                       unit cube, min_k min(X_k, 1 - X_k) <= band (inclusive);
 *                       ignored when fixed is given
 * Each problem needs 1 .. 524288 nodes (the global-placement kernel keeps a
 * problem's 64-node slice headers in LDS), every free node needs >= 1 fiber
 * and every fiber a nonzero reference length.
 */
typedef struct {
    int32_t n_problems;
    const int64_t *node_offsets;
    const int64_t *fiber_offsets;
    const double *X;
    const int32_t *fiber_nodes;
    const double *EA;
    const uint8_t *fixed;
    double band;
} dr_networks;

/*
 * Solver options (see the readings above).
 *   precision   DR_FP64 (FP64 state) or DR_FP32 (FP32 nodal state and force
 *               gather, FP64 norm reductions and stress)
 *   tol         > 0, convergence threshold on rho
 *   max_iter    >= 1, cap on DR passes per solve
 *   damping     >= 0, c = damping * w (dimensionless)
 *   dt_safety   in (0, 1], dt = dt_safety * 2 / w
 *   block       threads per workgroup: 0 = automatic, else 256, 512 or 1024
 *   placement   a dr_placement value; DR_PLACE_LDS is rejected at creation
 *               when the largest problem does not fit (3 * 8 B per node of
 *               LDS, at most 8 nodes per thread).  A problem of more than
 *               6720 nodes is packed in spatial tiles of 1024 nodes, and
 *               the FP64 global placement with 1024 threads and chunks of 1
 *               (the automatic choice for such problems, also in groups)
 *               stages each tile's states and those of its halo in LDS
 *               before gathering; the results are the same bits as the
 *               other global builds'.
 *   chunk       incidences per step of the force gather, whose loads are
 *               issued one step ahead: 0 = automatic, else 1, 2 or 4 (a
 *               tuning knob; results do not depend on it).  Global placement
 *               with 256 threads runs chunks of 1 only: DR_PLACE_GLOBAL with
 *               block 256 and chunk 2 or 4 is rejected (DR_E_INVALID); in the
 *               automatic split the global class then runs chunks of 1
 *               (dr_batch_class_info reports each class's chunk)
 *   stall_window  >= 0; 0 = off.  Otherwise a solve also ends (DR_STALLED)
 *               when its best residual has not improved by 0.1 % during the
 *               last stall_window passes.  Not part of the paper's loop: a
 *               guard for the FP32 state, whose force rounding puts a floor
 *               under the reachable residual.
 *   energy_tol  >= 0; 0 = off.  Otherwise the energy balance is tracked
 *               (Fig. 1, the optional check): the work of the internal
 *               forces W (trapezoid per pass), the work dissipated by damping
 *               D (half-step velocity over the step) and the kinetic energy
 *               KE; every 1024 passes and at the end of a launch a solve ends
 *               (DR_ENERGY) when |KE - W + D| > energy_tol * max(KE, |W|, D).
 *               The explicit scheme balances to a few percent in the first
 *               passes and to ~1e-3 later, so a useful tolerance is ~0.1.
 *               Costs 32 B of traffic per free node per pass; dr_energy
 *               reports W and D.
 *   tail_at     0..256; 0 = off.  Tail hand-off (section III: sub-problems
 *               converge at different rates, which leaves a launch waiting
 *               for its slowest ones): once at most tail_at problems of a
 *               launch are still running, each of them saves its exact state
 *               at its next check (every 256 passes) and a cooperative launch
 *               of the same call finishes them with tail_group workgroups per
 *               problem (global placement; the members of a group meet at a
 *               barrier in device memory every pass).  Every node's
 *               arithmetic is the same as in one workgroup; only the residual
 *               norms are summed in another order, which could move the
 *               stopping pass only if their last bits decided the test.
 *               Not used under dr_graph_capture.  The group launch needs all
 *               its workgroups resident at once: work from another batch or
 *               stream that holds compute units meanwhile can keep members
 *               out, and a group whose members do not all arrive within the
 *               barrier's 2 s wait ends its problem with DR_ABORTED (no
 *               kernel hangs).
 *   tail_group  0 = automatic (the most workgroups per problem, up to 16, that
 *               let tail_at problems be resident at once), else 2..16;
 *               DR_E_INVALID at creation when tail_at x tail_group workgroups
 *               cannot be resident at once.  With dt_rule 1 (which has no
 *               hand-off): 2..16 runs every problem of a call in a group of
 *               tail_group workgroups of 1024 threads from the start (one
 *               cooperative launch, one size class; the same bits as one
 *               workgroup per problem at a fixed pass count).  At most 256
 *               problems per call (DR_E_DEVICE otherwise), and
 *               8 x tail_group x ceil(n / 8) workgroups must fit on the
 *               device at once (the runtime refuses the launch otherwise:
 *               DR_E_DEVICE); size-class plans are DR_E_INVALID.
 *   dt_rule     0 = one constant step per solve (Fig. 1's "compute next
 *               time step" read as fixed for the solve); 1 = a step per
 *               pass from the current state: dt_n = min(dt_{n-1},
 *               dt_safety * 2 / w), w^2 = max over free nodes i of
 *               (2 / m_i) sum_{f at i} EA_f l_f / L_f^2 (axial tangent
 *               stiffness at the current length), from dt_0 = the constant
 *               step; the step never grows back.  Identical results wherever
 *               the step stays dt0; a fiber stretched beyond the constant
 *               step's headroom no longer makes the iteration diverge.  Runs
 *               its own kernel (global placement, 24 B more per node of
 *               device memory); FP64 only, and not with energy_tol, tail_at
 *               or the launch-loop comparator (DR_E_INVALID).
 */
typedef struct {
    int32_t precision;
    double tol;
    int64_t max_iter;
    double damping;
    double dt_safety;
    int32_t block;
    int32_t placement;
    int32_t chunk;
    int64_t stall_window;
    double energy_tol;
    int32_t tail_at;
    int32_t tail_group;
    int32_t dt_rule;
} dr_options;

/* Fills *opt with the defaults: FP64, tol 1e-8, max_iter 2000000,
 * damping 1e-3, dt_safety 0.9, block 0, placement DR_PLACE_AUTO, chunk 0,
 * stall_window 0, energy_tol 0, tail_at 0, tail_group 0, dt_rule 0. */
void dr_options_default(dr_options *opt);

/*
 * Validates and packs the networks (Fig. 1 steps 1-3: edge connectivity,
 * connectivity array, transfer to the device; step 5: lumped mass), computes
 * dt, c and the residual floor per problem, and uploads everything to HBM.
 *   nets, opt     read only; copied
 *   hip_stream    a hipStream_t (NULL = the default stream); all later device
 *                 work of the batch is enqueued on it
 *   out           receives the new handle (NULL on failure)
 * Errors: DR_E_INVALID (the message names problem and element), DR_E_NOMEM,
 * DR_E_DEVICE.  Validation runs before any HIP call.
 */
dr_status dr_batch_create(const dr_networks *nets, const dr_options *opt,
                          void *hip_stream, dr_batch **out);

/*
 * Device bytes a batch of these networks and options needs when it is made
 * with dr_batch_create_in (every device array of the batch, each rounded up
 * to 256 bytes).  Validates and packs on the host like dr_batch_create and
 * makes no HIP call (usable without a device).
 *   bytes   receives the size (0 on failure)
 * Errors: as dr_batch_create's validation.
 */
dr_status dr_batch_workspace_bytes(const dr_networks *nets, const dr_options *opt,
                                   size_t *bytes);

/*
 * As dr_batch_create, with every device array of the batch carved from a
 * caller-owned device buffer (for callers whose memory comes from their own
 * allocator, e.g. a framework tensor); the library allocates no device
 * memory for this batch, also not later.  Pinned host staging buffers,
 * streams and events are still the library's.
 *   device_workspace  device memory of the current device, 256-byte aligned;
 *                     the caller owns it, must keep it alive and untouched
 *                     until dr_batch_destroy, and frees it afterwards
 *   workspace_bytes   its size, at least dr_batch_workspace_bytes
 * Errors: DR_E_INVALID (as dr_batch_create; NULL, unaligned, foreign or too
 * small workspace, the message gives the size needed), DR_E_DEVICE.
 */
dr_status dr_batch_create_in(const dr_networks *nets, const dr_options *opt,
                             void *hip_stream, void *device_workspace,
                             size_t workspace_bytes, dr_batch **out);

/*
 * Enqueues one DR solve (Fig. 1 steps 4, 6, 7 and the loop, then the stress
 * average) for the problems listed in ids, asynchronously on the stream.
 *   F       [n_ids * 9] host, F of ids[k] at F + 9 k; copied before return
 *   ids     [n_ids] distinct problem indices in [0, n_problems), or NULL for
 *           all problems in order (n_ids must then equal n_problems)
 *   start   a dr_start value; DR_START_WARM uses the state the problem's
 *           previous solve left on the device (affine if it has none)
 * Errors: DR_E_INVALID (bad ids / F not finite / det F <= 0), DR_E_DEVICE.
 */
dr_status dr_solve(dr_batch *b, const double *F, const int32_t *ids,
                   int32_t n_ids, int32_t start);

/*
 * As dr_solve, with F_device [n_ids * 9] already in device memory; ids is a
 * host array as in dr_solve (NULL = all problems in order).  F_device must
 * stay valid until the solve has finished on the stream; F is not checked on
 * the host (a non-finite F ends that problem with DR_NONFINITE).
 */
dr_status dr_solve_device(dr_batch *b, const double *F_device, const int32_t *ids,
                          int32_t n_ids, int32_t start);

/*
 * Waits for the last dr_solve / dr_solve_device / dr_solve_loop / dr_advance
 * and returns its results in the order of that call's ids.  Any output may
 * be NULL.
 *   sigma      [n_ids * 9]  boundary (reaction) form of the Cauchy stress
 *   sigma_fib  [n_ids * 9]  fiber (virial) form
 *   u          [total_nodes * 3] displacements of ALL problems of the batch
 *              (each problem's last finished solve), caller node order
 *   result     [n_ids] dr_result
 *   iters      [n_ids] DR passes made
 *   resid      [n_ids] final rho
 *   ke         [n_ids] final kinetic energy 1/2 sum m |v|^2
 * Errors: DR_E_STATE (no solve yet), DR_E_DEVICE.
 */
dr_status dr_stress(dr_batch *b, double *sigma, double *sigma_fib, double *u,
                    int32_t *result, int64_t *iters, double *resid, double *ke);

/*
 * Iteration-level continuous batching: one launch that advances every listed
 * problem by at most `budget` DR passes, asynchronously.  Slot k works on
 * problem ids[k]:
 *   starts[k] a dr_start value  -> a new solve with F + 9 k (host array);
 *   starts[k] == DR_RESUME      -> continues the problem's running solve from
 *                                  the state saved in HBM (F + 9 k ignored).
 * A solve that reaches tol, max_iter or a non-finite value finishes inside the
 * launch (displacements, scalars and stress are then final); one that spends
 * the budget saves its exact state, so a solve split over several launches
 * gives the same bits as one dr_solve.  A problem's arithmetic does not
 * depend on the other slots of the launch.
 * Errors: DR_E_INVALID (ids out of range or repeated, DR_RESUME for a problem
 * that is not running, budget < 1, F of a new solve not finite or det <= 0),
 * DR_E_DEVICE.
 */
dr_status dr_advance(dr_batch *b, const double *F, const int32_t *ids, const int32_t *starts,
                     int32_t n_ids, int64_t budget);

/*
 * As dr_advance with a pass budget per slot: slot k may make at most
 * budgets[k] (>= 1) passes in this launch.  A scheduler gives slow problems
 * (many fibers, global placement) smaller budgets than fast ones so that
 * every slot of the launch finishes its budget at about the same time and no
 * compute unit waits for the slowest.  Errors as dr_advance (DR_E_INVALID
 * for budgets NULL or a budget < 1).
 */
dr_status dr_advance_each(dr_batch *b, const double *F, const int32_t *ids, const int32_t *starts,
                          const int64_t *budgets, int32_t n_ids);

/*
 * Waits for the batch's stream and returns the current results of the
 * listed problems (host array ids [n_ids]); any output may be NULL.  result
 * is DR_RUNNING for a solve still in progress (iters / resid / ke then
 * describe its last pass and sigma is not yet valid) and DR_IDLE for a
 * problem never solved.  Same layouts as dr_stress.
 */
dr_status dr_results(dr_batch *b, const int32_t *ids, int32_t n_ids, double *sigma,
                     double *sigma_fib, int32_t *result, int64_t *iters, double *resid,
                     double *ke);

/*
 * Energy balance of the last solve of each given problem (batch created with
 * energy_tol > 0; DR_E_STATE otherwise): work_int[k] = W, the work done by
 * the internal forces since the solve started, and work_damp[k] = D, the
 * work dissipated by the damping force; with the kinetic energy KE from
 * dr_results, KE - W + D is the balance error.  For a running solve the
 * values are those at the end of its last launch.  Waits for the stream.
 */
dr_status dr_energy(dr_batch *b, const int32_t *ids, int32_t n_ids, double *work_int,
                    double *work_damp);

/* Blocks until all work enqueued on the batch's stream has finished. */
dr_status dr_sync(dr_batch *b);

/*
 * Per-problem launch loop (the paper's "naive" design, section III): the same
 * iteration as dr_solve, run for one problem at a time with a few kernel
 * launches per DR pass and the residual read back and tested on the host
 * after every pass.  Comparator only; same arguments and results as
 * dr_solve followed by dr_stress for the given ids, and synchronous.  FP64
 * batches only (DR_E_INVALID for a DR_FP32 batch).
 */
dr_status dr_solve_loop(dr_batch *b, const double *F, const int32_t *ids,
                        int32_t n_ids, int32_t start);

/*
 * As dr_solve_loop, with the paper's own force kernel (section III): the
 * nodal forces are zeroed each pass and every fiber, evaluated once, adds
 * its force to both ends with FP64 atomic additions.  The order of those
 * additions varies from run to run, so results agree with dr_solve_loop to
 * round-off and are not bitwise reproducible.  Comparator only, FP64 only;
 * the first call allocates a force buffer of 32 B per node of the largest
 * problem (DR_E_DEVICE if that fails).
 */
dr_status dr_solve_loop_scatter(dr_batch *b, const double *F, const int32_t *ids,
                                int32_t n_ids, int32_t start);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * dr_solve_loop_scatter, but its scratch (the force accumulators, the
 * per-block partial sums and the reduced scalars) lives in one fixed device
 * array of the library (6.3 MB, one per GPU, held until the process ends)
 * instead of the batch's buffers, and the call allocates nothing.  Every
 * problem in ids must have at most 262144 nodes (DR_E_INVALID otherwise).
 * All calls on one GPU share that array: calls that overlap on one GPU (from
 * several threads or batches) race, and must be serialised by the caller.
 * The accumulators are cleared every pass, so nothing carries over from the
 * previous call.  Same inputs, outputs and errors as dr_solve_loop_scatter
 * otherwise (DR_E_DEVICE if the array's address cannot be looked up).
 */
dr_status dr_solve_loop_scatter_noalloc(dr_batch *b, const double *F, const int32_t *ids,
                                        int32_t n_ids, int32_t start);

/* Information about the packed batch and the launch chosen for it.
 *   n_problems, total_nodes, total_fibers, block (threads per workgroup),
 *   lds_bytes (dynamic LDS per workgroup), nodes_per_thread. Any may be NULL. */
dr_status dr_batch_info(const dr_batch *b, int32_t *n_problems, int64_t *total_nodes,
                        int64_t *total_fibers, int32_t *block, int32_t *lds_bytes,
                        int32_t *nodes_per_thread);

/*
 * Per-problem derived scalars computed at creation: dt, c and the residual
 * floor, each [n_problems] (any may be NULL).  Host only.
 */
dr_status dr_batch_scalars(const dr_batch *b, double *dt, double *c, double *s_floor);

/*
 * The library's estimate of the time one DR pass of each problem takes alone
 * on one compute unit, in the placement of its size class (seconds,
 * [n_problems]; a model fitted to MI355X measurements: about 1.5 us + 0.65 ns
 * per fiber in LDS placement, 2.2 us + 2.0 ns per fiber in global placement,
 * 4.8 ns per fiber beyond 38k fibers).  Schedulers use it to size per-slot
 * budgets (dr_advance_each); the serving pool does.  Host only.
 */
dr_status dr_batch_pass_costs(const dr_batch *b, double *seconds);

/*
 * Size classes.  A batch splits its problems by node count into classes; each
 * class has one launch shape (threads per workgroup, nodes per thread, gather
 * chunk, placement) used for every solve of the batch, and the classes of a
 * launch run concurrently on internal streams.  By default: the largest set
 * of problems the LDS / register variant can hold, then the rest in global
 * placement.  A problem's result depends neither on its class's shape nor on
 * which other problems share a launch.  Classes that would hold no problem
 * of the batch are dropped, so every listed class has n_problems > 0.
 *
 * dr_batch_class_info: class c in [0, *n_classes); any output may be NULL.
 *   n_lo, n_hi       node counts covered (inclusive)
 *   n_problems       problems of the batch in the class
 *   block, nodes_per_thread (0 = global placement), chunk, lds_bytes
 */
dr_status dr_batch_class_info(const dr_batch *b, int32_t c, int32_t *n_classes, int32_t *n_lo,
                              int32_t *n_hi, int32_t *n_problems, int32_t *block,
                              int32_t *nodes_per_thread, int32_t *chunk, int32_t *lds_bytes);

/*
 * Replaces the size classes (the autotuner's entry point): class k covers the
 * node counts (n_hi[k-1], n_hi[k]] with the given block (0/256/512/1024),
 * chunk (0/1/2/4) and placement (dr_placement); problems above n_hi[n-1] get the
 * automatic split.  n_hi must increase.  Every launch shape computes the
 * same per-node arithmetic in the same order, so results do not depend on
 * the plans and they may be changed at any time: the call waits for the
 * batch's queued work and drops a graph captured with dr_graph_capture.
 * DR_E_INVALID when a DR_PLACE_LDS class cannot hold its largest problem.
 */
dr_status dr_set_class_plans(dr_batch *b, int32_t n_classes, const int32_t *n_hi,
                             const int32_t *block, const int32_t *chunk, const int32_t *placement);

/*
 * Captures one solve step (as dr_solve_device with these arguments: F_device
 * [n_ids * 9] in device memory, host ids or NULL for all, start mode) into a
 * HIP graph held by the batch, replacing any earlier capture; dr_graph_launch
 * replays it on the batch stream (re-staging the slot lists first).  The
 * batch must have been created on a non-default stream (DR_E_STATE).  The
 * results of a replay are read with dr_stress as after dr_solve.
 */
dr_status dr_graph_capture(dr_batch *b, const double *F_device, const int32_t *ids, int32_t n_ids,
                           int32_t start);
dr_status dr_graph_launch(dr_batch *b);

/* Releases the handle and its device memory (waits for its stream first).
 * NULL is ignored. */
void dr_batch_destroy(dr_batch *b);

/*
 * Serving pool (section I: the macroscale's material points request solves
 * of their sub-problems; here a resident pool of networks served by
 * iteration-level continuous batching over dr_advance).  A handle is used
 * from one thread at a time.
 *
 * dr_pool_create: a batch of the networks (as dr_batch_create) plus an empty
 * request queue.
 *   state_budget_bytes  cap on the running state of in-flight solves, 0 =
 *                       none.  The running state of a solve is
 *                       dr_state_bytes_per_node bytes per node of its network
 *                       (two state records and one velocity record).  With a
 *                       budget below that of all networks together, the pool
 *                       allocates the running state as one device arena of
 *                       state_budget_bytes and places each admitted solve in a
 *                       contiguous run of it until the solve retires, so the
 *                       budget bounds the device memory of in-flight solves
 *                       (topology, masses and last displacements of every
 *                       network stay resident: they are the pool)
 *   max_slots           cap on in-flight solves (>= 1)
 *   tick_passes         length of a poll's launch, in DR passes of the pool's
 *                       cheapest network (>= 1); every in-flight solve makes
 *                       as many passes as fit that time by
 *                       dr_batch_pass_costs (at least 1), so a tick's compute
 *                       units finish together and a tick stays short whatever
 *                       mix is in flight
 * Errors: as dr_batch_create, DR_E_INVALID for the caps (a budget below one
 * node's running state).
 */
typedef struct dr_pool dr_pool;
dr_status dr_pool_create(const dr_networks *nets, const dr_options *opt, void *hip_stream,
                         int64_t state_budget_bytes, int32_t max_slots, int64_t tick_passes,
                         dr_pool **out);

/*
 * Queues a request: solve network id at F[9] (host, row-major; copied), warm
 * started from the displacements its previous solve left on the device
 * (affine if none); tag is returned with the result.  Requests of one
 * network are served in submission order, one at a time.
 * Errors: DR_E_INVALID (id out of range, F not finite or det F <= 0, the
 * network alone over the state budget).
 */
dr_status dr_pool_submit(dr_pool *pool, int32_t id, const double *F, int64_t tag);

/*
 * One scheduling step: admits queued requests first come first served (a
 * request whose network is in flight waits without blocking the queue; one
 * that exceeds the slot or budget cap, or finds no free run of the arena
 * long enough for its network, blocks it), runs one launch over every
 * in-flight solve (as many passes as fit tick_passes passes of the pool's
 * cheapest network; new ones start, the others
 * resume from their exact saved state: a result is the same bits as one
 * dr_solve with DR_START_WARM), waits for it, and retires the finished
 * solves.  Then returns up to max_out finished requests, oldest first (the
 * rest stay for later polls); any output may be NULL:
 *   tags [max_out], ids [max_out], sigma [max_out * 9], result [max_out]
 *   (dr_result), iters [max_out]; *n_out = number returned.
 * With nothing queued or in flight it only returns finished requests.
 * Errors: DR_E_INVALID, DR_E_DEVICE.
 */
dr_status dr_pool_poll(dr_pool *pool, int32_t max_out, int64_t *tags, int32_t *ids, double *sigma,
                       int32_t *result, int64_t *iters, int32_t *n_out);

/* Counts of queued, in-flight and finished-but-unreturned requests and the
 * running-state bytes in flight; any output may be NULL. */
dr_status dr_pool_status(const dr_pool *pool, int32_t *queued, int32_t *in_flight,
                         int32_t *completed, int64_t *state_bytes);

/* Releases the pool and its batch (waits for its stream).  NULL is ignored. */
void dr_pool_destroy(dr_pool *pool);

/* Device bytes of running state that one node of an in-flight solve needs
 * (the unit of a pool's state budget): 72 for DR_FP64 (two 24-byte state
 * records and a 24-byte velocity record), 80 for DR_FP32 (two 32-byte state
 * records and a 16-byte velocity record).  Host only.
 * Errors: DR_E_INVALID (NULL bytes, unknown precision). */
dr_status dr_state_bytes_per_node(int32_t precision, int64_t *bytes);

/* Message of the last failed call on this thread ("" if none). */
const char *dr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DR_H */
