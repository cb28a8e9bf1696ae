// Device data layout shared by the host packer (dr_host.cpp) and the HIP
// kernels (dr_kernels.hip).  Everything a batch needs lives in a few flat
// device arrays indexed through per-problem offsets: the "packed view" of
// section III (one offset array plus one value array for all sub-problems).
//
// Node order inside a problem (section III: prescribed degrees of freedom
// reordered to a trailing block so the update loops touch only free ones):
//   [free nodes][prescribed nodes], each block sorted by degree (descending)
//   and, within one degree, by a spatial (Morton) key.
//
// Fiber incidences (node -> fiber map, two per fiber) are stored sliced-ELL
// with slices of 64 consecutive nodes = one wavefront: slice q of a problem
// holds width_q * 64 entries, entry (k, lane) at slice_off[q] + k * 64 + lane,
// k < width_q = the largest degree in the slice.  Within a node the
// incidences follow ascending fiber id.  Each entry carries the neighbour's
// local id and the fiber constants: {EA / (2 L^2), L^2} in FP64, and for the
// FP32 state {dX (the reference vector to the neighbour), EA / (2 L^2)}.
// Padding entries of a node (its degree up to the slice width) hold zero
// constants and a neighbour at a positive distance (the node's first real
// neighbour), so they add exactly zero force; lanes past the problem's last
// node hold neighbour 0 and zero constants.  The L^2 of an incidence is
// rounded as the kernels form squared lengths, fma(dz, dz, fma(dy, dy,
// dx * dx)).
#pragma once
#include <stdint.h>

namespace drk {

constexpr int kWave = 64;
// Largest slice count of one problem: the global-placement kernel keeps the
// problem's slice headers (16 B each) in LDS, so a problem has at most
// 64 * kGlbHdrMax = 524288 nodes.
constexpr int kGlbHdrMax = 8192;

// Per-problem status values beyond dr_result: a solve that has been started
// and stopped at a pass budget, and a problem with no solve yet.
constexpr int kStatusRunning = 3;
constexpr int kStatusIdle = 4;
constexpr int kStatusStalled = 5;
constexpr int kStatusEnergy = 6;
constexpr int kStatusAborted = 7; // a group barrier's wait timed out

// Workgroup groups: at most kGroupMax workgroups share one problem, at most
// kTailMax problems go to one group launch.
constexpr int kGroupMax = 16;
constexpr int kTailMax = 256;

// Slot start codes: a dr_start value starts a new solve; kResume continues
// the problem's running solve from the state saved in HBM.
constexpr int kResume = -1;

struct ProbDesc {
    int32_t N;          // nodes
    int32_t N_free;     // free nodes (local ids [0, N_free))
    int32_t n_slices;   // ceil(N / 64)
    int32_t M;          // fibers
    int64_t node_base;  // first node in the per-node arrays
    int64_t slice_base; // first slice in the per-slice arrays
    int64_t inc_base;   // first entry in the per-incidence arrays
    double dt;          // pseudo-time step
    double c;           // mass-proportional damping coefficient
    double s_floor;     // residual denominator floor
    int64_t n_inc;      // per-incidence entries of the problem (slices x 64 x width)
    int32_t n_tiles;    // tiles of kTile nodes with halos (0: the problem has none)
    int32_t tile_pad;
    int64_t tile_base;  // first entry of the problem in the per-tile halo offsets
    int64_t halo_base;  // first entry of the problem in the halo node ids
};
static_assert(sizeof(ProbDesc) == 96, "ProbDesc layout");

// Tiles of the global placement's staged gather: kTile consecutive nodes
// (one per thread of a 1024-thread workgroup, one row of each wave), a
// problem is tiled when it is too large for the LDS variant (more than
// kTiledMinNodes nodes).  A tile's halo (the nodes outside it that its
// incidences reach) holds at most kHaloMax nodes.
constexpr int kTile = 1024;
constexpr int kTiledMinNodes = 6720;
constexpr int kHaloMax = 4096;

struct KL {
    double k;  // EA / (2 L^2)
    double L2; // L^2
};

struct KL32 {
    float dx, dy, dz; // X_neighbour - X_node
    float k;          // EA / (2 L^2)
};

// Arguments of one batched launch (passed by value as the kernel argument).
struct SolveArgs {
    const ProbDesc *probs;    // [P]
    const int32_t *ids;       // [n_solve] problem of each slot (NULL: slot = problem)
    const int32_t *order;     // [n_solve] launch order of the slots (NULL: identity)
    const int32_t *starts;    // [n_solve] dr_start of a new solve, or kResume (NULL: start)
    const double *F;          // [n_solve * 9] F of the slots that start a solve
    int32_t n_solve;
    int32_t start;            // dr_start used when starts == NULL
    double tol;
    int64_t max_iter;         // cap on the passes of one solve
    int64_t budget;           // cap on the passes made in this launch
    const int64_t *budgets;   // [P] per-problem cap for this launch (NULL: budget)
    int64_t stall_window;     // 0 = off, else passes without progress that end a solve
    double energy_tol;        // 0 = off, else the energy-balance check (enode, e_work, e_damp)
    // network (renumbered order)
    const double *X;          // [nodes * 3]
    const double *invm;       // [nodes]
    const double *mass;       // [nodes]
    const float *invm32;      // [nodes] (FP32 state)
    const float *mass32;      // [nodes] (FP32 state)
    const int32_t *deg;       // [nodes]
    const int32_t *slice_w;   // [slices]
    const int64_t *slice_off; // [slices], relative to the problem's inc_base
    const int32_t *nbr;       // [incidences]
    const KL *kl;             // [incidences]
    const KL32 *kl32;         // [incidences] (FP32 state)
    // state kept on the device
    double *u;                // [nodes * 3] displacement of the last finished solve
    const int64_t *state_off; // [P] first record of the problem in qbuf / wbuf
                              //   (its node_base, or its place in a pool's arena)
    double *qbuf;             // [2 * qhalf] running state, two buffers of qhalf
                              //   doubles: positions (FP64, 24 B per node) or
                              //   displacements and their compensation terms
                              //   (FP32, 32 B per node); the state after pass k
                              //   is in buffer k & 1
    int64_t qhalf;            // doubles per state buffer (3 or 4 per record)
    double *wbuf;             // running half-step velocities (24 B per record in
                              //   FP64, 16 B in FP32)
    double *F_cur;            // [P * 9] F of the current solve
    double *F_last;           // [P * 9] F of the last finished solve
    int32_t *has_state;       // [P] 1 once a solve has finished
    // results, per problem
    double *sigma;            // [P * 9]
    double *sigma_fib;        // [P * 9]
    int64_t *iters;           // [P] passes of the current / last solve
    double *rho_best;         // [P] best residual of the running solve (stall guard)
    int64_t *n_best;          // [P] pass at which it was reached
    double *rho;              // [P]
    double *ke;               // [P]
    int32_t *status;          // [P] dr_result, kStatusRunning or kStatusIdle
    double *enode;            // [nodes * 4] energy terms per free node (energy_tol > 0):
                              //   sum g.(w_old + w_new), sum m |w_old|^2, last g.w_new
    double *e_work;           // [P] work of the internal forces of the last / running solve
    double *e_damp;           // [P] work dissipated by damping
    // tail hand-off: once at most tail_at problems of a launch still run,
    // each leaves its workgroup (state saved) at its next check and joins the
    // tail list; a group launch then finishes them with `group` workgroups each
    int32_t tail_at;          // 0 = off
    int32_t *live;            // [1] problems of the launch not finished (tail_at > 0)
    int32_t *tail_list;       // [kTailMax] problems handed off
    int32_t *tail_count;      // [1] entries of tail_list
    int64_t *n_begin;         // [P] pass count at which a handed-off solve's launch began
    int32_t group;            // workgroups per problem of a group launch
    uint32_t *gbar;           // [kTailMax] barrier counters of the groups
    int32_t *gabort;          // [kTailMax] abort flags of the groups
    double *gpart;            // [kTailMax * 2 * kGroupMax * 4] partial sums of the groups
    const uint16_t *lslot;    // per incidence: the neighbour's slot in its tile's staged records
    const int32_t *tile_halo; // per tile (+1 per problem): first entry of its halo in halo_ids
    const int32_t *halo_ids;  // halo node ids (local to the problem)
    int32_t tile_hmax;        // largest halo of the batch's tiles (0: no tiled problem)
    // per-pass time step (dt_rule = 1): the step's safety factor, the
    // acceleration records and the step of each running solve's next pass
    int32_t dt_rule;          // 0 = constant step, 1 = per-pass step (k_dr_dtp)
    double dt_safety;
    double *abuf;             // [records * 3] accelerations (dt_rule = 1)
    double *dt_next;          // [P] step of the next pass of a running solve (dt_rule = 1)
};

// Launch shape of one batched solve.
struct LaunchPlan {
    int block;     // threads per workgroup
    int npt;       // nodes per thread (register-resident variant), 0 = global
    int lds_bytes; // dynamic LDS per workgroup
    int chunk;     // incidences per pipelined gather step (1, 2 or 4)
    int fp32;      // 1: FP32 nodal state and force gather
};

// Implemented in dr_kernels.hip.
int launch_solve(const SolveArgs &a, const LaunchPlan &plan, void *stream);
// Launch-loop comparator: phase 0 set-up, 1 one gather pass, 3 one pass with
// the zero + atomic-scatter force kernel (gbuf: 3 doubles per node), 2 finish.
int launch_loop_kernels(const SolveArgs &a, int slot, int phase, int n_nodes, double *partial,
                        double *out_scalars, int64_t n_done, double rho, double ke, int status,
                        double *gbuf, void *stream);
int launch_fill_i32(int32_t *p, int32_t value, int64_t n, void *stream);
// The per-pass time-step kernel (global placement, FP64) with `block`
// threads per workgroup (256, 512 or 1024).
// The per-pass step kernel; a.group > 1: its group form (a.group workgroups
// of 1024 threads per solve slot, a cooperative launch).
int launch_dtp(const SolveArgs &a, int block, void *stream);
// The group launch of the tail hand-off (cooperative: all its workgroups are
// co-resident) for up to n_groups handed-off problems, then the stress of the
// problems it finished; plan.block is the workgroup size (512 or 1024),
// plan.lds_bytes its LDS, a.group the workgroups per problem.
int launch_tail(const SolveArgs &a, const LaunchPlan &plan, int n_groups, void *stream);
// Workgroups of the group kernel (fp32, block, lds_bytes) that the current
// device holds at once.
int group_grid_capacity(int fp32, int block, int lds_bytes, int *capacity);
// Workgroups in a group launch for n_groups groups of G members: whole
// rounds of 8 groups (one per XCD).
inline int group_grid(int n_groups, int G) { return 8 * G * ((n_groups + 7) / 8); }
const char *kernel_error_string(int code);

// Allocation-free launch loop: the scratch of one problem's solve (force
// accumulators of the atomic scatter, per-block partial sums, the reduced
// scalars) in a fixed device array of the library, for problems of at most
// kNoAllocMaxNodes nodes.  Byte offsets within it:
constexpr int kNoAllocMaxNodes = 262144;
constexpr size_t kNoAllocForceOff = 0;
constexpr size_t kNoAllocPartialOff = 3 * sizeof(double) * (size_t)kNoAllocMaxNodes;
constexpr size_t kNoAllocScalarOff =
    kNoAllocPartialOff + ((3 * sizeof(double) * (size_t)(kNoAllocMaxNodes / 256 + 2) + 255) / 256) * 256;
constexpr size_t kNoAllocScratchBytes = kNoAllocScalarOff + 256;
// Device address of that array on the current device (looked up once per
// device); 0 or a hipError_t.
int noalloc_scratch(void **ptr);


} // namespace drk
