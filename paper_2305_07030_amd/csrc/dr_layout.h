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
// local id and the fiber constants {EA / (2 L^2), L^2}.
#pragma once
#include <stdint.h>

namespace drk {

constexpr int kWave = 64;

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
    double pad;
};
static_assert(sizeof(ProbDesc) == 72, "ProbDesc layout");

struct KL {
    double k;  // EA / (2 L^2)
    double L2; // L^2
};

// Arguments of one batched solve (passed by value as the kernel argument).
struct SolveArgs {
    const ProbDesc *probs;    // [P]
    const int32_t *ids;       // [n_solve] problem of each solve slot (NULL: slot = problem)
    const int32_t *order;     // [n_solve] launch order of the slots (NULL: identity)
    const double *F;          // [n_solve * 9]
    int32_t n_solve;
    int32_t start;            // dr_start
    double tol;
    int64_t max_iter;
    // network (renumbered order)
    const double *X;          // [nodes * 3]
    const double *invm;       // [nodes]
    const double *mass;       // [nodes]
    const int32_t *deg;       // [nodes]
    const int32_t *slice_w;   // [slices]
    const int64_t *slice_off; // [slices], relative to the problem's inc_base
    const int32_t *nbr;       // [incidences]
    const KL *kl;             // [incidences]
    // state kept on the device between solves
    double *u;                // [nodes * 3] displacement (renumbered)
    double *F_last;           // [P * 9] F of the last solve of each problem
    int32_t *has_state;       // [P] 1 once a solve has written u
    // scratch for the global-placement kernel
    double *xg;               // [nodes * 4] positions (x, y, z, pad)
    double *wg;               // [nodes * 4] half-step velocities
    // results, per solve slot
    double *sigma;            // [n_solve * 9]
    double *sigma_fib;        // [n_solve * 9]
    int64_t *iters;           // [n_solve]
    double *rho;              // [n_solve]
    double *ke;               // [n_solve]
    int32_t *status;          // [n_solve]
};

// Launch shape of one batched solve.
struct LaunchPlan {
    int block;     // threads per workgroup
    int npt;       // nodes per thread (register-resident variant), 0 = global
    int lds_bytes; // dynamic LDS per workgroup
};

// Implemented in dr_kernels.hip.
int launch_solve(const SolveArgs &a, const LaunchPlan &plan, void *stream);
int launch_loop_iteration_kernels(const SolveArgs &a, int slot, int phase, int n_nodes,
                                  double *partial, double *out_scalars, int64_t n_done,
                                  void *stream);
const char *kernel_error_string(int code);

} // namespace drk
