// libdr host side: argument validation, packing of a batch of networks into
// the device layout of dr_layout.h, per-problem constants, launch planning,
// result retrieval, and the per-problem launch-loop comparator.
//
// Section III of the paper: the networks are packed once (edge connectivity,
// connectivity array, one transfer to the device; prescribed degrees of
// freedom reordered to a trailing block) and every later solve of the batch
// is one kernel launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/dr.h"
#include "dr_layout.h"

using drk::KL;
using drk::KL32;
using drk::LaunchPlan;
using drk::ProbDesc;
using drk::SolveArgs;

namespace {

thread_local std::string g_err;

dr_status fail(dr_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHECK(expr)                                                                            \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(DR_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,   \
                        __LINE__);                                                                \
    } while (0)

constexpr int kLdsLimit = 160 * 1024;
constexpr int kMaxNpt = 8;

// Running-state records of one in-flight solve, per node: two state buffers
// (the state after pass k lives in buffer k & 1) of 3 doubles (FP64 position)
// or 4 doubles (FP32 state and its compensation terms), and one half-step
// velocity record of 3 doubles (FP64) or 2 (FP32: 4 floats).
int64_t state_doubles(int precision) { return precision == DR_FP32 ? 4 : 3; }
int64_t velocity_doubles(int precision) { return precision == DR_FP32 ? 2 : 3; }
int64_t state_bytes_per_node(int precision)
{
    return 8 * (2 * state_doubles(precision) + velocity_doubles(precision));
}

// Host copy of one packed problem's node permutation (caller id -> local id).
struct HostProblem {
    int32_t N, N_free, M;
    int64_t in_node_base; // caller's node offset
    std::vector<int32_t> new_of_old;
};

} // namespace

struct dr_batch {
    dr_options opt{};
    hipStream_t stream = nullptr;
    int device = 0;
    int32_t P = 0;
    int64_t total_nodes = 0, total_fibers = 0, total_slices = 0, total_inc = 0;
    int32_t n_max = 0;
    // running-state records (qbuf, wbuf): one per node of the batch, or a
    // pool's arena of fewer records that in-flight solves are placed in
    int64_t state_nodes = 0;
    std::vector<HostProblem> hp;
    std::vector<ProbDesc> desc;
    // device arrays: network
    ProbDesc *d_probs = nullptr;
    double *d_X = nullptr, *d_invm = nullptr, *d_mass = nullptr;
    float *d_invm32 = nullptr, *d_mass32 = nullptr;
    int32_t *d_deg = nullptr, *d_slice_w = nullptr, *d_nbr = nullptr;
    uint16_t *d_lslot = nullptr;
    int32_t *d_tile_halo = nullptr, *d_halo_ids = nullptr;
    int32_t tile_hmax = 0; // largest tile halo (0: no tiled problem)
    int64_t *d_slice_off = nullptr;
    KL *d_kl = nullptr;
    KL32 *d_kl32 = nullptr;
    // device arrays: state and results (per problem)
    double *d_u = nullptr, *d_qbuf = nullptr, *d_wbuf = nullptr;
    int64_t *d_state_off = nullptr; // [P] first running-state record of each problem
    double *d_F_cur = nullptr, *d_F_last = nullptr;
    int32_t *d_has_state = nullptr, *d_status = nullptr;
    double *d_sigma = nullptr, *d_sigma_fib = nullptr, *d_rho = nullptr, *d_ke = nullptr;
    int64_t *d_iters = nullptr, *d_n_best = nullptr;
    double *d_rho_best = nullptr;
    // device arrays: per launch slot
    double *d_F = nullptr;
    int32_t *d_ids = nullptr, *d_order = nullptr, *d_starts = nullptr;
    double *d_partial = nullptr, *d_scalars = nullptr;
    double *d_gscat = nullptr; // forces of the atomic-scatter comparator (allocated on first use)
    double *d_enode = nullptr, *d_e_work = nullptr, *d_e_damp = nullptr; // energy balance
    // tail hand-off: launch counters, the tail list, the groups' barriers
    int32_t *d_live = nullptr, *d_tail_list = nullptr, *d_tail_count = nullptr, *d_gabort = nullptr;
    uint32_t *d_gbar = nullptr;
    int64_t *d_n_begin = nullptr;
    double *d_gpart = nullptr;
    double *d_abuf = nullptr, *d_dt_next = nullptr; // per-pass time step (dt_rule = 1)
    int64_t *d_budgets = nullptr, *h_budgets = nullptr; // per-problem pass budgets of a launch
    int32_t tail_group = 0;     // workgroups per handed-off problem (0: hand-off off)
    LaunchPlan tail_plan{};     // launch shape of the group kernel
    // caller-owned device workspace (dr_batch_create_in): every device array
    // is carved from it at 256-byte boundaries and never freed here;
    // `counting` is the sizing pass of dr_batch_workspace_bytes (no HIP call)
    char *ws = nullptr;
    size_t ws_bytes = 0, ws_used = 0;
    bool counting = false;
    // pinned staging
    double *h_F = nullptr;
    int32_t *h_ids = nullptr, *h_order = nullptr, *h_starts = nullptr;
    double *h_scalars = nullptr;
    std::vector<int64_t> state_off; // host copy of d_state_off
    int64_t *h_state_off = nullptr;  // pinned staging of it
    bool state_off_dirty = false;    // changed since its last upload
    hipEvent_t staged = nullptr;
    // host mirror of which problems have a running solve (for DR_RESUME checks)
    std::vector<char> running;
    // passes of each problem's last finished solve (0: none yet), for the
    // launch order by estimated cost
    std::vector<int64_t> last_passes;
    std::vector<double> order_cost; // scratch of the launch order
    std::vector<char> seen; // [P] scratch of the id checks (all zero between calls)
    // last dr_solve* call
    int32_t last_n = -1;
    std::vector<int32_t> last_ids;
    // Size classes: each class has one launch shape.  Every shape computes
    // the same per-node arithmetic in the same order, so a problem's result
    // is the same, bit for bit, whatever its class's shape and whichever
    // problems share a launch.  Classes are launched concurrently on their
    // own streams (fork / join on the batch stream).
    struct Class {
        int32_t n_lo = 0, n_hi = 0; // node counts covered (inclusive)
        int32_t n_max = 0;          // largest problem of the batch in the class
        int32_t count = 0;          // problems of the batch in the class
        LaunchPlan plan{0, 0, 0, 4, 0};
        hipStream_t st = nullptr;
        hipEvent_t done = nullptr;
    };
    std::vector<Class> classes;
    std::vector<int8_t> class_of;       // per problem
    std::vector<int32_t> slot_count;    // per class, slots of the staged launch
    std::vector<int32_t> slot_off;      // per class, first entry in the slot order
    hipEvent_t fork = nullptr;
    // captured solve step
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int32_t> graph_ids;
};

namespace {

void free_all(dr_batch *b)
{
    void *dev[] = {b->d_probs, b->d_X, b->d_invm, b->d_mass, b->d_invm32, b->d_mass32, b->d_deg,
                   b->d_slice_w, b->d_nbr, b->d_lslot, b->d_tile_halo, b->d_halo_ids, b->d_slice_off, b->d_kl, b->d_kl32, b->d_u, b->d_qbuf,
                   b->d_wbuf, b->d_F_cur, b->d_F_last, b->d_has_state, b->d_status, b->d_sigma,
                   b->d_sigma_fib, b->d_rho, b->d_ke, b->d_iters, b->d_n_best, b->d_rho_best, b->d_F, b->d_ids, b->d_order,
                   b->d_starts, b->d_partial, b->d_scalars, b->d_gscat, b->d_enode,
                   b->d_e_work, b->d_e_damp, b->d_state_off, b->d_live, b->d_tail_list,
                   b->d_tail_count, b->d_gabort, b->d_gbar, b->d_n_begin, b->d_gpart,
                   b->d_abuf, b->d_dt_next, b->d_budgets};
    if (!b->ws)
        for (void *p : dev)
            if (p) (void)hipFree(p);
    void *host[] = {b->h_F, b->h_ids, b->h_order, b->h_starts, b->h_scalars, b->h_state_off, b->h_budgets};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (auto &c : b->classes) {
        if (c.done) (void)hipEventDestroy(c.done);
        if (c.st) (void)hipStreamDestroy(c.st);
    }
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
}

// 30-bit Morton key of a point in the unit cube (clamped).
uint32_t morton3(const double *x)
{
    uint32_t key = 0;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        double t = x[a];
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        q[a] = (uint32_t)(t * 1023.0);
    }
    for (int bit = 9; bit >= 0; --bit)
        for (int a = 0; a < 3; ++a) key = (key << 1) | ((q[a] >> bit) & 1u);
    return key;
}

dr_status validate_options(const dr_options *o)
{
    if (!o) return fail(DR_E_INVALID, "options is NULL");
    if (o->precision != DR_FP64 && o->precision != DR_FP32)
        return fail(DR_E_INVALID, "precision %d is not DR_FP64 or DR_FP32", o->precision);
    if (!(o->tol > 0.0) || !std::isfinite(o->tol))
        return fail(DR_E_INVALID, "tol must be finite and > 0 (got %g)", o->tol);
    if (o->max_iter < 1) return fail(DR_E_INVALID, "max_iter must be >= 1");
    if (!(o->damping >= 0.0) || !std::isfinite(o->damping))
        return fail(DR_E_INVALID, "damping must be finite and >= 0 (got %g)", o->damping);
    if (!(o->dt_safety > 0.0 && o->dt_safety <= 1.0))
        return fail(DR_E_INVALID, "dt_safety must be in (0, 1] (got %g)", o->dt_safety);
    if (o->block != 0 && o->block != 256 && o->block != 512 && o->block != 1024)
        return fail(DR_E_INVALID, "block must be 0, 256, 512 or 1024 (got %d)", o->block);
    if (o->placement < DR_PLACE_AUTO || o->placement > DR_PLACE_GLOBAL)
        return fail(DR_E_INVALID, "placement %d is not a dr_placement value", o->placement);
    if (o->chunk != 0 && o->chunk != 1 && o->chunk != 2 && o->chunk != 4)
        return fail(DR_E_INVALID, "chunk must be 0, 1, 2 or 4 (got %d)", o->chunk);
    if (o->stall_window < 0) return fail(DR_E_INVALID, "stall_window must be >= 0");
    if (!(o->energy_tol >= 0.0) || !std::isfinite(o->energy_tol))
        return fail(DR_E_INVALID, "energy_tol must be finite and >= 0 (got %g)", o->energy_tol);
    if (o->tail_at < 0 || o->tail_at > drk::kTailMax)
        return fail(DR_E_INVALID, "tail_at must be in [0, %d] (got %d)", drk::kTailMax, o->tail_at);
    if (o->tail_group != 0 && (o->tail_group < 2 || o->tail_group > drk::kGroupMax))
        return fail(DR_E_INVALID, "tail_group must be 0 or in [2, %d] (got %d)", drk::kGroupMax, o->tail_group);
    if (o->dt_rule != 0 && o->dt_rule != 1)
        return fail(DR_E_INVALID, "dt_rule must be 0 or 1 (got %d)", o->dt_rule);
    if (o->dt_rule == 1) {
        if (o->precision != DR_FP64) return fail(DR_E_INVALID, "dt_rule 1 is FP64 only");
        if (o->energy_tol != 0.0) return fail(DR_E_INVALID, "dt_rule 1 does not track the energy balance");
        if (o->tail_at != 0) return fail(DR_E_INVALID, "dt_rule 1 has no tail hand-off");
    }
    return DR_OK;
}

// Host-side packing of all problems (no HIP calls).
struct Packed {
    std::vector<ProbDesc> desc;
    std::vector<HostProblem> hp;
    std::vector<double> X, invm, mass;
    std::vector<float> invm32, mass32;
    std::vector<int32_t> deg, slice_w, nbr;
    std::vector<int64_t> slice_off;
    std::vector<KL> kl;
    std::vector<KL32> kl32;
    std::vector<uint16_t> lslot;    // per incidence (tiled problems; 0 elsewhere)
    std::vector<int32_t> tile_halo; // per tile, + 1 per tiled problem
    std::vector<int32_t> halo_ids;
    int32_t n_max = 0;
    int32_t tile_hmax = 0;
};

dr_status pack(const dr_networks *nets, const dr_options *opt, Packed &pk)
{
    if (!nets) return fail(DR_E_INVALID, "networks is NULL");
    const int32_t P = nets->n_problems;
    if (P < 1) return fail(DR_E_INVALID, "n_problems must be >= 1 (got %d)", P);
    if (!nets->node_offsets || !nets->fiber_offsets || !nets->X || !nets->EA)
        return fail(DR_E_INVALID, "a required network array is NULL");
    if (!nets->fixed && !(nets->band >= 0.0 && std::isfinite(nets->band)))
        return fail(DR_E_INVALID, "fixed is NULL and band (%g) is not finite and >= 0", nets->band);
    const bool fp32 = opt->precision == DR_FP32;
    const int64_t *no = nets->node_offsets, *fo = nets->fiber_offsets;
    if (no[0] != 0 || fo[0] != 0) return fail(DR_E_INVALID, "offsets must start at 0");
    for (int32_t p = 0; p < P; ++p) {
        if (no[p + 1] - no[p] < 1)
            return fail(DR_E_INVALID, "problem %d has no nodes", p);
        if (no[p + 1] - no[p] > (int64_t)drk::kWave * drk::kGlbHdrMax)
            return fail(DR_E_INVALID, "problem %d has %lld nodes (at most %d per problem)", p,
                        (long long)(no[p + 1] - no[p]), drk::kWave * drk::kGlbHdrMax);
        if (fo[p + 1] < fo[p]) return fail(DR_E_INVALID, "fiber_offsets decrease at problem %d", p);
    }
    if (fo[P] > 0 && !nets->fiber_nodes) return fail(DR_E_INVALID, "fiber_nodes is NULL");

    pk.desc.resize(P);
    pk.hp.resize(P);
    const int64_t total_nodes = no[P];
    for (int64_t i = 0; i < 3 * total_nodes; ++i)
        if (!std::isfinite(nets->X[i]))
            return fail(DR_E_INVALID, "X[%lld] is not finite", (long long)i);

    int64_t slice_base = 0, inc_base = 0, node_base = 0;
    pk.X.resize(3 * total_nodes);
    pk.invm.resize(total_nodes);
    pk.mass.resize(total_nodes);
    pk.deg.resize(total_nodes);
    if (fp32) {
        pk.invm32.resize(total_nodes);
        pk.mass32.resize(total_nodes);
    }

    for (int32_t p = 0; p < P; ++p) {
        const int32_t N = (int32_t)(no[p + 1] - no[p]);
        const int64_t M64 = fo[p + 1] - fo[p];
        if (M64 > INT32_MAX / 2) return fail(DR_E_INVALID, "problem %d has too many fibers", p);
        const int32_t M = (int32_t)M64;
        const double *X = nets->X + 3 * no[p];
        const int32_t *fib = nets->fiber_nodes + 2 * fo[p];
        const double *EA = nets->EA + fo[p];
        // prescribed nodes: the caller's mask, or the band rule (a node within
        // `band` of a face of the unit cube, inclusive)
        std::vector<uint8_t> band_mask;
        if (!nets->fixed) {
            band_mask.resize(N);
            for (int32_t i = 0; i < N; ++i) {
                double dmin = 1.0;
                for (int a = 0; a < 3; ++a)
                    dmin = std::min(dmin, std::min(X[3 * i + a], 1.0 - X[3 * i + a]));
                band_mask[i] = dmin <= nets->band ? 1 : 0;
            }
        }
        const uint8_t *fixed = nets->fixed ? nets->fixed + no[p] : band_mask.data();

        // L2g: L^2 rounded as the kernels form squared lengths,
        // fma(dz, dz, fma(dy, dy, dx * dx)), so that l^2 - L^2 is exactly 0
        // for a fiber at its reference length
        std::vector<double> L(M), L2(M), L2g(M);
        std::vector<int32_t> degree(N, 0);
        for (int32_t f = 0; f < M; ++f) {
            const int32_t a = fib[2 * f], b = fib[2 * f + 1];
            if (a < 0 || a >= N || b < 0 || b >= N)
                return fail(DR_E_INVALID, "problem %d fiber %d: node id out of range (%d, %d; N=%d)",
                            p, f, a, b, N);
            if (a == b) return fail(DR_E_INVALID, "problem %d fiber %d joins node %d to itself", p, f, a);
            if (!(EA[f] > 0.0) || !std::isfinite(EA[f]))
                return fail(DR_E_INVALID, "problem %d fiber %d: EA must be finite and > 0 (got %g)",
                            p, f, EA[f]);
            const double dx = X[3 * b] - X[3 * a], dy = X[3 * b + 1] - X[3 * a + 1],
                         dz = X[3 * b + 2] - X[3 * a + 2];
            L2[f] = dx * dx + dy * dy + dz * dz;
            L2g[f] = std::fma(dz, dz, std::fma(dy, dy, dx * dx));
            L[f] = std::sqrt(L2[f]);
            if (!(L[f] > 0.0))
                return fail(DR_E_INVALID, "problem %d fiber %d has zero reference length", p, f);
            ++degree[a];
            ++degree[b];
        }
        int32_t n_free = 0;
        for (int32_t i = 0; i < N; ++i) {
            if (!fixed[i]) {
                ++n_free;
                if (degree[i] == 0)
                    return fail(DR_E_INVALID, "problem %d node %d is free but has no fiber", p, i);
            }
        }
        // CSR node -> fibers in ascending fiber id
        std::vector<int32_t> rp(N + 1, 0), ent(2 * (size_t)M);
        for (int32_t i = 0; i < N; ++i) rp[i + 1] = rp[i] + degree[i];
        {
            std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
            for (int32_t f = 0; f < M; ++f) {
                ent[fill[fib[2 * f]]++] = f;
                ent[fill[fib[2 * f + 1]]++] = f;
            }
        }
        // lumped mass (half the length of every fiber at the node) and the
        // Gershgorin frequency bound, both summed in ascending fiber order
        std::vector<double> m(N, 0.0), ksum(N, 0.0);
        for (int32_t f = 0; f < M; ++f) {
            const int32_t a = fib[2 * f], b = fib[2 * f + 1];
            m[a] += 0.5 * L[f];
            m[b] += 0.5 * L[f];
            const double kh = 1.1 * EA[f] / L[f];
            ksum[a] += kh;
            ksum[b] += kh;
        }
        double w2 = 0.0, ea_sum = 0.0;
        int32_t n_fixed = 0;
        for (int32_t i = 0; i < N; ++i) {
            if (fixed[i]) { ++n_fixed; continue; }
            const double wi = 2.0 / m[i] * ksum[i];
            if (wi > w2) w2 = wi;
        }
        for (int32_t f = 0; f < M; ++f) ea_sum += EA[f];
        const double w = std::sqrt(w2);
        ProbDesc &d = pk.desc[p];
        std::memset(&d, 0, sizeof d);
        d.N = N;
        d.N_free = n_free;
        d.M = M;
        d.n_slices = (N + drk::kWave - 1) / drk::kWave;
        d.dt = w > 0.0 ? opt->dt_safety * 2.0 / w : 0.0;
        d.c = opt->damping * w;
        const double ea_mean = M > 0 ? ea_sum / M : 0.0;
        d.s_floor = 1e-4 * ea_mean * std::sqrt(3.0 * (n_fixed > 1 ? n_fixed : 1));

        // renumber: free block then prescribed block; degree descending, then
        // Morton.  A problem too large for the LDS variant is cut into tiles
        // of kTile nodes in Morton order (free block, then prescribed block),
        // and the degree order applies inside each tile, so that a tile is a
        // compact region whose neighbours mostly lie in the tile itself.
        std::vector<int32_t> order(N);
        std::iota(order.begin(), order.end(), 0);
        std::vector<uint32_t> key(N);
        for (int32_t i = 0; i < N; ++i) key[i] = morton3(X + 3 * i);
        auto by_degree = [&](int32_t i, int32_t j) {
            if ((fixed[i] != 0) != (fixed[j] != 0)) return fixed[i] == 0;
            if (degree[i] != degree[j]) return degree[i] > degree[j];
            return key[i] < key[j];
        };
        const bool tiled = N > drk::kTiledMinNodes;
        if (tiled) {
            std::stable_sort(order.begin(), order.end(), [&](int32_t i, int32_t j) {
                if ((fixed[i] != 0) != (fixed[j] != 0)) return fixed[i] == 0;
                return key[i] < key[j];
            });
            for (int32_t t0 = 0; t0 < N; t0 += drk::kTile)
                std::stable_sort(order.begin() + t0, order.begin() + std::min(N, t0 + drk::kTile), by_degree);
        } else {
            std::stable_sort(order.begin(), order.end(), by_degree);
        }
        HostProblem &h = pk.hp[p];
        h.N = N;
        h.N_free = n_free;
        h.M = M;
        h.in_node_base = no[p];
        h.new_of_old.assign(N, 0);
        for (int32_t r = 0; r < N; ++r) h.new_of_old[order[r]] = r;

        d.node_base = node_base;
        d.slice_base = slice_base;
        d.inc_base = inc_base;
        for (int32_t r = 0; r < N; ++r) {
            const int32_t i = order[r];
            for (int a = 0; a < 3; ++a) pk.X[3 * (node_base + r) + a] = X[3 * i + a];
            pk.mass[node_base + r] = m[i];
            pk.invm[node_base + r] = 1.0 / m[i];
            pk.deg[node_base + r] = degree[i];
            if (fp32) {
                pk.mass32[node_base + r] = (float)m[i];
                pk.invm32[node_base + r] = (float)(1.0 / m[i]);
            }
        }
        if (N > pk.n_max) pk.n_max = N;
        // sliced ELL incidences
        int64_t off = 0;
        for (int32_t q = 0; q < d.n_slices; ++q) {
            int32_t width = 0;
            for (int32_t lane = 0; lane < drk::kWave; ++lane) {
                const int32_t r = q * drk::kWave + lane;
                if (r < N) width = std::max(width, degree[order[r]]);
            }
            pk.slice_w.push_back(width);
            pk.slice_off.push_back(off);
            const size_t base = pk.nbr.size();
            pk.nbr.resize(base + (size_t)width * drk::kWave, 0);
            pk.kl.resize(base + (size_t)width * drk::kWave, KL{0.0, 0.0});
            if (fp32) pk.kl32.resize(base + (size_t)width * drk::kWave, KL32{0.f, 0.f, 0.f, 0.f});
            for (int32_t lane = 0; lane < drk::kWave; ++lane) {
                const int32_t r = q * drk::kWave + lane;
                if (r >= N) continue;
                const int32_t i = order[r];
                for (int32_t k = 0; k < degree[i]; ++k) {
                    const int32_t f = ent[rp[i] + k];
                    const int32_t other = fib[2 * f] == i ? fib[2 * f + 1] : fib[2 * f];
                    const size_t e = base + (size_t)k * drk::kWave + lane;
                    pk.nbr[e] = h.new_of_old[other];
                    const double kf = EA[f] / (2.0 * L2[f]);
                    pk.kl[e] = KL{kf, L2g[f]};
                    if (fp32)
                        pk.kl32[e] = KL32{(float)(X[3 * other] - X[3 * i]),
                                          (float)(X[3 * other + 1] - X[3 * i + 1]),
                                          (float)(X[3 * other + 2] - X[3 * i + 2]), (float)kf};
                }
                // Padding up to the slice width: zero constants and a
                // neighbour at a positive distance (the first real neighbour,
                // or for a node without fibers another node at a different
                // reference point), so the entry adds exactly zero force.
                if (degree[i] < width) {
                    int32_t pad = -1;
                    if (degree[i] > 0) {
                        const int32_t f = ent[rp[i]];
                        pad = fib[2 * f] == i ? fib[2 * f + 1] : fib[2 * f];
                    } else {
                        for (int32_t j = 0; j < N && pad < 0; ++j)
                            if (X[3 * j] != X[3 * i] || X[3 * j + 1] != X[3 * i + 1] ||
                                X[3 * j + 2] != X[3 * i + 2])
                                pad = j;
                        if (pad < 0)
                            return fail(DR_E_INVALID,
                                        "problem %d: every node sits at the same reference point", p);
                    }
                    for (int32_t k = degree[i]; k < width; ++k) {
                        const size_t e = base + (size_t)k * drk::kWave + lane;
                        pk.nbr[e] = h.new_of_old[pad];
                        if (fp32)
                            pk.kl32[e] = KL32{(float)(X[3 * pad] - X[3 * i]),
                                              (float)(X[3 * pad + 1] - X[3 * i + 1]),
                                              (float)(X[3 * pad + 2] - X[3 * i + 2]), 0.f};
                    }
                }
            }
            off += (int64_t)width * drk::kWave;
        }
        // the kernels address a problem's 16-byte incidence constants with
        // 32-bit byte offsets
        if (off * 16 > (int64_t)INT32_MAX)
            return fail(DR_E_INVALID, "problem %d: %lld incidence entries exceed 2^27", p, (long long)off);
        // tiles: each incidence's neighbour as a slot of its tile's staged
        // records (the tile's own nodes first, then its halo); entries of
        // lanes past N point at slot 0.  A problem with a halo above
        // kHaloMax keeps the plain gather.
        pk.lslot.resize(pk.nbr.size(), 0);
        d.n_tiles = 0;
        if (tiled) {
            const int32_t nt = (N + drk::kTile - 1) / drk::kTile;
            std::vector<int32_t> mark(N, -1), halo, toff(1, 0), ids;
            std::vector<uint16_t> slots;
            bool ok = true;
            int32_t hmax = 0;
            const int64_t e0 = (int64_t)pk.nbr.size() - off;
            for (int32_t t = 0; t < nt && ok; ++t) {
                const int32_t lo = t * drk::kTile, hi = std::min(N, lo + drk::kTile);
                halo.clear();
                for (int32_t q = lo / drk::kWave; q < (hi + drk::kWave - 1) / drk::kWave; ++q) {
                    const int64_t so = e0 + pk.slice_off[slice_base + q];
                    const int32_t width = pk.slice_w[slice_base + q];
                    for (int32_t k = 0; k < width; ++k)
                        for (int32_t lane = 0; lane < drk::kWave; ++lane) {
                            const int64_t e = so + (int64_t)k * drk::kWave + lane;
                            const int32_t r = q * drk::kWave + lane;
                            int32_t slot = 0;
                            if (r < N) {
                                const int32_t j = pk.nbr[e];
                                if (j >= lo && j < hi) {
                                    slot = j - lo;
                                } else {
                                    if (mark[j] < 0) {
                                        mark[j] = (int32_t)halo.size();
                                        halo.push_back(j);
                                    }
                                    slot = drk::kTile + mark[j];
                                }
                            }
                            pk.lslot[e] = (uint16_t)std::min(slot, 65535);
                        }
                }
                for (int32_t j : halo) mark[j] = -1;
                if ((int32_t)halo.size() > drk::kHaloMax) ok = false;
                hmax = std::max(hmax, (int32_t)halo.size());
                ids.insert(ids.end(), halo.begin(), halo.end());
                toff.push_back((int32_t)ids.size());
            }
            if (ok) {
                d.n_tiles = nt;
                d.tile_base = (int64_t)pk.tile_halo.size();
                d.halo_base = (int64_t)pk.halo_ids.size();
                pk.tile_halo.insert(pk.tile_halo.end(), toff.begin(), toff.end());
                pk.halo_ids.insert(pk.halo_ids.end(), ids.begin(), ids.end());
                pk.tile_hmax = std::max(pk.tile_hmax, hmax);
            } else {
                std::fill(pk.lslot.begin() + e0, pk.lslot.end(), (uint16_t)0);
            }
        }
        d.n_inc = off;
        slice_base += d.n_slices;
        inc_base += off;
        node_base += N;
    }
    // without a tiled problem the kernels never read the slots
    if (pk.tile_hmax == 0 && pk.tile_halo.empty()) pk.lslot.clear();
    return DR_OK;
}

constexpr size_t kWsAlign = 256;

// One device array of the batch: from hipMalloc, or carved from the caller's
// workspace, or (sizing pass) only counted.
dr_status dev_alloc(dr_batch *b, void **dst, size_t bytes)
{
    bytes = (bytes + kWsAlign - 1) / kWsAlign * kWsAlign;
    *dst = nullptr;
    if (b->counting) {
        b->ws_used += bytes;
        return DR_OK;
    }
    if (b->ws) {
        if (b->ws_used + bytes > b->ws_bytes)
            return fail(DR_E_INVALID, "the workspace of %zu bytes is too small", b->ws_bytes);
        *dst = b->ws + b->ws_used;
        b->ws_used += bytes;
        return DR_OK;
    }
    HIPCHECK(hipMalloc(dst, bytes));
    return DR_OK;
}

template <class T> dr_status dev_upload(dr_batch *b, T **dst, const std::vector<T> &src, hipStream_t st)
{
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    dr_status s = dev_alloc(b, reinterpret_cast<void **>(dst), bytes);
    if (s != DR_OK || b->counting) return s;
    if (!src.empty())
        HIPCHECK(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return DR_OK;
}

template <class T> dr_status dev_zeros(dr_batch *b, T **dst, size_t n, hipStream_t st)
{
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    dr_status s = dev_alloc(b, reinterpret_cast<void **>(dst), bytes);
    if (s != DR_OK || b->counting) return s;
    HIPCHECK(hipMemsetAsync(*dst, 0, bytes, st));
    return DR_OK;
}

dr_status create_device(dr_batch *b, Packed &pk)
{
    hipStream_t st = b->stream;
    if (!b->counting) HIPCHECK(hipGetDevice(&b->device));
    dr_status s;
#define UP(dst, vec)                                                                              \
    if ((s = dev_upload(b, &b->dst, pk.vec, st)) != DR_OK) return s;
    UP(d_probs, desc)
    UP(d_X, X)
    UP(d_invm, invm)
    UP(d_mass, mass)
    UP(d_invm32, invm32)
    UP(d_mass32, mass32)
    UP(d_deg, deg)
    UP(d_slice_w, slice_w)
    UP(d_slice_off, slice_off)
    UP(d_nbr, nbr)
    UP(d_lslot, lslot)
    UP(d_tile_halo, tile_halo)
    UP(d_halo_ids, halo_ids)
    UP(d_kl, kl)
    UP(d_kl32, kl32)
#undef UP
    if ((s = dev_upload(b, &b->d_state_off, b->state_off, st)) != DR_OK) return s;
    const size_t P = (size_t)b->P, nodes = (size_t)b->total_nodes;
    const size_t rec = (size_t)b->state_nodes;
#define ZS(dst, n)                                                                                \
    if ((s = dev_zeros(b, &b->dst, (n), st)) != DR_OK) return s;
    ZS(d_u, 3 * nodes)
    ZS(d_qbuf, 2 * (size_t)state_doubles(b->opt.precision) * rec) // two state buffers
    ZS(d_wbuf, (size_t)velocity_doubles(b->opt.precision) * rec)
    ZS(d_F_cur, 9 * P)
    ZS(d_F_last, 9 * P)
    ZS(d_has_state, P)
    ZS(d_status, P)
    ZS(d_sigma, 9 * P)
    ZS(d_sigma_fib, 9 * P)
    ZS(d_rho, P)
    ZS(d_ke, P)
    ZS(d_iters, P)
    ZS(d_n_best, P)
    ZS(d_rho_best, P)
    ZS(d_F, 9 * P)
    ZS(d_ids, P)
    ZS(d_order, P)
    ZS(d_starts, P)
    ZS(d_partial, 3 * ((size_t)pk.n_max / 256 + 2))
    ZS(d_scalars, 8)
    ZS(d_e_work, P)
    ZS(d_e_damp, P)
    if (b->opt.energy_tol > 0.0) ZS(d_enode, 4 * nodes)
    if (b->opt.dt_rule == 1) {
        ZS(d_abuf, 3 * rec)
        ZS(d_dt_next, P)
    }
    ZS(d_live, 1)
    ZS(d_tail_count, 1)
    ZS(d_tail_list, drk::kTailMax)
    ZS(d_gabort, drk::kTailMax)
    ZS(d_gbar, drk::kTailMax)
    ZS(d_n_begin, P)
    ZS(d_budgets, P)
    ZS(d_gpart, (size_t)drk::kTailMax * 2 * drk::kGroupMax * 4)
    // with a caller-owned workspace the scatter comparator's force buffer is
    // carved up front (it is allocated on first use otherwise)
    if (b->ws || b->counting) ZS(d_gscat, 3 * (size_t)std::max(pk.n_max, 1))
#undef ZS
    if (b->counting) return DR_OK;
    const int rc = drk::launch_fill_i32(b->d_status, DR_IDLE, (int64_t)P, st);
    if (rc != 0) return fail(DR_E_DEVICE, "status fill failed: %s", drk::kernel_error_string(rc));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&b->h_F), 9 * P * sizeof(double), 0));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&b->h_ids), P * sizeof(int32_t), 0));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&b->h_order), P * sizeof(int32_t), 0));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&b->h_starts), P * sizeof(int32_t), 0));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&b->h_scalars), 8 * sizeof(double), 0));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&b->h_state_off), P * sizeof(int64_t), 0));
    HIPCHECK(hipHostMalloc(reinterpret_cast<void **>(&b->h_budgets), P * sizeof(int64_t), 0));
    HIPCHECK(hipEventCreateWithFlags(&b->staged, hipEventDisableTiming));
    HIPCHECK(hipStreamSynchronize(st));
    return DR_OK;
}

// LDS of the global kernel: the reduction records (20 doubles per wave), the
// group barrier's flag word (16 B) and the slice headers (8 B each) of the
// workgroup's rows, for a problem of n_max nodes shared by G workgroups.
int glb_lds_bytes(int block, int G, int32_t n_max)
{
    const int nw = block / drk::kWave;
    const int slices = (n_max + drk::kWave - 1) / drk::kWave; // <= kGlbHdrMax (validated)
    const int rows = (slices + G * nw - 1) / (G * nw);
    return nw * 20 * 8 + 16 + 8 * rows * nw;
}

// Launch shape for a batch whose largest problem has n_max nodes.  Returns
// npt = -1 when DR_PLACE_LDS was asked for and the problem does not fit.
LaunchPlan plan_for(const dr_options &opt, int32_t n_max, int32_t tile_hmax = 0)
{
    LaunchPlan pl{};
    pl.fp32 = opt.precision == DR_FP32;
    const int elem = pl.fp32 ? 4 : 8; // bytes per state value in LDS
    const int block = opt.block;
    // node records (rounded up to 8 bytes), then one 160-byte record per wave
    auto reg_lds = [&](int blk, int n) { return (blk / drk::kWave) * 20 * 8 + (3 * n * elem + 7) / 8 * 8; };
    // register-resident variant when the state fits in LDS
    int blk = block;
    if (blk == 0) blk = n_max > 2048 ? 1024 : (n_max > 256 ? 512 : 256);
    int npt = (n_max + blk - 1) / blk;
    if (block == 0 && npt > kMaxNpt) {
        blk = 1024;
        npt = (n_max + blk - 1) / blk;
    }
    const bool fits = npt <= kMaxNpt && reg_lds(blk, n_max) <= kLdsLimit;
    if (opt.placement == DR_PLACE_LDS && !fits) {
        pl.block = blk;
        pl.npt = -1;
        return pl;
    }
    if (fits && opt.placement != DR_PLACE_GLOBAL) {
        // at 1024 threads (128 VGPRs) the prefetched chunk shrinks with the
        // nodes held per thread: 2 up to 4 nodes, then 1
        pl.chunk = opt.chunk ? opt.chunk : (blk == 1024 ? (npt <= 4 ? 2 : 1) : 4);
        pl.block = blk;
        pl.npt = npt < 1 ? 1 : npt;
        pl.lds_bytes = reg_lds(blk, n_max);
        return pl;
    }
    pl.block = block ? block : 1024;
    pl.npt = 0;
    // 256 threads: chunks of 1 only (the only global build of that width);
    // an explicit request for another chunk there is reported (npt = -2)
    // when the placement was asked for, and replaced by 1 in the automatic
    // split (dr_batch_class_info shows the chunk each class runs)
    if (pl.block == 256 && opt.chunk > 1 && opt.placement == DR_PLACE_GLOBAL) {
        pl.npt = -2;
        return pl;
    }
    pl.chunk = pl.block == 256 ? 1 : (opt.chunk ? opt.chunk : (pl.block == 1024 ? 1 : 2));
    pl.lds_bytes = glb_lds_bytes(pl.block, 1, n_max);
    // the FP64 1024-thread build stages the tiles of tiled problems (their
    // own records and halo) in LDS, ahead of its other records
    if (!pl.fp32 && pl.block == 1024 && pl.chunk == 1 && tile_hmax > 0)
        pl.lds_bytes += 24 * (drk::kTile + tile_hmax);
    return pl;
}

// One requested class plan (dr_set_class_plan).
struct ClassRequest {
    int32_t n_hi;
    int32_t block, chunk, placement;
};

// Splits the problems into size classes and gives each its launch shape.
// Requested classes (ascending n_hi) come first; the problems above the last
// requested bound get the automatic split: the largest set that fits the
// LDS / register variant, then the rest in global placement.
dr_status build_classes(dr_batch *b, const std::vector<ClassRequest> &req)
{
    std::vector<dr_batch::Class> cls;
    int32_t lo = 1;
    auto n_max_in = [&](int32_t a, int32_t z) {
        int32_t m = 0, c = 0;
        for (const auto &h : b->hp)
            if (h.N >= a && h.N <= z) { m = std::max(m, h.N); ++c; }
        return std::make_pair(m, c);
    };
    for (const auto &r : req) {
        dr_batch::Class c;
        c.n_lo = lo;
        c.n_hi = r.n_hi;
        auto mc = n_max_in(lo, r.n_hi);
        c.n_max = mc.first;
        c.count = mc.second;
        dr_options o = b->opt;
        o.block = r.block;
        o.chunk = r.chunk;
        o.placement = r.placement;
        c.plan = plan_for(o, std::max(c.n_max, 1), b->tile_hmax);
        if (c.plan.npt == -2)
            return fail(DR_E_INVALID, "class up to %d nodes: global placement with 256 threads "
                        "runs gather chunks of 1 only (got %d)", r.n_hi, r.chunk);
        if (c.plan.npt < 0)
            return fail(DR_E_INVALID, "class up to %d nodes: DR_PLACE_LDS cannot hold %d nodes",
                        r.n_hi, c.n_max);
        cls.push_back(c);
        lo = r.n_hi + 1;
    }
    // the per-pass step in groups runs one launch per call: one class
    const bool dtp_groups = b->opt.dt_rule == 1 && b->opt.tail_group > 1;
    if (dtp_groups && !req.empty())
        return fail(DR_E_INVALID, "the per-pass step in groups (dt_rule 1, tail_group > 1) runs one "
                    "class; size-class plans do not apply");
    // automatic split of the rest
    const int32_t top = INT32_MAX;
    if (b->opt.placement == DR_PLACE_GLOBAL || b->opt.placement == DR_PLACE_LDS || dtp_groups) {
        dr_batch::Class c;
        c.n_lo = lo;
        c.n_hi = top;
        auto mc = n_max_in(lo, top);
        c.n_max = mc.first;
        c.count = mc.second;
        c.plan = plan_for(b->opt, std::max(c.n_max, 1), b->tile_hmax);
        if (c.plan.npt == -2)
            return fail(DR_E_INVALID, "global placement with 256 threads runs gather chunks of 1 only "
                        "(got %d)", b->opt.chunk);
        if (c.plan.npt < 0)
            return fail(DR_E_INVALID, "placement DR_PLACE_LDS cannot hold a %d-node problem (block %d)",
                        c.n_max, b->opt.block);
        cls.push_back(c);
    } else {
        // largest N (among the remaining problems) that the register variant holds
        int32_t fit = 0;
        for (const auto &h : b->hp)
            if (h.N >= lo && h.N > fit && plan_for(b->opt, h.N).npt > 0) fit = h.N;
        if (fit >= lo) {
            dr_batch::Class c;
            c.n_lo = lo;
            c.n_hi = fit;
            auto mc = n_max_in(lo, fit);
            c.n_max = mc.first;
            c.count = mc.second;
            c.plan = plan_for(b->opt, c.n_max, b->tile_hmax);
            cls.push_back(c);
            lo = fit + 1;
        }
        dr_batch::Class g;
        g.n_lo = lo;
        g.n_hi = top;
        auto mc = n_max_in(lo, top);
        g.n_max = mc.first;
        g.count = mc.second;
        dr_options o = b->opt;
        o.placement = DR_PLACE_GLOBAL;
        if (o.block == 256) o.chunk = 1; // the only global build of that width
        g.plan = plan_for(o, std::max(g.n_max, 1), b->tile_hmax);
        cls.push_back(g);
    }
    // classes without problems launch nothing: drop them (at least one stays)
    std::vector<dr_batch::Class> kept;
    for (const auto &c : cls)
        if (c.count > 0) kept.push_back(c);
    if (!kept.empty()) cls.swap(kept);
    // keep the streams of the old classes for reuse
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> ev;
    for (auto &c : b->classes) { st.push_back(c.st); ev.push_back(c.done); }
    for (size_t k = 0; k < cls.size(); ++k) {
        if (k < st.size()) { cls[k].st = st[k]; cls[k].done = ev[k]; }
        else {
            HIPCHECK(hipStreamCreateWithFlags(&cls[k].st, hipStreamNonBlocking));
            HIPCHECK(hipEventCreateWithFlags(&cls[k].done, hipEventDisableTiming));
        }
    }
    for (size_t k = cls.size(); k < st.size(); ++k) {
        (void)hipEventDestroy(ev[k]);
        (void)hipStreamDestroy(st[k]);
    }
    b->classes = cls;
    b->class_of.assign(b->P, 0);
    for (int32_t p = 0; p < b->P; ++p)
        for (size_t k = 0; k < cls.size(); ++k)
            if (b->hp[p].N >= cls[k].n_lo && b->hp[p].N <= cls[k].n_hi) {
                b->class_of[p] = (int8_t)k;
                break;
            }
    b->slot_count.assign(cls.size(), 0);
    b->slot_off.assign(cls.size(), 0);
    return DR_OK;
}

// Launch shape of the tail hand-off's group kernel: 1024 threads per
// workgroup, and as many workgroups per problem (tail_group, or automatic:
// the most that let tail_at problems be co-resident, at most kGroupMax) as
// the device holds.
dr_status plan_tail(dr_batch *b)
{
    const int groups = b->opt.tail_at;
    LaunchPlan pl{};
    pl.block = 1024;
    pl.npt = 0;
    pl.chunk = 1;
    pl.fp32 = b->opt.precision == DR_FP32;
    int G = b->opt.tail_group;
    for (int pass = 0; pass < 2; ++pass) {
        const int g_try = G > 0 ? G : 2;
        pl.lds_bytes = glb_lds_bytes(pl.block, g_try, b->n_max);
        if (!pl.fp32 && b->tile_hmax > 0) pl.lds_bytes += 24 * (drk::kTile + b->tile_hmax);
        int cap = 0;
        const int rc = drk::group_grid_capacity(pl.fp32, pl.block, pl.lds_bytes, &cap);
        if (rc != 0) return fail(DR_E_DEVICE, "group kernel occupancy: %s", drk::kernel_error_string(rc));
        if (G == 0) {
            // the largest G whose grid (whole rounds of 8 groups) fits
            G = cap / (8 * ((groups + 7) / 8));
            G = std::min(G, drk::kGroupMax);
            if (G < 2)
                return fail(DR_E_INVALID, "tail_at %d: the device holds %d group workgroups, too few for "
                            "2 per problem", groups, cap);
            continue; // size the LDS for this G
        }
        if (drk::group_grid(groups, G) > cap)
            return fail(DR_E_INVALID, "tail_at %d x tail_group %d needs %d co-resident workgroups; the "
                        "device holds %d", groups, G, drk::group_grid(groups, G), cap);
        break;
    }
    pl.lds_bytes = glb_lds_bytes(pl.block, G, b->n_max);
    // the FP64 group kernel stages tiles as the 1024-thread global build does
    if (!pl.fp32 && b->tile_hmax > 0) pl.lds_bytes += 24 * (drk::kTile + b->tile_hmax);
    b->tail_plan = pl;
    b->tail_group = G;
    return DR_OK;
}

SolveArgs make_args(dr_batch *b, int32_t n_solve, int32_t start, int64_t budget)
{
    SolveArgs a{};
    a.tail_at = 0; // set by launch_or_fail when the hand-off runs
    a.live = b->d_live;
    a.tail_list = b->d_tail_list;
    a.tail_count = b->d_tail_count;
    a.n_begin = b->d_n_begin;
    // workgroups per problem: the tail hand-off's groups, or with the
    // per-pass step every problem's group from the start
    a.group = b->opt.dt_rule == 1 ? b->opt.tail_group : b->tail_group;
    a.gbar = b->d_gbar;
    a.gabort = b->d_gabort;
    a.gpart = b->d_gpart;
    a.probs = b->d_probs;
    a.ids = b->d_ids;
    a.order = b->d_order;
    a.starts = nullptr;
    a.F = b->d_F;
    a.n_solve = n_solve;
    a.start = start;
    a.tol = b->opt.tol;
    a.max_iter = b->opt.max_iter;
    a.budget = budget;
    a.X = b->d_X;
    a.invm = b->d_invm;
    a.mass = b->d_mass;
    a.invm32 = b->d_invm32;
    a.mass32 = b->d_mass32;
    a.deg = b->d_deg;
    a.slice_w = b->d_slice_w;
    a.slice_off = b->d_slice_off;
    a.nbr = b->d_nbr;
    a.lslot = b->d_lslot;
    a.tile_halo = b->d_tile_halo;
    a.halo_ids = b->d_halo_ids;
    a.tile_hmax = b->tile_hmax;
    a.kl = b->d_kl;
    a.kl32 = b->d_kl32;
    a.u = b->d_u;
    a.state_off = b->d_state_off;
    a.qbuf = b->d_qbuf;
    a.qhalf = state_doubles(b->opt.precision) * b->state_nodes;
    a.wbuf = b->d_wbuf;
    a.F_cur = b->d_F_cur;
    a.F_last = b->d_F_last;
    a.has_state = b->d_has_state;
    a.sigma = b->d_sigma;
    a.sigma_fib = b->d_sigma_fib;
    a.iters = b->d_iters;
    a.rho_best = b->d_rho_best;
    a.n_best = b->d_n_best;
    a.stall_window = b->opt.stall_window;
    a.rho = b->d_rho;
    a.ke = b->d_ke;
    a.status = b->d_status;
    a.energy_tol = b->opt.energy_tol;
    a.enode = b->d_enode;
    a.e_work = b->d_e_work;
    a.e_damp = b->d_e_damp;
    a.dt_rule = b->opt.dt_rule;
    a.dt_safety = b->opt.dt_safety;
    a.abuf = b->d_abuf;
    a.dt_next = b->d_dt_next;
    return a;
}

dr_status check_F(const double *F, int32_t k)
{
    const double *f = F + 9 * (int64_t)k;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(f[i])) return fail(DR_E_INVALID, "F of slot %d is not finite", k);
    const double J = f[0] * (f[4] * f[8] - f[5] * f[7]) - f[1] * (f[3] * f[8] - f[5] * f[6]) +
                     f[2] * (f[3] * f[7] - f[4] * f[6]);
    if (!(J > 0.0)) return fail(DR_E_INVALID, "det F of slot %d is not > 0 (%g)", k, J);
    return DR_OK;
}

dr_status check_ids(dr_batch *b, const int32_t *ids, int32_t n_ids)
{
    if (n_ids < 1 || n_ids > b->P)
        return fail(DR_E_INVALID, "n_ids must be in [1, %d] (got %d)", b->P, n_ids);
    if (!ids && n_ids != b->P)
        return fail(DR_E_INVALID, "ids is NULL but n_ids (%d) != n_problems (%d)", n_ids, b->P);
    if (ids) {
        // the batch's preallocated marks, cleared again before returning
        std::vector<char> &seen = b->seen;
        dr_status s = DR_OK;
        int32_t k = 0;
        for (; k < n_ids; ++k) {
            if (ids[k] < 0 || ids[k] >= b->P) {
                s = fail(DR_E_INVALID, "ids[%d] = %d is out of range", k, ids[k]);
                break;
            }
            if (seen[ids[k]]) {
                s = fail(DR_E_INVALID, "ids[%d] = %d is repeated", k, ids[k]);
                break;
            }
            seen[ids[k]] = 1;
        }
        for (int32_t j = 0; j < k; ++j) seen[ids[j]] = 0;
        return s;
    }
    return DR_OK;
}

dr_status check_start(int32_t start, bool allow_resume)
{
    if (start < (allow_resume ? DR_RESUME : DR_START_AFFINE) || start > DR_START_WARM)
        return fail(DR_E_INVALID, "start mode %d is not valid here", start);
    return DR_OK;
}

// Estimated seconds per pass of problem p alone on one compute unit, in its
// class's placement (MI355X measurements of one workgroup per problem): the
// register/LDS variant about 1.5 us + 0.65 ns per fiber; the global
// variant 2.2 us + 2.0 ns per fiber up to 38k fibers and 4.8 ns per fiber
// beyond (its node records no longer stay in the L2 share of one CU).
double pass_cost(const dr_batch *b, int32_t p)
{
    const double M = (double)b->hp[p].M;
    const LaunchPlan &pl = b->classes[b->class_of[p]].plan;
    if (pl.npt > 0 && b->opt.dt_rule == 0) return 1.5e-6 + 0.65e-9 * M;
    if (M <= 37800.0) return 2.2e-6 + 2.0e-9 * M;
    return 2.2e-6 + 2.0e-9 * 37800.0 + 4.8e-9 * (M - 37800.0);
}

// Stages F (may be NULL), ids, starts (may be NULL), per-slot budgets (may
// be NULL) and the costliest-first slot order, and uploads them.  order_slots = false leaves the identity
// order (the launch loop does not use it) and allocates no host memory
// (last_ids holds n_problems from creation on).
dr_status stage(dr_batch *b, const double *F, const int32_t *ids, const int32_t *starts,
                int32_t n_ids, bool order_slots = true, const int64_t *budgets = nullptr)
{
    HIPCHECK(hipEventSynchronize(b->staged)); // previous staging consumed
    if (F) std::memcpy(b->h_F, F, 9 * sizeof(double) * (size_t)n_ids);
    b->last_ids.resize(n_ids);
    for (int32_t k = 0; k < n_ids; ++k) {
        b->h_ids[k] = ids ? ids[k] : k;
        b->last_ids[k] = b->h_ids[k];
        b->h_order[k] = k;
        if (starts) b->h_starts[k] = starts[k];
        if (budgets) b->h_budgets[b->h_ids[k]] = budgets[k];
    }
    // slots grouped by size class; within a class the costliest first
    // (section III: sub-problems converge at different rates): estimated
    // time = pass time x passes of the problem's last solve (the mean over
    // the problems that have one, for those that have none), then size
    if (order_slots) {
        double known = 0.0;
        int64_t nk = 0;
        for (int32_t k = 0; k < n_ids; ++k)
            if (b->last_passes[b->h_ids[k]] > 0) {
                known += (double)b->last_passes[b->h_ids[k]];
                ++nk;
            }
        const double guess = nk > 0 ? known / (double)nk : 1.0;
        std::vector<double> &cost = b->order_cost;
        cost.resize(b->P);
        for (int32_t k = 0; k < n_ids; ++k) {
            const int32_t p = b->h_ids[k];
            cost[p] = pass_cost(b, p) * (b->last_passes[p] > 0 ? (double)b->last_passes[p] : guess);
        }
        std::stable_sort(b->h_order, b->h_order + n_ids, [&](int32_t s, int32_t t) {
            const int32_t ps = b->h_ids[s], pt = b->h_ids[t];
            const int cs = b->class_of[ps], ct = b->class_of[pt];
            if (cs != ct) return cs < ct;
            if (cost[ps] != cost[pt]) return cost[ps] > cost[pt];
            return b->hp[ps].N > b->hp[pt].N;
        });
    }
    std::fill(b->slot_count.begin(), b->slot_count.end(), 0);
    for (int32_t k = 0; k < n_ids; ++k) ++b->slot_count[b->class_of[b->h_ids[k]]];
    for (size_t c = 0, off = 0; c < b->classes.size(); ++c) {
        b->slot_off[c] = (int32_t)off;
        off += b->slot_count[c];
    }
    if (F)
        HIPCHECK(hipMemcpyAsync(b->d_F, b->h_F, 9 * sizeof(double) * (size_t)n_ids,
                                hipMemcpyHostToDevice, b->stream));
    HIPCHECK(hipMemcpyAsync(b->d_ids, b->h_ids, sizeof(int32_t) * (size_t)n_ids,
                            hipMemcpyHostToDevice, b->stream));
    HIPCHECK(hipMemcpyAsync(b->d_order, b->h_order, sizeof(int32_t) * (size_t)n_ids,
                            hipMemcpyHostToDevice, b->stream));
    if (starts)
        HIPCHECK(hipMemcpyAsync(b->d_starts, b->h_starts, sizeof(int32_t) * (size_t)n_ids,
                                hipMemcpyHostToDevice, b->stream));
    if (budgets)
        HIPCHECK(hipMemcpyAsync(b->d_budgets, b->h_budgets, sizeof(int64_t) * (size_t)b->P,
                                hipMemcpyHostToDevice, b->stream));
    if (b->state_off_dirty) {
        std::memcpy(b->h_state_off, b->state_off.data(), sizeof(int64_t) * (size_t)b->P);
        HIPCHECK(hipMemcpyAsync(b->d_state_off, b->h_state_off, sizeof(int64_t) * (size_t)b->P,
                                hipMemcpyHostToDevice, b->stream));
        b->state_off_dirty = false;
    }
    HIPCHECK(hipEventRecord(b->staged, b->stream));
    return DR_OK;
}

// Copies per-problem results for `ids` to the host (waits for the stream).
dr_status gather_results(dr_batch *b, const int32_t *ids, int32_t n, double *sigma,
                         double *sigma_fib, int32_t *result, int64_t *iters, double *resid,
                         double *ke)
{
    const size_t P = (size_t)b->P;
    std::vector<double> sg, sf, rh, kk;
    std::vector<int32_t> stt(P);
    std::vector<int64_t> it(P);
    hipStream_t st = b->stream;
    if (sigma) { sg.resize(9 * P); HIPCHECK(hipMemcpyAsync(sg.data(), b->d_sigma, 9 * P * 8, hipMemcpyDeviceToHost, st)); }
    if (sigma_fib) { sf.resize(9 * P); HIPCHECK(hipMemcpyAsync(sf.data(), b->d_sigma_fib, 9 * P * 8, hipMemcpyDeviceToHost, st)); }
    HIPCHECK(hipMemcpyAsync(stt.data(), b->d_status, P * 4, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(it.data(), b->d_iters, P * 8, hipMemcpyDeviceToHost, st));
    if (resid) { rh.resize(P); HIPCHECK(hipMemcpyAsync(rh.data(), b->d_rho, P * 8, hipMemcpyDeviceToHost, st)); }
    if (ke) { kk.resize(P); HIPCHECK(hipMemcpyAsync(kk.data(), b->d_ke, P * 8, hipMemcpyDeviceToHost, st)); }
    HIPCHECK(hipStreamSynchronize(st));
    for (int32_t k = 0; k < n; ++k) {
        const int32_t p = ids[k];
        if (sigma) std::memcpy(sigma + 9 * (size_t)k, sg.data() + 9 * (size_t)p, 72);
        if (sigma_fib) std::memcpy(sigma_fib + 9 * (size_t)k, sf.data() + 9 * (size_t)p, 72);
        if (result) result[k] = stt[p];
        if (iters) iters[k] = it[p];
        if (resid) resid[k] = rh[p];
        if (ke) ke[k] = kk[p];
    }
    // the stream is idle: refresh the host mirror of running solves and the
    // pass counts of finished ones
    for (size_t p = 0; p < P; ++p) {
        b->running[p] = stt[p] == DR_RUNNING;
        if (stt[p] != DR_RUNNING && stt[p] != drk::kStatusIdle && it[p] > 0) b->last_passes[p] = it[p];
    }
    return DR_OK;
}

// Launches the staged slots: one DR + stress launch per size class with
// slots, concurrently on the class streams (fork / join on the batch stream).
// With the tail hand-off, the problems still running once at most tail_at
// of the launch remain leave their workgroups and a cooperative group launch
// finishes them (tail = false: no hand-off, e.g. under graph capture).
dr_status launch_or_fail(dr_batch *b, const SolveArgs &a_in, bool tail = true)
{
    SolveArgs a = a_in;
    const bool hand_off = tail && b->tail_group > 0 && b->opt.tail_at > 0;
    if (hand_off) {
        a.tail_at = b->opt.tail_at;
        int rc = drk::launch_fill_i32(b->d_live, a.n_solve, 1, b->stream);
        if (rc == 0) rc = drk::launch_fill_i32(b->d_tail_count, 0, 1, b->stream);
        if (rc != 0) return fail(DR_E_DEVICE, "tail counters: %s", drk::kernel_error_string(rc));
    }
    auto tail_launch = [&]() -> dr_status {
        if (!hand_off) return DR_OK;
        SolveArgs at = a;
        at.tail_at = 0;
        at.group = b->tail_group;
        const int rc = drk::launch_tail(at, b->tail_plan, b->opt.tail_at, b->stream);
        if (rc != 0) return fail(DR_E_DEVICE, "group launch failed: %s", drk::kernel_error_string(rc));
        return DR_OK;
    };
    int used = 0, only = -1;
    for (size_t c = 0; c < b->classes.size(); ++c)
        if (b->slot_count[c] > 0) { ++used; only = (int)c; }
    auto one = [&](size_t c, hipStream_t st) -> dr_status {
        SolveArgs ac = a;
        ac.order = a.order + b->slot_off[c];
        ac.n_solve = b->slot_count[c];
        const int rc = drk::launch_solve(ac, b->classes[c].plan, st);
        if (rc != 0) return fail(DR_E_DEVICE, "solve launch failed: %s", drk::kernel_error_string(rc));
        return DR_OK;
    };
    if (used == 1) {
        dr_status s = one((size_t)only, b->stream);
        return s != DR_OK ? s : tail_launch();
    }
    HIPCHECK(hipEventRecord(b->fork, b->stream));
    for (size_t c = 0; c < b->classes.size(); ++c) {
        if (b->slot_count[c] == 0) continue;
        HIPCHECK(hipStreamWaitEvent(b->classes[c].st, b->fork, 0));
        dr_status s = one(c, b->classes[c].st);
        if (s != DR_OK) return s;
        HIPCHECK(hipEventRecord(b->classes[c].done, b->classes[c].st));
    }
    for (size_t c = 0; c < b->classes.size(); ++c)
        if (b->slot_count[c] > 0) HIPCHECK(hipStreamWaitEvent(b->stream, b->classes[c].done, 0));
    return tail_launch();
}

} // namespace


// ---------------------------------------------------------------------------
// Serving pool: continuous batching of solve requests over a resident batch.
// Requests wait in a FIFO queue until admitted (a free slot, room in the
// state budget, no other request of the same network in flight); each poll
// is one dr_advance launch over the in-flight requests (new ones start warm
// from the network's previous solve, the others resume) with a fixed pass
// budget; finished solves retire into a completion queue.
//
// With a state budget, the running state of in-flight solves (two state
// records and one velocity record per node) lives in a device arena of
// budget / state_bytes_per_node records: a request is admitted only when a
// contiguous run of records for its network is free, keeps that run until it
// retires, and the arena is all the running-state memory the pool has.
// What stays resident for every network is its topology, masses and the
// displacements of its last solve (the warm start).
// ---------------------------------------------------------------------------
struct dr_pool {
    dr_batch *b = nullptr;
    int32_t P = 0;
    std::vector<int64_t> nodes; // per network
    int64_t state_budget = 0;   // bytes of running state in flight; 0 = unlimited
    int64_t bytes_per_node = 0; // running state of one node of an in-flight solve
    int64_t arena = 0;          // records of the state arena; 0 = one per node of the pool
    std::map<int64_t, int64_t> free_runs; // arena: first record -> length of a free run
    int32_t max_slots = 0;
    int64_t tick_passes = 0;
    double cost_min = 0.0;      // per-pass cost of the pool's cheapest network
    struct Req {
        int32_t id;
        int64_t tag;
        double F[9];
    };
    struct Flight {
        Req r;
        bool started;
        int64_t rec; // first arena record (arena > 0)
    };
    struct Done {
        int64_t tag;
        int32_t id;
        int32_t result;
        int64_t iters;
        double sigma[9];
    };
    std::deque<Req> queue;
    std::map<int32_t, Flight> active; // by network
    int64_t bytes = 0;
    std::deque<Done> done;
};

namespace {

// First fit: takes a run of n records from the arena's free runs.
bool arena_take(dr_pool *pl, int64_t n, int64_t *first)
{
    for (auto it = pl->free_runs.begin(); it != pl->free_runs.end(); ++it) {
        if (it->second < n) continue;
        *first = it->first;
        const int64_t rest = it->second - n, at = it->first + n;
        pl->free_runs.erase(it);
        if (rest > 0) pl->free_runs[at] = rest;
        return true;
    }
    return false;
}

// Returns a run to the arena, merged with free neighbours.
void arena_give(dr_pool *pl, int64_t first, int64_t n)
{
    auto next = pl->free_runs.lower_bound(first);
    if (next != pl->free_runs.end() && next->first == first + n) {
        n += next->second;
        next = pl->free_runs.erase(next);
    }
    if (next != pl->free_runs.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == first) {
            prev->second += n;
            return;
        }
    }
    pl->free_runs[first] = n;
}

} // namespace

namespace {

// Validation, packing and device set-up shared by dr_batch_create,
// dr_batch_create_in (device arrays carved from ws) and
// dr_batch_workspace_bytes (counting: sizes only, no HIP call).
dr_status create_impl(const dr_networks *nets, const dr_options *opt, void *hip_stream, char *ws,
                      size_t ws_bytes, bool counting, dr_batch **out, size_t *bytes,
                      int64_t arena_nodes = 0)
{
    dr_status s = validate_options(opt);
    if (s != DR_OK) return s;
    Packed pk;
    s = pack(nets, opt, pk);
    if (s != DR_OK) return s;
    if (plan_for(*opt, pk.n_max).npt == -2)
        return fail(DR_E_INVALID, "global placement with 256 threads runs gather chunks of 1 only "
                    "(got %d)", opt->chunk);
    if (plan_for(*opt, pk.n_max).npt < 0)
        return fail(DR_E_INVALID, "placement DR_PLACE_LDS cannot hold a %d-node problem (block %d)",
                    pk.n_max, opt->block);
    if (ws) {
        hipPointerAttribute_t attr;
        int dev = -1;
        if (hipPointerGetAttributes(&attr, ws) != hipSuccess || attr.type != hipMemoryTypeDevice ||
            hipGetDevice(&dev) != hipSuccess || attr.device != dev) {
            (void)hipGetLastError();
            return fail(DR_E_INVALID, "device_workspace is not device memory of the current device");
        }
    }
    dr_batch *b = new dr_batch();
    b->opt = *opt;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->P = nets->n_problems;
    b->total_nodes = nets->node_offsets[b->P];
    b->total_fibers = nets->fiber_offsets[b->P];
    b->total_slices = (int64_t)pk.slice_w.size();
    b->total_inc = (int64_t)pk.nbr.size();
    b->n_max = pk.n_max;
    b->tile_hmax = pk.tile_hmax;
    b->desc = pk.desc;
    b->running.assign(b->P, 0);
    b->last_passes.assign(b->P, 0);
    b->seen.assign(b->P, 0);
    b->last_ids.reserve(b->P);
    // running-state records: each problem at its node_base, or (a pool's
    // arena) placed when a solve is admitted
    b->state_nodes = arena_nodes > 0 ? arena_nodes : b->total_nodes;
    b->state_off.assign(b->P, 0);
    if (arena_nodes <= 0)
        for (int32_t p = 0; p < b->P; ++p) b->state_off[p] = pk.desc[p].node_base;
    b->hp = std::move(pk.hp);
    if (ws || counting) {
        // sizing pass (no HIP call), then the workspace check
        b->counting = true;
        s = create_device(b, pk);
        const size_t need = b->ws_used;
        b->counting = false;
        b->ws_used = 0;
        if (s == DR_OK && counting) *bytes = need;
        if (s != DR_OK || counting) {
            delete b;
            return s;
        }
        if (need > ws_bytes) {
            delete b;
            return fail(DR_E_INVALID, "the workspace holds %zu bytes; the batch needs %zu", ws_bytes, need);
        }
        b->ws = ws;
        b->ws_bytes = ws_bytes;
    }
    s = create_device(b, pk);
    if (s == DR_OK) s = build_classes(b, {});
    if (s == DR_OK && opt->tail_at > 0) s = plan_tail(b);
    if (s == DR_OK) {
        hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e != hipSuccess) s = fail(DR_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    if (s != DR_OK) {
        free_all(b);
        delete b;
        return s;
    }
    *out = b;
    return DR_OK;
}

} // namespace

extern "C" {

void dr_options_default(dr_options *o)
{
    if (!o) return;
    o->precision = DR_FP64;
    o->tol = 1e-8;
    o->max_iter = 2000000;
    o->damping = 1e-3;
    o->dt_safety = 0.9;
    o->block = 0;
    o->placement = DR_PLACE_AUTO;
    o->chunk = 0;
    o->stall_window = 0;
    o->energy_tol = 0.0;
    o->tail_at = 0;
    o->tail_group = 0;
    o->dt_rule = 0;
}

const char *dr_last_error(void) { return g_err.c_str(); }

dr_status dr_batch_create(const dr_networks *nets, const dr_options *opt, void *hip_stream,
                          dr_batch **out)
{
    try {
        g_err.clear();
        if (!out) return fail(DR_E_INVALID, "out is NULL");
        *out = nullptr;
        return create_impl(nets, opt, hip_stream, nullptr, 0, false, out, nullptr);
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_batch_create");
    }
}

dr_status dr_batch_workspace_bytes(const dr_networks *nets, const dr_options *opt, size_t *bytes)
{
    try {
        g_err.clear();
        if (!bytes) return fail(DR_E_INVALID, "bytes is NULL");
        *bytes = 0;
        return create_impl(nets, opt, nullptr, nullptr, 0, true, nullptr, bytes);
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_batch_workspace_bytes");
    }
}

dr_status dr_batch_create_in(const dr_networks *nets, const dr_options *opt, void *hip_stream,
                             void *device_workspace, size_t workspace_bytes, dr_batch **out)
{
    try {
        g_err.clear();
        if (!out) return fail(DR_E_INVALID, "out is NULL");
        *out = nullptr;
        if (!device_workspace) return fail(DR_E_INVALID, "device_workspace is NULL");
        if (reinterpret_cast<uintptr_t>(device_workspace) % kWsAlign != 0)
            return fail(DR_E_INVALID, "device_workspace is not aligned to %zu bytes", kWsAlign);
        return create_impl(nets, opt, hip_stream, static_cast<char *>(device_workspace), workspace_bytes,
                           false, out, nullptr);
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_batch_create_in");
    }
}

dr_status dr_solve(dr_batch *b, const double *F, const int32_t *ids, int32_t n_ids, int32_t start)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!F) return fail(DR_E_INVALID, "F is NULL");
        dr_status s = check_start(start, false);
        if (s != DR_OK) return s;
        if ((s = check_ids(b, ids, n_ids)) != DR_OK) return s;
        for (int32_t k = 0; k < n_ids; ++k)
            if ((s = check_F(F, k)) != DR_OK) return s;
        if ((s = stage(b, F, ids, nullptr, n_ids)) != DR_OK) return s;
        if ((s = launch_or_fail(b, make_args(b, n_ids, start, b->opt.max_iter))) != DR_OK) return s;
        for (int32_t k = 0; k < n_ids; ++k) b->running[b->h_ids[k]] = 0;
        b->last_n = n_ids;
        return DR_OK;
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_solve");
    }
}

dr_status dr_solve_device(dr_batch *b, const double *F_device, const int32_t *ids, int32_t n_ids,
                          int32_t start)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!F_device) return fail(DR_E_INVALID, "F_device is NULL");
        dr_status s = check_start(start, false);
        if (s != DR_OK) return s;
        if ((s = check_ids(b, ids, n_ids)) != DR_OK) return s;
        if ((s = stage(b, nullptr, ids, nullptr, n_ids)) != DR_OK) return s;
        SolveArgs a = make_args(b, n_ids, start, b->opt.max_iter);
        a.F = F_device;
        if ((s = launch_or_fail(b, a)) != DR_OK) return s;
        for (int32_t k = 0; k < n_ids; ++k) b->running[b->h_ids[k]] = 0;
        b->last_n = n_ids;
        return DR_OK;
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_solve_device");
    }
}

namespace {

// dr_advance with one budget for every slot (budgets NULL) or one per slot.
dr_status advance_impl(dr_batch *b, const double *F, const int32_t *ids, const int32_t *starts,
                       int32_t n_ids, int64_t budget, const int64_t *budgets)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!F || !ids || !starts) return fail(DR_E_INVALID, "F, ids and starts are required");
        if (!budgets && budget < 1) return fail(DR_E_INVALID, "budget must be >= 1");
        if (budgets)
            for (int32_t k = 0; k < n_ids; ++k)
                if (budgets[k] < 1) return fail(DR_E_INVALID, "budgets[%d] must be >= 1", k);
        dr_status s = check_ids(b, ids, n_ids);
        if (s != DR_OK) return s;
        for (int32_t k = 0; k < n_ids; ++k) {
            if ((s = check_start(starts[k], true)) != DR_OK) return s;
            if (starts[k] == DR_RESUME) {
                if (!b->running[ids[k]])
                    return fail(DR_E_INVALID, "slot %d resumes problem %d, which is not running", k,
                                ids[k]);
            } else if ((s = check_F(F, k)) != DR_OK) {
                return s;
            }
        }
        if ((s = stage(b, F, ids, starts, n_ids, true, budgets)) != DR_OK) return s;
        SolveArgs a = make_args(b, n_ids, DR_START_AFFINE, budgets ? 1 : budget);
        a.starts = b->d_starts;
        if (budgets) a.budgets = b->d_budgets;
        if ((s = launch_or_fail(b, a)) != DR_OK) return s;
        // Until dr_results reads the device status, every slot may still be running.
        for (int32_t k = 0; k < n_ids; ++k) b->running[ids[k]] = 1;
        b->last_n = n_ids;
        return DR_OK;
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_advance");
    }
}

} // namespace

dr_status dr_advance(dr_batch *b, const double *F, const int32_t *ids, const int32_t *starts,
                     int32_t n_ids, int64_t budget)
{
    return advance_impl(b, F, ids, starts, n_ids, budget, nullptr);
}

dr_status dr_advance_each(dr_batch *b, const double *F, const int32_t *ids, const int32_t *starts,
                          const int64_t *budgets, int32_t n_ids)
{
    if (!budgets) return fail(DR_E_INVALID, "budgets is NULL");
    return advance_impl(b, F, ids, starts, n_ids, 0, budgets);
}

dr_status dr_results(dr_batch *b, const int32_t *ids, int32_t n_ids, double *sigma,
                     double *sigma_fib, int32_t *result, int64_t *iters, double *resid, double *ke)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!ids && n_ids > 0) return fail(DR_E_INVALID, "ids is NULL");
        for (int32_t k = 0; k < n_ids; ++k)
            if (ids[k] < 0 || ids[k] >= b->P)
                return fail(DR_E_INVALID, "ids[%d] = %d is out of range", k, ids[k]);
        return gather_results(b, ids, n_ids, sigma, sigma_fib, result, iters, resid, ke);
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_results");
    }
}

dr_status dr_energy(dr_batch *b, const int32_t *ids, int32_t n_ids, double *work_int,
                    double *work_damp)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!(b->opt.energy_tol > 0.0))
            return fail(DR_E_STATE, "the batch was created without the energy balance (energy_tol 0)");
        dr_status s = check_ids(b, ids, n_ids);
        if (s != DR_OK) return s;
        std::vector<double> w((size_t)b->P), d((size_t)b->P);
        HIPCHECK(hipStreamSynchronize(b->stream));
        HIPCHECK(hipMemcpy(w.data(), b->d_e_work, sizeof(double) * b->P, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(d.data(), b->d_e_damp, sizeof(double) * b->P, hipMemcpyDeviceToHost));
        for (int32_t k = 0; k < n_ids; ++k) {
            const int32_t p = ids ? ids[k] : k;
            if (work_int) work_int[k] = w[p];
            if (work_damp) work_damp[k] = d[p];
        }
        return DR_OK;
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_energy");
    }
}

dr_status dr_sync(dr_batch *b)
{
    g_err.clear();
    if (!b) return fail(DR_E_INVALID, "batch is NULL");
    HIPCHECK(hipStreamSynchronize(b->stream));
    return DR_OK;
}

dr_status dr_stress(dr_batch *b, double *sigma, double *sigma_fib, double *u, int32_t *result,
                    int64_t *iters, double *resid, double *ke)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (b->last_n < 0) return fail(DR_E_STATE, "dr_stress called before any dr_solve");
        dr_status s = gather_results(b, b->last_ids.data(), b->last_n, sigma, sigma_fib, result,
                                     iters, resid, ke);
        if (s != DR_OK) return s;
        if (u) {
            std::vector<double> ur(3 * (size_t)b->total_nodes);
            HIPCHECK(hipMemcpyAsync(ur.data(), b->d_u, ur.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, b->stream));
            HIPCHECK(hipStreamSynchronize(b->stream));
            for (int32_t p = 0; p < b->P; ++p) {
                const HostProblem &h = b->hp[p];
                const int64_t nb = b->desc[p].node_base;
                for (int32_t i = 0; i < h.N; ++i) {
                    const int64_t src = 3 * (nb + h.new_of_old[i]);
                    const int64_t dst = 3 * (h.in_node_base + i);
                    u[dst] = ur[src];
                    u[dst + 1] = ur[src + 1];
                    u[dst + 2] = ur[src + 2];
                }
            }
        }
        return DR_OK;
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_stress");
    }
}

namespace {

// The per-problem launch loop: one problem after the other, a few kernels per
// pass and the stop test on the host.  scatter: forces by the zero + atomic
// scatter kernel instead of the deterministic gather.  noalloc: the scratch
// (force accumulators, partial sums, scalars) comes from the library's fixed
// per-device array instead of the batch's buffers, and nothing is allocated.
dr_status solve_loop(dr_batch *b, const double *F, const int32_t *ids, int32_t n_ids,
                     int32_t start, bool scatter, bool noalloc = false)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!F) return fail(DR_E_INVALID, "F is NULL");
        if (b->opt.precision != DR_FP64)
            return fail(DR_E_INVALID, "the launch-loop comparator is FP64 only");
        if (b->opt.dt_rule != 0)
            return fail(DR_E_INVALID, "the launch-loop comparator runs the constant step only");
        dr_status s = check_start(start, false);
        if (s != DR_OK) return s;
        if ((s = check_ids(b, ids, n_ids)) != DR_OK) return s;
        for (int32_t k = 0; k < n_ids; ++k)
            if ((s = check_F(F, k)) != DR_OK) return s;
        double *gbuf = b->d_gscat, *partial = b->d_partial, *scalars = b->d_scalars;
        if (noalloc) {
            for (int32_t k = 0; k < n_ids; ++k) {
                const int32_t p = ids ? ids[k] : k;
                if (b->hp[p].N > drk::kNoAllocMaxNodes)
                    return fail(DR_E_INVALID, "problem %d has %d nodes; the allocation-free loop takes "
                                "at most %d", p, b->hp[p].N, drk::kNoAllocMaxNodes);
            }
            HIPCHECK(hipSetDevice(b->device));
            void *base = nullptr;
            const int rc = drk::noalloc_scratch(&base);
            if (rc != 0) return fail(DR_E_DEVICE, "scratch address: %s", drk::kernel_error_string(rc));
            char *c = static_cast<char *>(base);
            gbuf = reinterpret_cast<double *>(c + drk::kNoAllocForceOff);
            partial = reinterpret_cast<double *>(c + drk::kNoAllocPartialOff);
            scalars = reinterpret_cast<double *>(c + drk::kNoAllocScalarOff);
        } else if (scatter && !b->d_gscat) {
            HIPCHECK(hipMalloc(&b->d_gscat, sizeof(double) * 3 * (size_t)std::max(b->n_max, 1)));
            gbuf = b->d_gscat;
        }
        if ((s = stage(b, F, ids, nullptr, n_ids, false)) != DR_OK) return s;
        SolveArgs a = make_args(b, n_ids, start, b->opt.max_iter);
        a.order = nullptr;
        hipStream_t st = b->stream;
        for (int32_t slot = 0; slot < n_ids; ++slot) {
            const ProbDesc &d = b->desc[b->h_ids[slot]];
            int rc = drk::launch_loop_kernels(a, slot, 0, d.N, partial, scalars, 0, 0.0,
                                              0.0, 0, gbuf, st);
            if (rc != 0) return fail(DR_E_DEVICE, "loop set-up launch failed: %s", drk::kernel_error_string(rc));
            int64_t n = 0;
            double rho = 0.0, ke = 0.0;
            int status = DR_MAX_ITER;
            for (;;) {
                rc = drk::launch_loop_kernels(a, slot, scatter ? 3 : 1, d.N, partial, scalars, n, 0.0,
                                              0.0, 0, gbuf, st);
                if (rc != 0) return fail(DR_E_DEVICE, "loop pass launch failed: %s", drk::kernel_error_string(rc));
                HIPCHECK(hipMemcpyAsync(b->h_scalars, scalars, 3 * sizeof(double),
                                        hipMemcpyDeviceToHost, st));
                HIPCHECK(hipStreamSynchronize(st));
                ++n;
                double den = std::sqrt(b->h_scalars[1]);
                if (den < d.s_floor) den = d.s_floor;
                rho = std::sqrt(b->h_scalars[0]) / den;
                ke = 0.5 * b->h_scalars[2];
                if (!std::isfinite(rho) || !std::isfinite(ke)) { status = DR_NONFINITE; break; }
                if (rho <= b->opt.tol) { status = DR_CONVERGED; break; }
                if (n >= b->opt.max_iter) { status = DR_MAX_ITER; break; }
            }
            rc = drk::launch_loop_kernels(a, slot, 2, d.N, partial, scalars, n, rho, ke, status, gbuf,
                                          st);
            if (rc != 0) return fail(DR_E_DEVICE, "loop stress launch failed: %s", drk::kernel_error_string(rc));
            b->running[b->h_ids[slot]] = 0;
        }
        HIPCHECK(hipStreamSynchronize(st));
        b->last_n = n_ids;
        return DR_OK;
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_solve_loop");
    }
}

} // namespace

dr_status dr_solve_loop(dr_batch *b, const double *F, const int32_t *ids, int32_t n_ids,
                        int32_t start)
{
    return solve_loop(b, F, ids, n_ids, start, false);
}

dr_status dr_solve_loop_scatter(dr_batch *b, const double *F, const int32_t *ids, int32_t n_ids,
                                int32_t start)
{
    return solve_loop(b, F, ids, n_ids, start, true);
}

dr_status dr_solve_loop_scatter_noalloc(dr_batch *b, const double *F, const int32_t *ids,
                                        int32_t n_ids, int32_t start)
{
    return solve_loop(b, F, ids, n_ids, start, true, true);
}

dr_status dr_batch_info(const dr_batch *b, int32_t *n_problems, int64_t *total_nodes,
                        int64_t *total_fibers, int32_t *block, int32_t *lds_bytes,
                        int32_t *nodes_per_thread)
{
    g_err.clear();
    if (!b) return fail(DR_E_INVALID, "batch is NULL");
    // the class holding the largest problem
    const LaunchPlan &pl = b->classes[b->class_of[0]].plan;
    size_t big = 0;
    for (int32_t p = 0; p < b->P; ++p)
        if (b->hp[p].N == b->n_max) { big = (size_t)b->class_of[p]; break; }
    const LaunchPlan &pb = b->classes[big].plan;
    (void)pl;
    if (n_problems) *n_problems = b->P;
    if (total_nodes) *total_nodes = b->total_nodes;
    if (total_fibers) *total_fibers = b->total_fibers;
    if (block) *block = pb.block;
    if (lds_bytes) *lds_bytes = pb.lds_bytes;
    if (nodes_per_thread) *nodes_per_thread = pb.npt;
    return DR_OK;
}

dr_status dr_batch_class_info(const dr_batch *b, int32_t c, int32_t *n_classes, int32_t *n_lo,
                              int32_t *n_hi, int32_t *n_problems, int32_t *block,
                              int32_t *nodes_per_thread, int32_t *chunk, int32_t *lds_bytes)
{
    g_err.clear();
    if (!b) return fail(DR_E_INVALID, "batch is NULL");
    if (n_classes) *n_classes = (int32_t)b->classes.size();
    if (c < 0 || c >= (int32_t)b->classes.size())
        return fail(DR_E_INVALID, "class %d out of range (%d classes)", c, (int)b->classes.size());
    const auto &k = b->classes[c];
    if (n_lo) *n_lo = k.n_lo;
    if (n_hi) *n_hi = k.n_hi;
    if (n_problems) *n_problems = k.count;
    if (block) *block = k.plan.block;
    if (nodes_per_thread) *nodes_per_thread = k.plan.npt;
    if (chunk) *chunk = k.plan.chunk;
    if (lds_bytes) *lds_bytes = k.plan.lds_bytes;
    return DR_OK;
}

dr_status dr_set_class_plans(dr_batch *b, int32_t n_classes, const int32_t *n_hi,
                             const int32_t *block, const int32_t *chunk, const int32_t *placement)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (n_classes < 0 || n_classes > 16) return fail(DR_E_INVALID, "n_classes must be in [0, 16]");
        if (n_classes > 0 && (!n_hi || !block || !chunk || !placement))
            return fail(DR_E_INVALID, "a class-plan array is NULL");
        std::vector<ClassRequest> req;
        for (int32_t k = 0; k < n_classes; ++k) {
            if (k > 0 && n_hi[k] <= n_hi[k - 1])
                return fail(DR_E_INVALID, "n_hi must increase (class %d)", k);
            if (n_hi[k] < 1) return fail(DR_E_INVALID, "n_hi of class %d must be >= 1", k);
            if (block[k] != 0 && block[k] != 256 && block[k] != 512 && block[k] != 1024)
                return fail(DR_E_INVALID, "block of class %d must be 0, 256, 512 or 1024", k);
            if (chunk[k] != 0 && chunk[k] != 1 && chunk[k] != 2 && chunk[k] != 4)
                return fail(DR_E_INVALID, "chunk of class %d must be 0, 1, 2 or 4", k);
            if (placement[k] < DR_PLACE_AUTO || placement[k] > DR_PLACE_GLOBAL)
                return fail(DR_E_INVALID, "placement of class %d is not a dr_placement value", k);
            req.push_back(ClassRequest{n_hi[k], block[k], chunk[k], placement[k]});
        }
        // Launch shapes do not change results, so plans may change between
        // solves: wait for the batch's work (the class streams join it), and
        // drop a captured graph, which holds the old shapes.
        HIPCHECK(hipStreamSynchronize(b->stream));
        if (b->graph_exec) { (void)hipGraphExecDestroy(b->graph_exec); b->graph_exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        return build_classes(b, req);
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_set_class_plans");
    }
}

dr_status dr_graph_capture(dr_batch *b, const double *F_device, const int32_t *ids, int32_t n_ids,
                           int32_t start)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!F_device) return fail(DR_E_INVALID, "F_device is NULL");
        if (!b->stream)
            return fail(DR_E_STATE, "graph capture needs a batch created on a non-default stream");
        dr_status s = check_start(start, false);
        if (s != DR_OK) return s;
        if ((s = check_ids(b, ids, n_ids)) != DR_OK) return s;
        if ((s = stage(b, nullptr, ids, nullptr, n_ids)) != DR_OK) return s;
        HIPCHECK(hipStreamSynchronize(b->stream));
        if (b->graph_exec) { (void)hipGraphExecDestroy(b->graph_exec); b->graph_exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        SolveArgs a = make_args(b, n_ids, start, b->opt.max_iter);
        a.F = F_device;
        HIPCHECK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        s = launch_or_fail(b, a, false); // the cooperative group launch is not captured
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (s != DR_OK) { if (g) (void)hipGraphDestroy(g); return s; }
        if (e != hipSuccess) return fail(DR_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        b->graph = g;
        HIPCHECK(hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0));
        b->graph_ids = b->last_ids;
        return DR_OK;
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_graph_capture");
    }
}

dr_status dr_graph_launch(dr_batch *b)
{
    try {
        g_err.clear();
        if (!b) return fail(DR_E_INVALID, "batch is NULL");
        if (!b->graph_exec) return fail(DR_E_STATE, "no captured solve (dr_graph_capture)");
        // the slot arrays the graph's kernels read are re-staged first
        dr_status s = stage(b, nullptr, b->graph_ids.data(), nullptr, (int32_t)b->graph_ids.size());
        if (s != DR_OK) return s;
        HIPCHECK(hipGraphLaunch(b->graph_exec, b->stream));
        for (int32_t p : b->graph_ids) b->running[p] = 0;
        b->last_n = (int32_t)b->graph_ids.size();
        return DR_OK;
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_graph_launch");
    }
}

dr_status dr_batch_pass_costs(const dr_batch *b, double *seconds)
{
    g_err.clear();
    if (!b) return fail(DR_E_INVALID, "batch is NULL");
    if (!seconds) return fail(DR_E_INVALID, "seconds is NULL");
    for (int32_t p = 0; p < b->P; ++p) seconds[p] = pass_cost(b, p);
    return DR_OK;
}

dr_status dr_batch_scalars(const dr_batch *b, double *dt, double *c, double *s_floor)
{
    g_err.clear();
    if (!b) return fail(DR_E_INVALID, "batch is NULL");
    for (int32_t p = 0; p < b->P; ++p) {
        if (dt) dt[p] = b->desc[p].dt;
        if (c) c[p] = b->desc[p].c;
        if (s_floor) s_floor[p] = b->desc[p].s_floor;
    }
    return DR_OK;
}

void dr_batch_destroy(dr_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    free_all(b);
    delete b;
}

dr_status dr_pool_create(const dr_networks *nets, const dr_options *opt, void *hip_stream,
                         int64_t state_budget_bytes, int32_t max_slots, int64_t tick_passes,
                         dr_pool **out)
{
    try {
        g_err.clear();
        if (!out) return fail(DR_E_INVALID, "out is NULL");
        *out = nullptr;
        if (state_budget_bytes < 0)
            return fail(DR_E_INVALID, "state_budget_bytes must be >= 0 (got %lld)", (long long)state_budget_bytes);
        if (max_slots < 1) return fail(DR_E_INVALID, "max_slots must be >= 1 (got %d)", max_slots);
        if (tick_passes < 1)
            return fail(DR_E_INVALID, "tick_passes must be >= 1 (got %lld)", (long long)tick_passes);
        dr_status s = validate_options(opt);
        if (s != DR_OK) return s;
        if (!nets || nets->n_problems < 1 || !nets->node_offsets)
            return fail(DR_E_INVALID, "networks is NULL or empty");
        const int64_t bpn = state_bytes_per_node(opt->precision);
        const int64_t total = nets->node_offsets[nets->n_problems];
        // an arena only when the budget holds less than every network's state
        int64_t arena = state_budget_bytes / bpn;
        if (state_budget_bytes > 0 && arena < 1)
            return fail(DR_E_INVALID, "state_budget_bytes %lld holds no node's running state (%lld B)",
                        (long long)state_budget_bytes, (long long)bpn);
        if (state_budget_bytes == 0 || arena >= total) arena = 0;
        dr_batch *b = nullptr;
        s = create_impl(nets, opt, hip_stream, nullptr, 0, false, &b, nullptr, arena);
        if (s != DR_OK) return s;
        dr_pool *pl = new dr_pool();
        pl->b = b;
        pl->P = nets->n_problems;
        pl->nodes.resize(pl->P);
        for (int32_t p = 0; p < pl->P; ++p) pl->nodes[p] = nets->node_offsets[p + 1] - nets->node_offsets[p];
        pl->bytes_per_node = bpn;
        pl->arena = arena;
        if (arena > 0) pl->free_runs[0] = arena;
        pl->state_budget = state_budget_bytes;
        pl->max_slots = max_slots;
        pl->tick_passes = tick_passes;
        pl->cost_min = 1e300;
        for (int32_t p = 0; p < pl->P; ++p) pl->cost_min = std::min(pl->cost_min, pass_cost(b, p));
        *out = pl;
        return DR_OK;
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_pool_create");
    }
}

dr_status dr_pool_submit(dr_pool *pl, int32_t id, const double *F, int64_t tag)
{
    try {
        g_err.clear();
        if (!pl) return fail(DR_E_INVALID, "pool is NULL");
        if (!F) return fail(DR_E_INVALID, "F is NULL");
        if (id < 0 || id >= pl->P) return fail(DR_E_INVALID, "network %d out of range [0, %d)", id, pl->P);
        dr_status s = check_F(F, 0);
        if (s != DR_OK) return s;
        const int64_t need = pl->bytes_per_node * pl->nodes[id];
        if (pl->state_budget > 0 && need > pl->state_budget)
            return fail(DR_E_INVALID, "network %d alone needs %lld state bytes, over the budget of %lld", id,
                        (long long)need, (long long)pl->state_budget);
        dr_pool::Req r;
        r.id = id;
        r.tag = tag;
        std::memcpy(r.F, F, sizeof(r.F));
        pl->queue.push_back(r);
        return DR_OK;
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_pool_submit");
    }
}

dr_status dr_pool_poll(dr_pool *pl, int32_t max_out, int64_t *tags, int32_t *ids, double *sigma,
                       int32_t *result, int64_t *iters, int32_t *n_out)
{
    try {
        g_err.clear();
        if (!pl) return fail(DR_E_INVALID, "pool is NULL");
        if (!n_out) return fail(DR_E_INVALID, "n_out is NULL");
        *n_out = 0;
        if (max_out < 0) return fail(DR_E_INVALID, "max_out must be >= 0 (got %d)", max_out);
        // admission, FIFO: a request whose network is busy waits without
        // blocking the ones behind it; one blocked by slots or budget blocks
        std::deque<dr_pool::Req> kept;
        while (!pl->queue.empty()) {
            const dr_pool::Req r = pl->queue.front();
            if (pl->active.count(r.id)) {
                kept.push_back(r);
                pl->queue.pop_front();
                continue;
            }
            const int64_t need = pl->bytes_per_node * pl->nodes[r.id];
            if ((int32_t)pl->active.size() >= pl->max_slots ||
                (pl->state_budget > 0 && pl->bytes + need > pl->state_budget))
                break;
            int64_t rec = 0;
            if (pl->arena > 0) {
                if (!arena_take(pl, pl->nodes[r.id], &rec)) break; // no free run long enough
                pl->b->state_off[r.id] = rec;
                pl->b->state_off_dirty = true;
            }
            pl->active[r.id] = dr_pool::Flight{r, false, rec};
            pl->bytes += need;
            pl->queue.pop_front();
        }
        for (auto it = pl->queue.begin(); it != pl->queue.end(); ++it) kept.push_back(*it);
        pl->queue.swap(kept);
        // one tick over the in-flight requests
        const int32_t n = (int32_t)pl->active.size();
        if (n > 0) {
            std::vector<int32_t> slot_ids(n), starts(n), res(n);
            std::vector<double> F(9 * (size_t)n), sig(9 * (size_t)n), cost(n);
            std::vector<int64_t> it(n), budgets(n);
            int32_t k = 0;
            for (auto &kv : pl->active) {
                slot_ids[k] = kv.first;
                starts[k] = kv.second.started ? DR_RESUME : DR_START_WARM;
                std::memcpy(&F[9 * (size_t)k], kv.second.r.F, 9 * sizeof(double));
                cost[k] = pass_cost(pl->b, kv.first);
                ++k;
            }
            // balanced tick of a fixed length, tick_passes passes of the
            // pool's cheapest network: every solve makes as many passes as
            // fit that time, so the launch's compute units finish together
            // instead of waiting for the slowest, and a tick stays short
            // whatever mix of networks is in flight
            for (k = 0; k < n; ++k)
                budgets[k] = std::max<int64_t>(
                    1, (int64_t)std::llround((double)pl->tick_passes * pl->cost_min / cost[k]));
            dr_status s = advance_impl(pl->b, F.data(), slot_ids.data(), starts.data(), n, 0, budgets.data());
            if (s != DR_OK) return s;
            for (auto &kv : pl->active) kv.second.started = true;
            s = dr_results(pl->b, slot_ids.data(), n, sig.data(), nullptr, res.data(), it.data(), nullptr,
                           nullptr);
            if (s != DR_OK) return s;
            for (k = 0; k < n; ++k) {
                if (res[k] == DR_RUNNING) continue;
                auto f = pl->active.find(slot_ids[k]);
                dr_pool::Done d;
                d.tag = f->second.r.tag;
                d.id = slot_ids[k];
                d.result = res[k];
                d.iters = it[k];
                std::memcpy(d.sigma, &sig[9 * (size_t)k], sizeof(d.sigma));
                pl->done.push_back(d);
                pl->bytes -= pl->bytes_per_node * pl->nodes[slot_ids[k]];
                if (pl->arena > 0) arena_give(pl, f->second.rec, pl->nodes[slot_ids[k]]);
                pl->active.erase(f);
            }
        }
        // completions, oldest first
        int32_t m = 0;
        while (m < max_out && !pl->done.empty()) {
            const dr_pool::Done &d = pl->done.front();
            if (tags) tags[m] = d.tag;
            if (ids) ids[m] = d.id;
            if (sigma) std::memcpy(sigma + 9 * (size_t)m, d.sigma, sizeof(d.sigma));
            if (result) result[m] = d.result;
            if (iters) iters[m] = d.iters;
            pl->done.pop_front();
            ++m;
        }
        *n_out = m;
        return DR_OK;
    } catch (const std::bad_alloc &) {
        return fail(DR_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(DR_E_INVALID, "unexpected exception in dr_pool_poll");
    }
}

dr_status dr_pool_status(const dr_pool *pl, int32_t *queued, int32_t *in_flight, int32_t *completed,
                         int64_t *state_bytes)
{
    g_err.clear();
    if (!pl) return fail(DR_E_INVALID, "pool is NULL");
    if (queued) *queued = (int32_t)pl->queue.size();
    if (in_flight) *in_flight = (int32_t)pl->active.size();
    if (completed) *completed = (int32_t)pl->done.size();
    if (state_bytes) *state_bytes = pl->bytes;
    return DR_OK;
}

dr_status dr_state_bytes_per_node(int32_t precision, int64_t *bytes)
{
    g_err.clear();
    if (!bytes) return fail(DR_E_INVALID, "bytes is NULL");
    if (precision != DR_FP64 && precision != DR_FP32)
        return fail(DR_E_INVALID, "precision %d is not DR_FP64 or DR_FP32", precision);
    *bytes = state_bytes_per_node(precision);
    return DR_OK;
}

void dr_pool_destroy(dr_pool *pl)
{
    if (!pl) return;
    dr_batch_destroy(pl->b);
    delete pl;
}

} // extern "C"
