// HIP kernels for batched dynamic relaxation on CDNA4 (gfx950).
//
// One workgroup runs the whole dynamic-relaxation loop of Fig. 1 for one
// sub-problem (section III: the loop moved inside a single kernel, one thread
// team per sub-problem).  Per pass, every thread
//   1. moves its free nodes: x += dt w            (w = half-step velocity)
//   2. barrier
//   3. gathers the internal force on each of its nodes over the node's
//      incidences (deterministic node -> fiber gather, no atomics)
//   4. forms the damped acceleration, the full-step and next half-step
//      velocities, and its share of |g_free|^2, |g_B|^2 and 2 KE
//   5. wavefront reduction -> LDS -> every thread sums the wave partials in
//      the same fixed order, so the stop decision is uniform.
// After the loop the final displacements go to HBM and a separate launch
// (k_stress) gathers the reactions and both stress forms from them.
//
// Two placements:
//   k_dr_reg<BLOCK, NPT>: positions in LDS (SoA), the half-step velocity and
//     degree of each owned node in registers, NPT nodes per thread; for
//     problems whose positions fit in LDS (3 * 8 B per node).
//   k_dr_glb<BLOCK>: positions and half-step velocities in device memory,
//     any problem size.
// In both, the topology (neighbour id and fiber constants) streams from
// device memory every pass; it is read-only and stays in L2 / MALL.
#include <hip/hip_runtime.h>

#include "dr_layout.h"

namespace drk {

enum { kConverged = 0, kMaxIter = 1, kNonFinite = 2 };
enum { kStartAffine = 0, kStartZero = 1, kStartWarm = 2 };

// Partial sums kept per wave in LDS: 3 per pass, 18 in the stress epilogue.
constexpr int kRedStride = 20;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct LdsPos {
    double *xs, *ys, *zs;
    __device__ __forceinline__ void load(int j, double &x, double &y, double &z) const
    {
        x = xs[j]; y = ys[j]; z = zs[j];
    }
    __device__ __forceinline__ void store(int j, double x, double y, double z) const
    {
        xs[j] = x; ys[j] = y; zs[j] = z;
    }
};

struct GlbPos {
    double *base; // 4 doubles per node
    __device__ __forceinline__ void load(int j, double &x, double &y, double &z) const
    {
        const double2 a = *reinterpret_cast<const double2 *>(base + 4 * (int64_t)j);
        x = a.x; y = a.y; z = base[4 * (int64_t)j + 2];
    }
    __device__ __forceinline__ void store(int j, double x, double y, double z) const
    {
        *reinterpret_cast<double2 *>(base + 4 * (int64_t)j) = make_double2(x, y);
        base[4 * (int64_t)j + 2] = z;
    }
};

// Slice of node r: first entry (without the lane offset) and width.
struct Row {
    int64_t e0;
    int width;
};

__device__ __forceinline__ Row node_row(const SolveArgs &A, const ProbDesc &P, int r)
{
    const int q = __builtin_amdgcn_readfirstlane(r >> 6);
    Row row;
    row.width = A.slice_w[P.slice_base + q];
    row.e0 = P.inc_base + A.slice_off[P.slice_base + q];
    return row;
}

// Squared length, rounded as the host rounds L^2 (no fused multiply-add), so
// a fiber at its reference length carries exactly zero force.
__device__ __forceinline__ double len2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

// Internal force on node r (Fig. 1, getInternalForces): sum over the node's
// fibers of T d / l with d = x_j - x_i and T = EA (l^2 / L^2 - 1) / 2
// = k (l^2 - L^2), k = EA / (2 L^2).
template <class Pos>
__device__ __forceinline__ void gather_force(const SolveArgs &A, const Row &row, const Pos &pos,
                                             int lane, int d, double xi, double yi, double zi,
                                             double &gx, double &gy, double &gz)
{
    gx = 0.0; gy = 0.0; gz = 0.0;
    const int64_t e0 = row.e0 + lane;
    for (int k = 0; k < row.width; ++k) {
        if (k < d) {
            const int64_t e = e0 + (int64_t)k * kWave;
            const int j = A.nbr[e];
            const KL c = A.kl[e];
            double xj, yj, zj;
            pos.load(j, xj, yj, zj);
            const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
            const double l2 = len2(dx, dy, dz);
            const double s = c.k * (l2 - c.L2) * rsqrt(l2);
            gx += s * dx; gy += s * dy; gz += s * dz;
        }
    }
}

// Same gather, also accumulating 1/2 (T / l) d (x) d into the fiber stress
// (each fiber is visited from both ends).
template <class Pos>
__device__ __forceinline__ void gather_force_stress(const SolveArgs &A, const Row &row,
                                                    const Pos &pos, int lane, int d, double xi,
                                                    double yi, double zi, double &gx, double &gy,
                                                    double &gz, double *sf)
{
    gx = 0.0; gy = 0.0; gz = 0.0;
    const int64_t e0 = row.e0 + lane;
    for (int k = 0; k < row.width; ++k) {
        if (k < d) {
            const int64_t e = e0 + (int64_t)k * kWave;
            const int j = A.nbr[e];
            const KL c = A.kl[e];
            double xj, yj, zj;
            pos.load(j, xj, yj, zj);
            const double dv[3] = {xj - xi, yj - yi, zj - zi};
            const double l2 = len2(dv[0], dv[1], dv[2]);
            const double s = c.k * (l2 - c.L2) * rsqrt(l2);
            gx += s * dv[0]; gy += s * dv[1]; gz += s * dv[2];
            const double hs = 0.5 * s;
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) sf[3 * p + q] += hs * dv[p] * dv[q];
        }
    }
}

struct Solve {
    ProbDesc P;
    int slot, p;
    double F[9];
    double Fl[9];
    bool warm;
};

__device__ __forceinline__ Solve load_solve(const SolveArgs &A)
{
    Solve S;
    S.slot = A.order ? A.order[blockIdx.x] : (int)blockIdx.x;
    S.p = A.ids ? A.ids[S.slot] : S.slot;
    S.P = A.probs[S.p];
#pragma unroll
    for (int k = 0; k < 9; ++k) S.F[k] = A.F[9 * (int64_t)S.slot + k];
    S.warm = (A.start == kStartWarm) && A.has_state[S.p];
#pragma unroll
    for (int k = 0; k < 9; ++k) S.Fl[k] = S.warm ? A.F_last[9 * (int64_t)S.p + k] : S.F[k];
    return S;
}

// Start position of local node r (Fig. 1 step 4 and the initialisation):
// prescribed nodes x = F X; free nodes from the affine field, from u = 0, or
// warm (u_prev + (F - F_prev) X).
__device__ __forceinline__ void start_position(const SolveArgs &A, const Solve &S, int r,
                                               double x[3])
{
    const int64_t gi = S.P.node_base + r;
    const double X[3] = {A.X[3 * gi], A.X[3 * gi + 1], A.X[3 * gi + 2]};
    const bool free_node = r < S.P.N_free;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double u;
        const double fx = (S.F[3 * a] - (a == 0 ? 1.0 : 0.0)) * X[0] +
                          (S.F[3 * a + 1] - (a == 1 ? 1.0 : 0.0)) * X[1] +
                          (S.F[3 * a + 2] - (a == 2 ? 1.0 : 0.0)) * X[2];
        if (!free_node || A.start == kStartAffine || (A.start == kStartWarm && !S.warm)) {
            u = fx;
        } else if (A.start == kStartZero) {
            u = 0.0;
        } else {
            const double dfx = (S.F[3 * a] - S.Fl[3 * a]) * X[0] +
                               (S.F[3 * a + 1] - S.Fl[3 * a + 1]) * X[1] +
                               (S.F[3 * a + 2] - S.Fl[3 * a + 2]) * X[2];
            u = A.u[3 * gi + a] + dfx;
        }
        x[a] = X[a] + u;
    }
}

// Displacement written back for node r at the end of a solve.
__device__ __forceinline__ void write_u(const SolveArgs &A, const Solve &S, int r, const double x[3])
{
    const int64_t gi = S.P.node_base + r;
    const double X[3] = {A.X[3 * gi], A.X[3 * gi + 1], A.X[3 * gi + 2]};
    if (r < S.P.N_free) {
#pragma unroll
        for (int a = 0; a < 3; ++a) A.u[3 * gi + a] = x[a] - X[a];
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            A.u[3 * gi + a] = (S.F[3 * a] - (a == 0 ? 1.0 : 0.0)) * X[0] +
                              (S.F[3 * a + 1] - (a == 1 ? 1.0 : 0.0)) * X[1] +
                              (S.F[3 * a + 2] - (a == 2 ? 1.0 : 0.0)) * X[2];
    }
}

// Block-wide sums of three values; every thread returns the same totals
// (fixed summation order over waves).
template <int NW>
__device__ __forceinline__ void block_sum3(double *red, int lane, int wave, double &a, double &b,
                                           double &c)
{
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c);
    if (lane == 0) {
        red[wave * kRedStride + 0] = a;
        red[wave * kRedStride + 1] = b;
        red[wave * kRedStride + 2] = c;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0, tc = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        ta += red[w * kRedStride + 0];
        tb += red[w * kRedStride + 1];
        tc += red[w * kRedStride + 2];
    }
    a = ta; b = tb; c = tc;
}

// Residual and stop test (Fig. 1: force residual, iteration count, until
// converged).  Returns true when the loop must end.
__device__ __forceinline__ bool stop_test(const SolveArgs &A, const ProbDesc &P, double gf2,
                                          double gb2, double ke2, int64_t n, double &rho,
                                          double &ke, int &status)
{
    double den = sqrt(gb2);
    if (den < P.s_floor) den = P.s_floor;
    rho = sqrt(gf2) / den;
    ke = 0.5 * ke2;
    if (!isfinite(rho) || !isfinite(ke)) { status = kNonFinite; return true; }
    if (rho <= A.tol) { status = kConverged; return true; }
    if (n >= A.max_iter) { status = kMaxIter; return true; }
    return false;
}

// End of a solve: iteration count, residual, energy and status of the slot,
// and the state kept for a warm start (thread 0 writes).
__device__ __forceinline__ void finish_solve(const SolveArgs &A, const Solve &S, int tid, int64_t n,
                                             double rho, double ke, int status)
{
    if (tid == 0) {
        A.iters[S.slot] = n;
        A.rho[S.slot] = rho;
        A.ke[S.slot] = ke;
        A.status[S.slot] = status;
        for (int k = 0; k < 9; ++k) A.F_last[9 * (int64_t)S.p + k] = S.F[k];
        A.has_state[S.p] = 1;
    }
}

__device__ __forceinline__ void fc0_of(const double *F, double fc0[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) fc0[a] = 0.5 * (F[3 * a] + F[3 * a + 1] + F[3 * a + 2]);
}

// ---------------------------------------------------------------------------
// Register-resident variant: positions in LDS, the half-step velocity and the
// degree of each owned node in registers (7 VGPRs per node); 1/m and m are
// re-read from L2 every pass.
// ---------------------------------------------------------------------------
template <int BLOCK, int NPT>
__global__ void __launch_bounds__(BLOCK) k_dr_reg(SolveArgs A)
{
    extern __shared__ double smem[];
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const Solve S = load_solve(A);
    const ProbDesc &P = S.P;
    const int N = P.N, Nf = P.N_free;
    double *red = smem;
    const LdsPos pos{smem + NW * kRedStride, smem + NW * kRedStride + N,
                     smem + NW * kRedStride + 2 * N};
    const double dt = P.dt, hdt = 0.5 * P.dt, cdamp = P.c;
    const double *invm = A.invm + P.node_base;
    const double *mass = A.mass + P.node_base;

    double w[NPT][3];
    int dg[NPT];
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
        const int r = s * BLOCK + tid;
        w[s][0] = w[s][1] = w[s][2] = 0.0;
        dg[s] = 0;
        if (r < N) {
            double x[3];
            start_position(A, S, r, x);
            pos.store(r, x[0], x[1], x[2]);
            dg[s] = A.deg[P.node_base + r];
        }
    }
    __syncthreads();
    // Initial internal force and acceleration (v = 0), then the first
    // partial velocity update of the loop: w = 0 + dt/2 a.
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
        const int r = s * BLOCK + tid;
        // the wave's slice exists only if its first node does
        if (s * BLOCK + wave * kWave < Nf) {
            const Row row = node_row(A, P, r);
            if (r < Nf) {
                double xi, yi, zi, gx, gy, gz;
                pos.load(r, xi, yi, zi);
                gather_force(A, row, pos, lane, dg[s], xi, yi, zi, gx, gy, gz);
                const double im = invm[r];
                w[s][0] = hdt * (gx * im);
                w[s][1] = hdt * (gy * im);
                w[s][2] = hdt * (gz * im);
            }
        }
    }
    __syncthreads();

    int64_t n = 0;
    double rho = 0.0, ke = 0.0;
    int status = kMaxIter;
    for (;;) {
        // displacement update (free dof)
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + tid;
            if (r < Nf) {
                double x, y, z;
                pos.load(r, x, y, z);
                x += dt * w[s][0];
                y += dt * w[s][1];
                z += dt * w[s][2];
                pos.store(r, x, y, z);
            }
        }
        __syncthreads();
        double gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + tid;
            if (s * BLOCK + wave * kWave < N) {
                const Row row = node_row(A, P, r);
                if (r < N) {
                    double xi, yi, zi, g[3];
                    pos.load(r, xi, yi, zi);
                    gather_force(A, row, pos, lane, dg[s], xi, yi, zi, g[0], g[1], g[2]);
                    const double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
                    if (r < Nf) {
                        const double im = invm[r];
                        double vv = 0.0;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            // damping force, acceleration, partial velocity updates
                            const double acc = g[a] * im - cdamp * w[s][a];
                            const double v = w[s][a] + hdt * acc;
                            vv += v * v;
                            w[s][a] = v + hdt * acc;
                        }
                        gf2 += gg;
                        ke2 += mass[r] * vv;
                    } else {
                        gb2 += gg;
                    }
                }
            }
        }
        block_sum3<NW>(red, lane, wave, gf2, gb2, ke2);
        ++n;
        if (stop_test(A, P, gf2, gb2, ke2, n, rho, ke, status)) break;
    }

    // Displacements of the final iterate (the stress kernel reads them).
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
        const int r = s * BLOCK + tid;
        if (r < N) {
            double x[3];
            pos.load(r, x[0], x[1], x[2]);
            write_u(A, S, r, x);
        }
    }
    finish_solve(A, S, tid, n, rho, ke, status);
}

// ---------------------------------------------------------------------------
// Global-placement variant: positions and half-step velocities in device
// memory (L2-resident for one problem), any problem size.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_dr_glb(SolveArgs A)
{
    extern __shared__ double smem[];
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const Solve S = load_solve(A);
    const ProbDesc &P = S.P;
    const int N = P.N, Nf = P.N_free;
    double *red = smem;
    const GlbPos pos{A.xg + 4 * P.node_base};
    double *W = A.wg + 4 * P.node_base;
    const double dt = P.dt, hdt = 0.5 * P.dt, cdamp = P.c;

    for (int r = tid; r < N; r += BLOCK) {
        double x[3];
        start_position(A, S, r, x);
        pos.store(r, x[0], x[1], x[2]);
    }
    __syncthreads();
    for (int r = tid; r < Nf; r += BLOCK) {
        double xi, yi, zi, gx, gy, gz;
        pos.load(r, xi, yi, zi);
        const double imr = A.invm[P.node_base + r];
        gather_force(A, node_row(A, P, r), pos, lane, A.deg[P.node_base + r], xi, yi, zi, gx, gy,
                     gz);
        W[4 * r + 0] = hdt * (gx * imr);
        W[4 * r + 1] = hdt * (gy * imr);
        W[4 * r + 2] = hdt * (gz * imr);
    }
    __syncthreads();

    int64_t n = 0;
    double rho = 0.0, ke = 0.0;
    int status = kMaxIter;
    for (;;) {
        for (int r = tid; r < Nf; r += BLOCK) {
            double x, y, z;
            pos.load(r, x, y, z);
            x += dt * W[4 * r + 0];
            y += dt * W[4 * r + 1];
            z += dt * W[4 * r + 2];
            pos.store(r, x, y, z);
        }
        __syncthreads();
        double gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
        for (int r = tid; r < N; r += BLOCK) {
            double xi, yi, zi, g[3];
            pos.load(r, xi, yi, zi);
            gather_force(A, node_row(A, P, r), pos, lane, A.deg[P.node_base + r], xi, yi, zi,
                         g[0], g[1], g[2]);
            const double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
            if (r < Nf) {
                const double imr = A.invm[P.node_base + r];
                double vv = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double wa = W[4 * r + a];
                    const double acc = g[a] * imr - cdamp * wa;
                    const double v = wa + hdt * acc;
                    vv += v * v;
                    W[4 * r + a] = v + hdt * acc;
                }
                gf2 += gg;
                ke2 += A.mass[P.node_base + r] * vv;
            } else {
                gb2 += gg;
            }
        }
        block_sum3<NW>(red, lane, wave, gf2, gb2, ke2);
        ++n;
        if (stop_test(A, P, gf2, gb2, ke2, n, rho, ke, status)) break;
    }

    for (int r = tid; r < N; r += BLOCK) {
        double x[3];
        pos.load(r, x[0], x[1], x[2]);
        write_u(A, S, r, x);
    }
    finish_solve(A, S, tid, n, rho, ke, status);
}

// ---------------------------------------------------------------------------
// Per-problem launch loop (the paper's naive design): the same pass split
// into kernels over nodes, with the residual read back by the host.
// ---------------------------------------------------------------------------
constexpr int kLoopBlock = 256;

// phase 0: start positions; phase 1: initial acceleration -> w.
__global__ void __launch_bounds__(kLoopBlock) k_loop_setup(SolveArgs A, int slot, int phase)
{
    Solve S;
    S.slot = slot;
    S.p = A.ids ? A.ids[slot] : slot;
    S.P = A.probs[S.p];
    for (int k = 0; k < 9; ++k) S.F[k] = A.F[9 * (int64_t)slot + k];
    S.warm = (A.start == kStartWarm) && A.has_state[S.p];
    for (int k = 0; k < 9; ++k) S.Fl[k] = S.warm ? A.F_last[9 * (int64_t)S.p + k] : S.F[k];
    const ProbDesc &P = S.P;
    const GlbPos pos{A.xg + 4 * P.node_base};
    double *W = A.wg + 4 * P.node_base;
    const int r = blockIdx.x * kLoopBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    if (phase == 0) {
        if (r < P.N) {
            double x[3];
            start_position(A, S, r, x);
            pos.store(r, x[0], x[1], x[2]);
        }
    } else {
        const int wbase = blockIdx.x * kLoopBlock + (threadIdx.x / kWave) * kWave;
        if (wbase >= P.N) return;
        const Row row = node_row(A, P, wbase);
        if (r < P.N_free) {
            double xi, yi, zi, gx, gy, gz;
            pos.load(r, xi, yi, zi);
            const double imr = A.invm[P.node_base + r];
            gather_force(A, row, pos, lane, A.deg[P.node_base + r], xi, yi, zi, gx, gy, gz);
            const double hdt = 0.5 * P.dt;
            W[4 * r + 0] = hdt * (gx * imr);
            W[4 * r + 1] = hdt * (gy * imr);
            W[4 * r + 2] = hdt * (gz * imr);
        }
    }
}

__global__ void __launch_bounds__(kLoopBlock) k_loop_update(SolveArgs A, int slot)
{
    const int p = A.ids ? A.ids[slot] : slot;
    const ProbDesc P = A.probs[p];
    const GlbPos pos{A.xg + 4 * P.node_base};
    const double *W = A.wg + 4 * P.node_base;
    const int r = blockIdx.x * kLoopBlock + threadIdx.x;
    if (r < P.N_free) {
        double x, y, z;
        pos.load(r, x, y, z);
        x += P.dt * W[4 * r + 0];
        y += P.dt * W[4 * r + 1];
        z += P.dt * W[4 * r + 2];
        pos.store(r, x, y, z);
    }
}

// Force gather + damped velocity update; per-block partial sums.
__global__ void __launch_bounds__(kLoopBlock) k_loop_force(SolveArgs A, int slot, double *partial)
{
    __shared__ double red[(kLoopBlock / kWave) * kRedStride];
    const int p = A.ids ? A.ids[slot] : slot;
    const ProbDesc P = A.probs[p];
    const GlbPos pos{A.xg + 4 * P.node_base};
    double *W = A.wg + 4 * P.node_base;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int r = blockIdx.x * kLoopBlock + tid;
    const double hdt = 0.5 * P.dt;
    double gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
    const int wbase = blockIdx.x * kLoopBlock + wave * kWave;
    Row row;
    row.e0 = 0; row.width = 0;
    if (wbase < P.N) row = node_row(A, P, wbase);
    if (r < P.N) {
        double xi, yi, zi, g[3];
        pos.load(r, xi, yi, zi);
        gather_force(A, row, pos, lane, A.deg[P.node_base + r], xi, yi, zi, g[0], g[1], g[2]);
        const double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (r < P.N_free) {
            const double imr = A.invm[P.node_base + r];
            double vv = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double wa = W[4 * r + a];
                const double acc = g[a] * imr - P.c * wa;
                const double v = wa + hdt * acc;
                vv += v * v;
                W[4 * r + a] = v + hdt * acc;
            }
            gf2 = gg;
            ke2 = A.mass[P.node_base + r] * vv;
        } else {
            gb2 = gg;
        }
    }
    block_sum3<kLoopBlock / kWave>(red, lane, wave, gf2, gb2, ke2);
    if (tid == 0) {
        partial[3 * blockIdx.x + 0] = gf2;
        partial[3 * blockIdx.x + 1] = gb2;
        partial[3 * blockIdx.x + 2] = ke2;
    }
}

// Sums the block partials in order; out = {gf2, gb2, ke2}.
__global__ void __launch_bounds__(kWave) k_loop_reduce(const double *partial, int nblk, double *out)
{
    const int lane = threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = lane; i < nblk; i += kWave) {
        a += partial[3 * i]; b += partial[3 * i + 1]; c += partial[3 * i + 2];
    }
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c);
    if (lane == 0) { out[0] = a; out[1] = b; out[2] = c; }
}

// End of a solve in the loop design: displacements and scalars of the slot.
__global__ void __launch_bounds__(kLoopBlock) k_loop_finish(SolveArgs A, int slot, int64_t n,
                                                            double rho, double ke, int status)
{
    Solve S;
    S.slot = slot;
    S.p = A.ids ? A.ids[slot] : slot;
    S.P = A.probs[S.p];
    for (int k = 0; k < 9; ++k) S.F[k] = A.F[9 * (int64_t)slot + k];
    for (int k = 0; k < 9; ++k) S.Fl[k] = S.F[k];
    S.warm = false;
    const GlbPos pos{A.xg + 4 * S.P.node_base};
    const int r = blockIdx.x * kLoopBlock + threadIdx.x;
    if (r < S.P.N) {
        double x[3];
        pos.load(r, x[0], x[1], x[2]);
        write_u(A, S, r, x);
    }
    if (blockIdx.x == 0) finish_solve(A, S, threadIdx.x, n, rho, ke, status);
}

// ---------------------------------------------------------------------------
// Stress average (section I: the sub-problem returns the volume-averaged
// stress to the macroscale), one workgroup per solve slot, FP64, from the
// final displacements:
//   sigma     = 1/J sum over prescribed nodes of (-g_b) (x) (x_b - F c0)
//   sigma_fib = 1/J sum over fibers of T d (x) d / l
// ---------------------------------------------------------------------------
struct UPos {
    const double *X, *u; // renumbered, 3 per node, offset to the problem
    __device__ __forceinline__ void load(int j, double &x, double &y, double &z) const
    {
        x = X[3 * (int64_t)j] + u[3 * (int64_t)j];
        y = X[3 * (int64_t)j + 1] + u[3 * (int64_t)j + 1];
        z = X[3 * (int64_t)j + 2] + u[3 * (int64_t)j + 2];
    }
};

constexpr int kStressBlock = 256;

__global__ void __launch_bounds__(kStressBlock) k_stress(SolveArgs A, int slot0)
{
    __shared__ double red[(kStressBlock / kWave) * kRedStride];
    constexpr int NW = kStressBlock / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int slot = slot0 + (int)blockIdx.x;
    const int p = A.ids ? A.ids[slot] : slot;
    const ProbDesc P = A.probs[p];
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F[9 * (int64_t)slot + k];
    const UPos pos{A.X + 3 * P.node_base, A.u + 3 * P.node_base};
    double fc0[3];
    fc0_of(F, fc0);
    double sb[9], sf[9];
    for (int k = 0; k < 9; ++k) { sb[k] = 0.0; sf[k] = 0.0; }
    for (int r = tid; r < P.N; r += kStressBlock) {
        double x[3], g[3];
        pos.load(r, x[0], x[1], x[2]);
        gather_force_stress(A, node_row(A, P, r), pos, lane, A.deg[P.node_base + r], x[0], x[1],
                            x[2], g[0], g[1], g[2], sf);
        if (r >= P.N_free) {
            const double y[3] = {x[0] - fc0[0], x[1] - fc0[1], x[2] - fc0[2]};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) sb[3 * a + b] -= g[a] * y[b];
        }
    }
    for (int k = 0; k < 9; ++k) { sb[k] = wave_sum(sb[k]); sf[k] = wave_sum(sf[k]); }
    if (lane == 0) {
        for (int k = 0; k < 9; ++k) {
            red[wave * kRedStride + k] = sb[k];
            red[wave * kRedStride + 9 + k] = sf[k];
        }
    }
    __syncthreads();
    if (tid < 18) {
        const double J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                         F[2] * (F[3] * F[7] - F[4] * F[6]);
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += red[w * kRedStride + tid];
        if (tid < 9) A.sigma[9 * (int64_t)slot + tid] = t / J;
        else A.sigma_fib[9 * (int64_t)slot + tid - 9] = t / J;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <class K>
static int launch(K kernel, int grid, int block, int lds, hipStream_t st, const SolveArgs &a)
{
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, st, a);
    return (int)hipGetLastError();
}

#define DR_REG_CASE(B, NP)                                                                       \
    case NP:                                                                                     \
        return launch(k_dr_reg<B, NP>, a.n_solve, B, plan.lds_bytes, st, a);

template <int B>
static int launch_reg(const SolveArgs &a, const LaunchPlan &plan, hipStream_t st)
{
    switch (plan.npt) {
        DR_REG_CASE(B, 1)
        DR_REG_CASE(B, 2)
        DR_REG_CASE(B, 3)
        DR_REG_CASE(B, 4)
        DR_REG_CASE(B, 5)
        DR_REG_CASE(B, 6)
        DR_REG_CASE(B, 7)
        DR_REG_CASE(B, 8)
    default:
        return -1000;
    }
}

static int launch_dr(const SolveArgs &a, const LaunchPlan &plan, hipStream_t st)
{
    if (plan.npt > 0) {
        switch (plan.block) {
        case 256: return launch_reg<256>(a, plan, st);
        case 512: return launch_reg<512>(a, plan, st);
        case 1024: return launch_reg<1024>(a, plan, st);
        default: return -1001;
        }
    }
    switch (plan.block) {
    case 256: return launch(k_dr_glb<256>, a.n_solve, 256, plan.lds_bytes, st, a);
    case 512: return launch(k_dr_glb<512>, a.n_solve, 512, plan.lds_bytes, st, a);
    case 1024: return launch(k_dr_glb<1024>, a.n_solve, 1024, plan.lds_bytes, st, a);
    default: return -1001;
    }
}

// The batched solve: one persistent DR launch, then the stress launch.
int launch_solve(const SolveArgs &a, const LaunchPlan &plan, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (a.n_solve <= 0) return 0;
    const int rc = launch_dr(a, plan, st);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_stress, dim3(a.n_solve), dim3(kStressBlock), 0, st, a, 0);
    return (int)hipGetLastError();
}

// One step of the launch-loop design for solve slot `slot`:
//   phase 0: set-up (start positions, initial acceleration)
//   phase 1: one DR pass (update, force, reduce -> out_scalars[0..2])
//   phase 2: displacements, scalars and stress; out_scalars[3..5] is a HOST
//            array {rho, ke, status} passed by value to the kernels
int launch_loop_iteration_kernels(const SolveArgs &a, int slot, int phase, int n_nodes,
                                  double *partial, double *out_scalars, int64_t n_done,
                                  void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nblk = (n_nodes + kLoopBlock - 1) / kLoopBlock;
    if (phase == 0) {
        hipLaunchKernelGGL(k_loop_setup, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, 0);
        hipLaunchKernelGGL(k_loop_setup, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, 1);
    } else if (phase == 1) {
        hipLaunchKernelGGL(k_loop_update, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot);
        hipLaunchKernelGGL(k_loop_force, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, partial);
        hipLaunchKernelGGL(k_loop_reduce, dim3(1), dim3(kWave), 0, st, partial, nblk, out_scalars);
    } else {
        hipLaunchKernelGGL(k_loop_finish, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, n_done,
                           out_scalars[3], out_scalars[4], (int)out_scalars[5]);
        hipLaunchKernelGGL(k_stress, dim3(1), dim3(kStressBlock), 0, st, a, slot);
    }
    return (int)hipGetLastError();
}

const char *kernel_error_string(int code)
{
    if (code == -1000) return "no kernel instantiated for this nodes-per-thread count";
    if (code == -1001) return "unsupported workgroup size";
    return hipGetErrorString((hipError_t)code);
}

} // namespace drk
