// HIP kernels of libdr that are not templates (stress average, the
// launch-loop comparator, fills) and the launch dispatch.  The persistent
// DR kernels are instantiated in dr_k_reg_*.hip and dr_k_glb_*.hip.
#include <mutex>

#include "dr_device.h"

namespace drk {

// ---------------------------------------------------------------------------
// Stress average (section I: the sub-problem returns the volume-averaged
// stress to the macroscale), one workgroup per slot whose solve has finished,
// FP64, from the final displacements:
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

// Both stress forms of problem p (one workgroup of kStressBlock threads).
__device__ void stress_of(const SolveArgs &A, int p)
{
    __shared__ double red[(kStressBlock / kWave) * kRedStride];
    constexpr int NW = kStressBlock / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id(tid);
    const int st = A.status[p];
    // nothing to do while a solve runs, before any solve, or after an abort
    if (st == kStatusRunning || st == kStatusIdle || st == kStatusAborted) return; // uniform
    const ProbDesc P = A.probs[p];
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = A.F_cur[9 * (int64_t)p + k];
    const UPos pos{A.X + 3 * P.node_base, A.u + 3 * P.node_base};
    double fc0[3];
    for (int a = 0; a < 3; ++a) fc0[a] = 0.5 * (F[3 * a] + F[3 * a + 1] + F[3 * a + 2]);
    double sb[9], sf[9];
    for (int k = 0; k < 9; ++k) { sb[k] = 0.0; sf[k] = 0.0; }
    for (int r = tid; r < P.N; r += kStressBlock) {
        double x[3], g[3];
        pos.load(r, x[0], x[1], x[2]);
        gather_stress(A, node_row(A, P, r), pos, lane, A.deg[P.node_base + r], x[0], x[1], x[2],
                      g[0], g[1], g[2], sf);
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
        if (tid < 9) A.sigma[9 * (int64_t)p + tid] = t / J;
        else A.sigma_fib[9 * (int64_t)p + tid - 9] = t / J;
    }
}

// One workgroup per slot (slots slot0 + blockIdx of the launch order).
__global__ void __launch_bounds__(kStressBlock) k_stress(SolveArgs A, int slot0)
{
    const int slot = A.order ? A.order[slot0 + (int)blockIdx.x] : slot0 + (int)blockIdx.x;
    stress_of(A, A.ids ? A.ids[slot] : slot);
}

// One workgroup per entry of the tail list (the problems a group launch finished).
__global__ void __launch_bounds__(kStressBlock) k_stress_tail(SolveArgs A)
{
    if ((int)blockIdx.x >= *A.tail_count) return;
    stress_of(A, A.tail_list[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// Per-problem launch loop (the paper's naive design): the same pass split
// into kernels over nodes, with the residual read back by the host.  FP64;
// the running state uses the records of the persistent kernels (buffer 0 of
// qbuf, wbuf) at the problem's state offset, so a loop solve never touches
// another problem's saved state.
// ---------------------------------------------------------------------------
constexpr int kLoopBlock = 256;
constexpr int kQS = kQStride<double>, kWS = kWStride<double>;

// The problem's state records (buffer 0) and half-step velocity records.
__device__ __forceinline__ GlbQ<double> loop_pos(const SolveArgs &A, int p)
{
    return GlbQ<double>{A.qbuf + kQS * A.state_off[p]};
}
__device__ __forceinline__ double *loop_w(const SolveArgs &A, int p)
{
    return A.wbuf + kWS * A.state_off[p];
}

// phase 0: start positions; phase 1: initial acceleration -> w.
__global__ void __launch_bounds__(kLoopBlock) k_loop_setup(SolveArgs A, int slot, int phase)
{
    const Slot S = load_slot(A, slot);
    const ProbDesc &P = S.P;
    const GlbQ<double> pos = loop_pos(A, S.p);
    double *W = loop_w(A, S.p);
    const int r = blockIdx.x * kLoopBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    if (phase == 0) {
        if (r < P.N) {
            double q[3];
            start_q<P64>(A, S, r, q);
            pos.store(r, q[0], q[1], q[2]);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) begin_solve(A, S);
    } else {
        const int wbase = blockIdx.x * kLoopBlock + (threadIdx.x / kWave) * kWave;
        if (wbase >= P.N) return;
        const Row row = node_row(A, P, wbase);
        if (r < P.N_free) {
            double qi[3], g[3];
            pos.load(r, qi[0], qi[1], qi[2]);
            gather<P64, 4>(A, Aff32{}, row, pos, lane, A.deg[P.node_base + r], qi[0], qi[1], qi[2], g[0],
                           g[1], g[2]);
            const double im = A.invm[P.node_base + r];
            const double hdt = 0.5 * P.dt;
            for (int a = 0; a < 3; ++a) node_rec<kWS>(W, r)[a] = hdt * (g[a] * im);
        }
    }
}

__global__ void __launch_bounds__(kLoopBlock) k_loop_update(SolveArgs A, int slot)
{
    const int p = A.ids ? A.ids[slot] : slot;
    const ProbDesc P = A.probs[p];
    const GlbQ<double> pos = loop_pos(A, p);
    double *W = loop_w(A, p);
    const int r = blockIdx.x * kLoopBlock + threadIdx.x;
    if (r < P.N_free) {
        double x, y, z;
        pos.load(r, x, y, z);
        x = fma(P.dt, node_rec<kWS>(W, r)[0], x);
        y = fma(P.dt, node_rec<kWS>(W, r)[1], y);
        z = fma(P.dt, node_rec<kWS>(W, r)[2], z);
        pos.store(r, x, y, z);
    }
}

// Force gather + damped velocity update; per-block partial sums.
__global__ void __launch_bounds__(kLoopBlock) k_loop_force(SolveArgs A, int slot, double *partial)
{
    __shared__ double red[(kLoopBlock / kWave) * kRedStride];
    const int p = A.ids ? A.ids[slot] : slot;
    const ProbDesc P = A.probs[p];
    const GlbQ<double> pos = loop_pos(A, p);
    double *W = loop_w(A, p);
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id(tid);
    const int r = blockIdx.x * kLoopBlock + tid;
    const double hdt = 0.5 * P.dt;
    double gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
    const int wbase = blockIdx.x * kLoopBlock + wave * kWave;
    Row row;
    row.e0 = 0;
    row.width = 0;
    if (wbase < P.N) row = node_row(A, P, wbase);
    if (r < P.N) {
        double qi[3], g[3];
        pos.load(r, qi[0], qi[1], qi[2]);
        gather<P64, 4>(A, Aff32{}, row, pos, lane, A.deg[P.node_base + r], qi[0], qi[1], qi[2], g[0], g[1],
                       g[2]);
        const double gg = sq3(g[0], g[1], g[2]);
        if (r < P.N_free) {
            const double im = A.invm[P.node_base + r];
            double vv = 0.0;
            for (int a = 0; a < 3; ++a) {
                double wa = node_rec<kWS>(W, r)[a];
                const double v = vel_step(g[a], im, P.c, hdt, wa);
                vv = fma(v, v, vv);
                node_rec<kWS>(W, r)[a] = wa;
            }
            gf2 = gg;
            ke2 = A.mass[P.node_base + r] * vv;
        } else {
            gb2 = gg;
        }
    }
    block_sum2<kLoopBlock / kWave>(red, lane, wave, gf2, gb2);
    ke2 = block_sum1<kLoopBlock / kWave>(red, lane, wave, ke2);
    if (tid == 0) {
        partial[3 * blockIdx.x + 0] = gf2;
        partial[3 * blockIdx.x + 1] = gb2;
        partial[3 * blockIdx.x + 2] = ke2;
    }
}

// The paper's force kernel (section III) for the launch-loop comparator:
// forces zeroed, then every fiber evaluated once, from the incidences of its
// lower-numbered end, and added to both ends with FP64 atomics.  The
// summation order depends on the timing of the atomics, so results vary at
// round-off from run to run.
__global__ void __launch_bounds__(kLoopBlock) k_loop_zero(SolveArgs A, int slot, double *g)
{
    const int p = A.ids ? A.ids[slot] : slot;
    const int r = blockIdx.x * kLoopBlock + threadIdx.x;
    if (r < A.probs[p].N) {
        g[3 * r + 0] = 0.0;
        g[3 * r + 1] = 0.0;
        g[3 * r + 2] = 0.0;
    }
}

__global__ void __launch_bounds__(kLoopBlock) k_loop_scatter(SolveArgs A, int slot, double *g)
{
    const int p = A.ids ? A.ids[slot] : slot;
    const ProbDesc P = A.probs[p];
    const GlbQ<double> pos = loop_pos(A, p);
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id(tid);
    const int r = blockIdx.x * kLoopBlock + tid;
    const int wbase = blockIdx.x * kLoopBlock + wave * kWave;
    if (wbase >= P.N) return;
    const Row row = node_row(A, P, wbase);
    if (r >= P.N) return;
    double xi, yi, zi;
    pos.load(r, xi, yi, zi);
    const int d = A.deg[P.node_base + r];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int k = 0; k < d; ++k) {
        const int64_t e = row.e0 + (int64_t)k * kWave + lane;
        const int j = A.nbr[e];
        if (j < r) continue; // the other end evaluates this fiber
        const KL c = A.kl[e];
        double dx, dy, dz;
        pos.load(j, dx, dy, dz);
        dx -= xi; dy -= yi; dz -= zi;
        const double l2 = len2(dx, dy, dz);
        const double s = c.k * (l2 - c.L2) * rsq64(l2);
        axpy3(s, dx, dy, dz, gx, gy, gz);
        unsafeAtomicAdd(g + 3 * j + 0, -s * dx);
        unsafeAtomicAdd(g + 3 * j + 1, -s * dy);
        unsafeAtomicAdd(g + 3 * j + 2, -s * dz);
    }
    unsafeAtomicAdd(g + 3 * r + 0, gx);
    unsafeAtomicAdd(g + 3 * r + 1, gy);
    unsafeAtomicAdd(g + 3 * r + 2, gz);
}

// Damped velocity update and partial norms from the scattered forces.
__global__ void __launch_bounds__(kLoopBlock) k_loop_accel(SolveArgs A, int slot, const double *g,
                                                           double *partial)
{
    __shared__ double red[(kLoopBlock / kWave) * kRedStride];
    const int p = A.ids ? A.ids[slot] : slot;
    const ProbDesc P = A.probs[p];
    double *W = loop_w(A, p);
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id(tid);
    const int r = blockIdx.x * kLoopBlock + tid;
    const double hdt = 0.5 * P.dt;
    double gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
    if (r < P.N) {
        const double gr[3] = {g[3 * r], g[3 * r + 1], g[3 * r + 2]};
        const double gg = sq3(gr[0], gr[1], gr[2]);
        if (r < P.N_free) {
            const double im = A.invm[P.node_base + r];
            double vv = 0.0;
            for (int a = 0; a < 3; ++a) {
                double wa = node_rec<kWS>(W, r)[a];
                const double v = vel_step(gr[a], im, P.c, hdt, wa);
                vv = fma(v, v, vv);
                node_rec<kWS>(W, r)[a] = wa;
            }
            gf2 = gg;
            ke2 = A.mass[P.node_base + r] * vv;
        } else {
            gb2 = gg;
        }
    }
    block_sum2<kLoopBlock / kWave>(red, lane, wave, gf2, gb2);
    ke2 = block_sum1<kLoopBlock / kWave>(red, lane, wave, ke2);
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
    Slot S = load_slot(A, slot);
    for (int k = 0; k < 9; ++k) S.F[k] = A.F_cur[9 * (int64_t)S.p + k];
    const GlbQ<double> pos = loop_pos(A, S.p);
    const int r = blockIdx.x * kLoopBlock + threadIdx.x;
    if (r < S.P.N) {
        double q[3];
        pos.load(r, q[0], q[1], q[2]);
        write_u<P64>(A, S, r, q);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) record(A, S, n, rho, ke, status, Progress{rho * rho, n});
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
// One DR launch of a class: the register/LDS variant or the global one.
static int launch_dr(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    if (pl.npt > 0) {
        switch (pl.block) {
        case 256: return pl.fp32 ? launch_reg_p32_256(a, pl, st) : launch_reg_p64_256(a, pl, st);
        case 512: return pl.fp32 ? launch_reg_p32_512(a, pl, st) : launch_reg_p64_512(a, pl, st);
        case 1024: return pl.fp32 ? launch_reg_p32_1024(a, pl, st) : launch_reg_p64_1024(a, pl, st);
        default: return -1001;
        }
    }
    return pl.fp32 ? launch_glb_p32(a, pl, st) : launch_glb_p64(a, pl, st);
}

// One batched launch: the persistent DR kernel, then the stress kernel (which
// skips the slots whose solve is still running).
int launch_solve(const SolveArgs &a, const LaunchPlan &plan, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (a.n_solve <= 0) return 0;
    const int rc = a.dt_rule ? launch_dtp(a, plan.block, stream) : launch_dr(a, plan, st);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_stress, dim3(a.n_solve), dim3(kStressBlock), 0, st, a, 0);
    return (int)hipGetLastError();
}

// One step of the launch-loop design for solve slot `slot`:
//   phase 0: set-up (start positions, initial acceleration)
//   phase 1: one DR pass (update, force, reduce -> out_scalars[0..2])
//   phase 2: displacements, scalars and stress of the finished solve
int launch_loop_kernels(const SolveArgs &a, int slot, int phase, int n_nodes, double *partial,
                        double *out_scalars, int64_t n_done, double rho, double ke, int status,
                        double *gbuf, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nblk = (n_nodes + kLoopBlock - 1) / kLoopBlock;
    if (phase == 3) {
        // one pass with the zero + atomic-scatter force kernel
        hipLaunchKernelGGL(k_loop_update, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot);
        hipLaunchKernelGGL(k_loop_zero, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, gbuf);
        hipLaunchKernelGGL(k_loop_scatter, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, gbuf);
        hipLaunchKernelGGL(k_loop_accel, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, gbuf, partial);
        hipLaunchKernelGGL(k_loop_reduce, dim3(1), dim3(kWave), 0, st, partial, nblk, out_scalars);
    } else if (phase == 0) {
        hipLaunchKernelGGL(k_loop_setup, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, 0);
        hipLaunchKernelGGL(k_loop_setup, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, 1);
    } else if (phase == 1) {
        hipLaunchKernelGGL(k_loop_update, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot);
        hipLaunchKernelGGL(k_loop_force, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, partial);
        hipLaunchKernelGGL(k_loop_reduce, dim3(1), dim3(kWave), 0, st, partial, nblk, out_scalars);
    } else {
        hipLaunchKernelGGL(k_loop_finish, dim3(nblk), dim3(kLoopBlock), 0, st, a, slot, n_done,
                           rho, ke, status);
        hipLaunchKernelGGL(k_stress, dim3(1), dim3(kStressBlock), 0, st, a, slot);
    }
    return (int)hipGetLastError();
}

int group_grid_capacity(int fp32, int block, int lds_bytes, int *capacity)
{
    int per_cu = 0, dev = 0, cus = 0;
    int rc = fp32 ? group_capacity_p32(block, lds_bytes, &per_cu) : group_capacity_p64(block, lds_bytes, &per_cu);
    if (rc != 0) return rc;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    *capacity = per_cu * cus;
    return 0;
}

int launch_tail(const SolveArgs &a, const LaunchPlan &plan, int n_groups, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n_groups <= 0) return 0;
    const int slots = 8 * ((n_groups + 7) / 8);
    // fresh barrier counters and abort flags for the groups of this launch
    int rc = launch_fill_i32(reinterpret_cast<int32_t *>(a.gbar), 0, slots, stream);
    if (rc == 0) rc = launch_fill_i32(a.gabort, 0, slots, stream);
    if (rc != 0) return rc;
    const int grid = group_grid(n_groups, a.group);
    rc = plan.fp32 ? launch_group_p32(a, plan, grid, st) : launch_group_p64(a, plan, grid, st);
    if (rc != 0) return rc;
    hipLaunchKernelGGL(k_stress_tail, dim3(n_groups), dim3(kStressBlock), 0, st, a);
    return (int)hipGetLastError();
}

int launch_fill_i32(int32_t *p, int32_t value, int64_t n, void *stream)
{
    if (n <= 0) return 0;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, n);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free launch loop: one array per device, held by
// the library until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current, and is kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];
} // namespace

int noalloc_scratch(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        g_scratch_addr[dev] = p;
    }
    *ptr = g_scratch_addr[dev];
    return 0;
}

const char *kernel_error_string(int code)
{
    if (code == -1000) return "no kernel instantiated for this nodes-per-thread count";
    if (code == -1001) return "unsupported workgroup size";
    if (code == -1002) return "no global-placement kernel for this chunk at 256 threads";
    if (code == -1003) return "a group launch of the per-pass step takes at most 256 problems per call";
    return hipGetErrorString((hipError_t)code);
}

} // namespace drk

