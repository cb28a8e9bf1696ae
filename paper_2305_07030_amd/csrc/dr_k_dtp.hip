// Dynamic relaxation with a per-pass time step (Fig. 1, "compute next time
// step", read literally): global placement, FP64, one workgroup per problem.
//
// The step of each pass comes from the current state: dt_n = min(dt_{n-1},
// s 2 / w), w^2 = max over free nodes i of (2 / m_i) sum_{f at i} EA_f l_f /
// L_f^2 (the fibers' axial tangent stiffness at their current length, a
// Gershgorin bound on M^-1 K), starting from the constant step dt0 the batch
// derives from the reference state.  The step never grows back (a step that
// follows the stiffness up and down pumps energy into a violent transient).
// Both half velocity updates of a pass use its step,
// so the pass's second update cannot be fused with the next pass's first
// one before the next step is known: the force phase stores the mid-pass
// velocity and the acceleration, the block reduction forms the next step
// with the residual norms, and a sweep then makes the next pass's first
// velocity update and its displacement update.  Where the step stays dt0
// every operation, and its order, is that of the constant-step kernels, so
// the results are the same bits.
//
// Records (at the problem's state offset): positions in two buffers (the
// state after pass k in buffer k & 1, as in the other kernels), the
// velocity record (the half-step velocity between passes; the mid-pass
// velocity inside a pass) and the acceleration record.  A solve stopped by
// the pass budget saves the next pass's step, so a resume continues with the
// same bits.
//
// Group form (GRP): G workgroups per problem from the start of the launch,
// one group per solve slot, as a cooperative launch.  The members act as one
// virtual workgroup of G * BLOCK threads (node -> row -> wave as in the
// group form of the global kernel, so every node's arithmetic is unchanged)
// and meet at the group barrier twice per pass: after the reduction (the
// norms summed over the members in member order, the stiffness bound as
// their max, which is exact, so the steps and states are the same bits as
// one workgroup's) and after the sweep.
#include "dr_device.h"

namespace drk {

// max over the lanes of a row of 16 / of a wave (exact: max needs no order).
template <int CTRL> __device__ __forceinline__ double dpp_max(double v)
{
    return fmax(v, dpp_f64<CTRL>(v));
}

__device__ __forceinline__ double row_max(double v)
{
    v = dpp_max<0xB1>(v);  // quad_perm [1,0,3,2]
    v = dpp_max<0x4E>(v);  // quad_perm [2,3,0,1]
    v = dpp_max<0x124>(v); // row_ror:4
    v = dpp_max<0x128>(v); // row_ror:8
    return v;
}

__device__ __forceinline__ double max_xor(double v, bool half)
{
    const unsigned lo = __double2loint(v), hi = __double2hiint(v);
    const auto l = half ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                        : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = half ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                        : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return fmax(__hiloint2double(h[0], l[0]), __hiloint2double(h[1], l[1]));
}

__device__ __forceinline__ double wave_max(double v)
{
    v = row_max(v);
    v = max_xor(v, false);
    v = max_xor(v, true);
    return v;
}

// Force on a node (the gather of the other kernels: the same operations in
// the same incidence order) and the sum of its fibers' axial tangent
// stiffness EA l / L^2 = 2 k l, k = EA / (2 L^2).  Padding entries have k = 0
// and are masked as in the force.
template <int C, class Pos>
__device__ __forceinline__ void chunk64_k(const SolveArgs &A, int64_t e, const Pos &pos, int k0, int d,
                                          double xi, double yi, double zi, double &gx, double &gy,
                                          double &gz, double &ks)
{
    int j[C];
    KL c[C];
#pragma unroll
    for (int t = 0; t < C; ++t) {
        j[t] = A.nbr[e + (int64_t)t * kWave];
        c[t] = A.kl[e + (int64_t)t * kWave];
    }
    double dx[C], dy[C], dz[C];
#pragma unroll
    for (int t = 0; t < C; ++t) {
        pos.load(j[t], dx[t], dy[t], dz[t]);
        dx[t] -= xi; dy[t] -= yi; dz[t] -= zi;
    }
#pragma unroll
    for (int t = 0; t < C; ++t) {
        const double l2 = len2(dx[t], dy[t], dz[t]);
        const double rl = rsq64(l2);
        double s = c[t].k * (l2 - c[t].L2) * rl;
        double kt = 2.0 * c[t].k * (l2 * rl);
        const bool live = k0 + t < d;
        s = live ? s : 0.0;
        kt = live ? kt : 0.0;
        axpy3(s, dx[t], dy[t], dz[t], gx, gy, gz);
        ks += kt;
    }
}

template <class Pos>
__device__ __forceinline__ void gather_k(const SolveArgs &A, const Row &row, const Pos &pos, int lane,
                                         int d, double xi, double yi, double zi, double &gx, double &gy,
                                         double &gz, double &ks)
{
    gx = 0.0; gy = 0.0; gz = 0.0; ks = 0.0;
    int64_t e = row.e0 + lane;
    int k0 = 0;
    for (; k0 + 2 <= row.width; k0 += 2, e += 2 * kWave)
        chunk64_k<2>(A, e, pos, k0, d, xi, yi, zi, gx, gy, gz, ks);
    if (k0 < row.width) chunk64_k<1>(A, e, pos, k0, d, xi, yi, zi, gx, gy, gz, ks);
}

// The step after one of dt_prev, from the largest nodal bound
// w2 = max_i 2 ks_i / m_i.
__device__ __forceinline__ double step_of(double dt_prev, double safety, double w2)
{
    if (!(w2 > 0.0)) return dt_prev;
    const double dt = safety * 2.0 / sqrt(w2);
    return dt < dt_prev ? dt : dt_prev;
}

template <int BLOCK, bool GRP = false>
__global__ void __launch_bounds__(BLOCK) k_dr_dtp(SolveArgs A)
{
    constexpr int NW = BLOCK / kWave;
    __shared__ double red[NW * kRedStride];
    __shared__ int gflag;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id(tid);
    GroupCtx gc{nullptr, nullptr, nullptr, 1, 0, 0u};
    int slot = (int)blockIdx.x;
    if constexpr (GRP) {
        // group g = solve slot g; its members are blockIdx values of one
        // residue modulo 8 (one XCD)
        const int b = blockIdx.x, G = A.group;
        const int g = ((b >> 3) / G) * 8 + (b & 7);
        if (g >= A.n_solve) return; // uniform per group
        gc.G = G;
        gc.member = (b >> 3) % G;
        gc.bar = A.gbar + g;
        gc.abort = A.gabort + g;
        gc.part = A.gpart + (int64_t)g * 2 * kGroupMax * 4;
        slot = g;
    }
    const Slot S = load_slot(A, A.order ? A.order[slot] : slot);
    // a resume of a solve that is not running is a no-op (uniform per
    // workgroup and group: no member writes the status before all have met)
    if (S.start == kResume && A.status[S.p] != kStatusRunning) return;
    const ProbDesc &P = S.P;
    const int N = P.N, Nf = P.N_free;
    const int64_t nb = P.node_base;
    double *const qbase = A.qbuf + 3 * S.sb;
    auto qbuf_of = [&](int64_t k) { return qbase + (k & 1) * A.qhalf; };
    double *const W = A.wbuf + 3 * S.sb;
    double *const Acc = A.abuf + 3 * S.sb;
    const double dt0 = P.dt, cdamp = P.c;
    // virtual workgroup: this thread's index, the stride, this wave's first node
    const int VB = gc.G * BLOCK;
    const int vt = gc.member * BLOCK + tid;
    const int vbase = (gc.member * NW + wave) * kWave;
    const bool lead = tid == 0 && gc.member == 0;

    // Barrier of the workgroup, or of the group (false once the group was
    // aborted).
    bool alive = true;
    auto sync = [&]() {
        if constexpr (GRP) alive = group_barrier(gc, &gflag) && alive;
        else __syncthreads();
    };

    // Reduction of two sums and one max over the workgroup, then over the
    // group's members (sums in member order, max exact); every thread gets
    // the same bits.  The caller guarantees a barrier since the last read
    // of the records.
    auto reduce3 = [&](double &a, double &b, double &mx) {
        a = wave_sum(a);
        b = wave_sum(b);
        mx = wave_max(mx);
        if (lane == 0) {
            red[wave * kRedStride + 0] = a;
            red[wave * kRedStride + 1] = b;
            red[wave * kRedStride + 2] = mx;
        }
        __syncthreads();
        double ta = 0.0, tb = 0.0, tm = 0.0;
        if (lane < NW) {
            ta = red[lane * kRedStride + 0];
            tb = red[lane * kRedStride + 1];
            tm = red[lane * kRedStride + 2];
        }
        a = lane0(row_sum(ta));
        b = lane0(row_sum(tb));
        mx = lane0(row_max(tm));
        if constexpr (GRP) {
            double *mine = gc.part + ((gc.nbar & 1u) * kGroupMax + gc.member) * 4;
            if (tid == 0) {
                mine[0] = a;
                mine[1] = b;
                mine[2] = mx;
            }
            sync();
            const double *all = gc.part + ((gc.nbar - 1u) & 1u) * kGroupMax * 4;
            double pa = 0.0, pb = 0.0, pm = 0.0;
            if (lane < gc.G) {
                pa = group_load(all + lane * 4 + 0);
                pb = group_load(all + lane * 4 + 1);
                pm = group_load(all + lane * 4 + 2);
            }
            a = lane0(row_sum(pa));
            b = lane0(row_sum(pb));
            mx = lane0(row_max(pm));
        }
    };

    int64_t n = 0;
    double dt; // the step of the next pass
    if (S.start != kResume) {
        const GlbQ<double> q0{qbase};
        for (int r = vt; r < N; r += VB) {
            double q[3];
            start_q<P64>(A, S, r, q);
            q0.store(r, q[0], q[1], q[2]);
        }
        if (lead) begin_solve(A, S);
        sync();
        // initial force and acceleration (v = 0), the stiffness bound at the
        // start state, then the first half velocity update with its step
        double w2 = 0.0, z0 = 0.0, z1 = 0.0;
        for (int base = vbase; base < Nf; base += VB) {
            const int r = base + lane;
            const Row row = node_row(A, P, base);
            double qi[3] = {0.0, 0.0, 0.0}, g[3], ks;
            if (r < N) q0.load(r, qi[0], qi[1], qi[2]);
            gather_k(A, row, q0, lane, r < N ? A.deg[nb + r] : 0, qi[0], qi[1], qi[2], g[0], g[1], g[2], ks);
            if (r < Nf) {
                const double im = A.invm[nb + r];
#pragma unroll
                for (int a = 0; a < 3; ++a) node_rec<3>(Acc, r)[a] = g[a] * im;
                w2 = fmax(w2, 2.0 * im * ks);
            }
        }
        reduce3(z0, z1, w2);
        dt = step_of(dt0, A.dt_safety, w2);
        const double hdt = 0.5 * dt;
        for (int r = vt; r < Nf; r += VB)
#pragma unroll
            for (int a = 0; a < 3; ++a) node_rec<3>(W, r)[a] = hdt * node_rec<3>(Acc, r)[a];
    } else {
        n = A.iters[S.p];
        dt = A.dt_next[S.p];
    }
    __syncthreads();

    // the first displacement update of this launch, from buffer n & 1 into
    // (n + 1) & 1; prescribed nodes are copied so that both buffers hold them
    {
        const GlbQ<double> src{qbuf_of(n)}, dst{qbuf_of(n + 1)};
        for (int r = vt; r < N; r += VB) {
            double q[3];
            src.load(r, q[0], q[1], q[2]);
            if (r < Nf)
#pragma unroll
                for (int a = 0; a < 3; ++a) q[a] = fma(dt, node_rec<3>(W, r)[a], q[a]);
            dst.store(r, q[0], q[1], q[2]);
        }
    }
    sync();

    const int64_t n0 = n;
    const int64_t budget = launch_budget(A, S.p);
    const double tol2 = A.tol * A.tol;
    double rho = 0.0, ke = 0.0, gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
    int status = kStatusRunning;
    Progress pg{__builtin_huge_val(), n};
    if (S.start == kResume) {
        pg.best = A.rho_best[S.p];
        pg.nbest = A.n_best[S.p];
    }
    while (alive) {
        // pass n + 1 at the state in buffer (n + 1) & 1, with step dt
        const double hdt = 0.5 * dt;
        const GlbQ<double> pos{qbuf_of(n + 1)};
        gf2 = 0.0; gb2 = 0.0; ke2 = 0.0;
        double w2 = 0.0;
        for (int base = vbase; base < N; base += VB) {
            const int r = base + lane;
            const Row row = node_row(A, P, base);
            double qi[3] = {0.0, 0.0, 0.0}, g[3], ks;
            if (r < N) pos.load(r, qi[0], qi[1], qi[2]);
            gather_k(A, row, pos, lane, r < N ? A.deg[nb + r] : 0, qi[0], qi[1], qi[2], g[0], g[1], g[2], ks);
            if (r < N) {
                const double gg = sq3(g[0], g[1], g[2]);
                if (r < Nf) {
                    const double im = A.invm[nb + r], m = A.mass[nb + r];
                    double vv = 0.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        // damping force, acceleration, the pass's second half
                        // velocity update (mid-pass velocity kept)
                        const double w = node_rec<3>(W, r)[a];
                        const double acc = fma(g[a], im, -(cdamp * w));
                        const double v = fma(hdt, acc, w);
                        vv = fma(v, v, vv);
                        node_rec<3>(W, r)[a] = v;
                        node_rec<3>(Acc, r)[a] = acc;
                    }
                    gf2 += gg;
                    ke2 = fma(m, vv, ke2);
                    w2 = fmax(w2, 2.0 * im * ks);
                } else {
                    gb2 += gg;
                }
            }
        }
        reduce3(gf2, gb2, w2);
        if (!alive) break;
        ++n;
        if (stop_test(A, P, tol2, gf2, gb2, n, status, pg)) break;
        // compute next time step, then the next pass's first half velocity
        // update and displacement update (buffer n & 1 into (n + 1) & 1)
        dt = step_of(dt, A.dt_safety, w2);
        const double hn = 0.5 * dt;
        const bool more = n - n0 < budget;
        const GlbQ<double> src{qbuf_of(n)}, dst{qbuf_of(n + 1)};
        for (int r = vt; r < Nf; r += VB) {
            double q[3];
            if (more) src.load(r, q[0], q[1], q[2]);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double w = fma(hn, node_rec<3>(Acc, r)[a], node_rec<3>(W, r)[a]);
                node_rec<3>(W, r)[a] = w;
                if (more) q[a] = fma(dt, w, q[a]);
            }
            if (more) dst.store(r, q[0], q[1], q[2]);
        }
        if (!more) break; // budget spent: the state after pass n stays in buffer n & 1
        sync();
    }
    if (!alive) status = kStatusAborted;
    // kinetic energy of the last pass (reported only), once every wave has
    // read the last reduction's records
    __syncthreads();
    if constexpr (GRP) {
        if (alive) {
            double z0 = 0.0, z1 = 0.0;
            reduce3(ke2, z0, z1);
            if (!alive) status = kStatusAborted;
        }
    } else {
        ke2 = block_sum1<NW>(red, lane, wave, ke2);
    }
    final_scalars(P, gf2, gb2, ke2, rho, ke);
    if (status != kStatusRunning && status != kStatusAborted) {
        // every node's final state was written by its own thread
        const GlbQ<double> fin{qbuf_of(n)};
        for (int r = vt; r < N; r += VB) {
            double q[3];
            fin.load(r, q[0], q[1], q[2]);
            write_u<P64>(A, S, r, q);
        }
    }
    if (lead) {
        record(A, S, n, rho, ke, status, pg);
        if (status == kStatusRunning) A.dt_next[S.p] = dt;
    }
}

int launch_dtp(const SolveArgs &a, int block, void *stream)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (a.group > 1) {
        // one group of a.group workgroups (1024 threads) per solve slot, all
        // resident at once (the runtime refuses a larger cooperative grid)
        if (a.n_solve > kTailMax) return -1003;
        const int slots = 8 * ((a.n_solve + 7) / 8);
        int rc = launch_fill_i32(reinterpret_cast<int32_t *>(a.gbar), 0, slots, stream);
        if (rc == 0) rc = launch_fill_i32(a.gabort, 0, slots, stream);
        if (rc != 0) return rc;
        SolveArgs arg = a;
        void *args[] = {&arg};
        hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_dr_dtp<1024, true>),
                                                  dim3(group_grid(a.n_solve, a.group)), dim3(1024), args, 0, st);
        if (e != hipSuccess) return (int)e;
        return (int)hipGetLastError();
    }
    switch (block) {
    case 256: hipLaunchKernelGGL(k_dr_dtp<256>, dim3(a.n_solve), dim3(256), 0, st, a); break;
    case 512: hipLaunchKernelGGL(k_dr_dtp<512>, dim3(a.n_solve), dim3(512), 0, st, a); break;
    case 1024: hipLaunchKernelGGL(k_dr_dtp<1024>, dim3(a.n_solve), dim3(1024), 0, st, a); break;
    default: return -1001;
    }
    return (int)hipGetLastError();
}

} // namespace drk
