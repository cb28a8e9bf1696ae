// Device code of libdr: the templates of the dynamic-relaxation kernels
// and their helpers, included by every translation unit that instantiates
// kernels (dr_kernels.hip, dr_k_reg_*.hip, dr_k_glb_*.hip).
//
// HIP kernels for batched dynamic relaxation on CDNA4 (gfx950).
//
// One workgroup runs the dynamic-relaxation loop of Fig. 1 for one
// sub-problem (section III: the loop moved inside a single kernel, one thread
// team per sub-problem).  Per pass, every thread
//   1. moves its free nodes: q += dt w            (w = half-step velocity)
//   2. barrier
//   3. gathers the internal force on each of its nodes over the node's
//      incidences (deterministic node -> fiber gather, no atomics)
//   4. forms the damped acceleration, the full-step and next half-step
//      velocities, and its share of |g_free|^2, |g_B|^2 and 2 KE (FP64)
//   5. wavefront reduction -> LDS -> every wave reduces the wave partials
//      in the same fixed order and takes lane 0's totals, so the stop
//      decision is uniform.
// A launch makes at most `budget` passes per problem.  A solve that is still
// running when the budget is spent saves its state (exactly) to HBM and a
// later launch resumes it, so a solve split over several launches gives the
// same bits as one launch.  A finished solve writes its displacements; a
// separate launch (k_stress) forms the reactions and both stress forms.
//
// Placements:
//   k_dr_reg<P, BLOCK, NPT, CH>: state q in LDS (24 B per node), the half-step velocity
//     and degree of each owned node in registers, NPT nodes per thread;
//   k_dr_glb<P, BLOCK>: state and velocities in device memory, any size.
// Precision policies:
//   P64: q = positions x (FP64), fiber constants {EA/(2L^2), L^2};
//   P32: q = displacement beyond the affine field, u - (F - I) X (FP32),
//        fiber constants {dX, EA/(2L^2)} in FP32, strain numerator in the
//        Green form dX.(F^T F - I)dX + 2 (F dX).dq + dq.dq (exactly zero at
//        the reference state); the norm reductions and the stress are FP64.
// The topology streams from device memory every pass (L2 / MALL resident).
#pragma once
#include <hip/hip_runtime.h>

#include "dr_layout.h"

namespace drk {

// No implicit contraction in this file: every multiply-add that the
// iteration's state depends on is written as an explicit fma, so all kernels
// and launch shapes round the per-node arithmetic identically (the compiler
// would otherwise fuse differently in different instantiations).
#pragma clang fp contract(off)

enum { kConverged = 0, kMaxIter = 1, kNonFinite = 2 };
// passes between two energy-balance checks
constexpr int kEnergyEvery = 1024;
// passes between two checks of how many problems of a launch still run
// (the tail hand-off); divides kEnergyEvery
constexpr int kDrainEvery = 256;
// LDS slot (in wave 0's reduction record) of the hand-off decision:
// doubles 4.. of each record hold the register variant's row headers
constexpr int kDrainSlotReg = 3;
constexpr int kDrainSlotGlb = 4;

// Progress of a running solve for the optional stall guard.
struct Progress {
    double best;   // best squared residual ratio rho^2 so far
    int64_t nbest; // pass at which it was reached
};
enum { kStartAffine = 0, kStartZero = 1, kStartWarm = 2 };

// Per-wave LDS record (doubles): the 3 partial sums of a pass (18 in the
// stress kernel); in k_dr_reg doubles 4.. hold the wave's row headers.
constexpr int kRedStride = 20;

// Cross-lane move of a double with a DPP control (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Index of the thread's wave in the workgroup, known to the compiler to be
// uniform over the wave (scalar registers).
__device__ __forceinline__ int wave_id(int tid)
{
    return __builtin_amdgcn_readfirstlane(tid / kWave);
}

// v + (v of lane ^ 16), resp. ^ 32, in every lane, with the gfx950 row
// swaps: swapping the odd 16-lane rows of one copy of v with the even rows of
// another leaves (row 0, row 0, row 2, row 2) and (row 1, row 1, row 3,
// row 3), whose sum is the butterfly step; the 32-lane swap does the same
// with the two halves.
__device__ __forceinline__ double add_xor16(double v)
{
    const unsigned lo = __double2loint(v), hi = __double2hiint(v);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}

__device__ __forceinline__ double add_xor32(double v)
{
    const unsigned lo = __double2loint(v), hi = __double2hiint(v);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}

// Wavefront sum in a fixed order: quad swaps and row rotations (DPP, within
// rows of 16 lanes: row_sum), then the two cross-row steps (row swaps).
// Deterministic; lane 0's value is the one the callers use.  The second
// level of the block sums has its NW <= 16 partials in lanes 0..NW-1 and
// zeros elsewhere, so row_sum alone gives lane 0 the same total.
__device__ __forceinline__ double row_sum(double v)
{
    v += dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);  // quad_perm [2,3,0,1]
    v += dpp_f64<0x124>(v); // row_ror:4
    v += dpp_f64<0x128>(v); // row_ror:8
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
    v = row_sum(v);
    v = add_xor16(v);
    v = add_xor32(v);
    return v;
}

// Squared length fma(dz, dz, fma(dy, dy, dx * dx)).  The host forms the L^2
// of every incidence with the same operations in the same order, so a fiber
// at its reference length carries exactly zero force.
__device__ __forceinline__ double len2(double dx, double dy, double dz)
{
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// 1 / sqrt(x) for a positive normal x: the hardware estimate refined by one
// second-order Householder step, e = 1 - x y^2, y <- y + y e (1/2 + 3/8 e)
// (no special-case handling: every l^2 reaching it is positive).
__device__ __forceinline__ double rsq64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// x^2 + y^2 + z^2 as fma(z, z, fma(y, y, x x)).
template <class T> __device__ __forceinline__ T sq3(T x, T y, T z)
{
    return fma(z, z, fma(y, y, x * x));
}

// g += s d, one fma per component.
template <class T>
__device__ __forceinline__ void axpy3(T s, T dx, T dy, T dz, T &gx, T &gy, T &gz)
{
    gx = fma(s, dx, gx);
    gy = fma(s, dy, gy);
    gz = fma(s, dz, gz);
}

// One component of the damped velocity update (Fig. 1: damping force,
// acceleration a = g / m - c w, then the two half-step updates w + dt/2 a):
// returns the mid-pass velocity, leaves the new half-step velocity in w.
template <class T>
__device__ __forceinline__ T vel_step(T g, T im, T cdamp, T hdt, T &w)
{
    const T acc = fma(g, im, -(cdamp * w));
    const T v = fma(hdt, acc, w);
    w = fma(hdt, acc, v);
    return v;
}

struct P64 {
    using T = double;
    static constexpr bool kDisp = false;
};
struct P32 {
    using T = float;
    static constexpr bool kDisp = true;
};

// Running state of one problem in LDS: 3 values per node, node after node
// (one address per node, the components at immediate offsets).  The byte
// offset of a node is a 24-bit product (node ids stay below 2^21).
template <class T> struct LdsQ {
    T *a;
    int n;
    __device__ __forceinline__ const T *rec(int j) const
    {
        return reinterpret_cast<const T *>(reinterpret_cast<const char *>(a) +
                                           __umul24((uint32_t)j, 3u * sizeof(T)));
    }
    __device__ __forceinline__ void load(int j, T &x, T &y, T &z) const
    {
        const T *q = rec(j);
        x = q[0]; y = q[1]; z = q[2];
    }
    __device__ __forceinline__ void store(int j, T x, T y, T z) const
    {
        T *q = a + 3 * j;
        q[0] = x; q[1] = y; q[2] = z;
    }
};

// Running state of a node in device memory: a 24-byte record holding the
// FP64 position (x, y, z), or a 32-byte one holding the FP32 state
// (q0, q1, q2, -) followed by the compensation terms of its summed updates
// (c0, c1, c2, -).  (The neighbour reads of the global variant come from
// beyond L2; a record without padding makes them fewer bytes.)
template <class T> constexpr int kQStride = sizeof(T) == 8 ? 3 : 8;
// The half-step velocity record of a node kept between launches (and in
// device memory by the global variant): 24 bytes in FP64, 16 in FP32.
template <class T> constexpr int kWStride = sizeof(T) == 8 ? 3 : 4;

template <class T> struct GlbQ {
    T *base;
    // a uniform base plus a 32-bit byte offset (node ids stay below 2^21)
    __device__ __forceinline__ void load(int j, T &x, T &y, T &z) const
    {
        const T *q = reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                                 (uint32_t)j * (uint32_t)(kQStride<T> * sizeof(T)));
        x = q[0]; y = q[1]; z = q[2];
    }
    __device__ __forceinline__ void store(int j, T x, T y, T z) const
    {
        T *q = base + kQStride<T> * (int64_t)j;
        q[0] = x; q[1] = y; q[2] = z;
    }
};

// q += dt w.  FP64 adds directly.  FP32 uses compensated (Kahan) summation:
// near convergence dt w falls below half an ulp of q and a plain FP32 add
// would drop it, freezing the iteration short of equilibrium.
template <class T>
__device__ __forceinline__ void advance_q(T &q, T dt, T w, T &comp)
{
    if constexpr (sizeof(T) == 8) {
        q = fma(dt, w, q);
    } else {
        const T y = dt * w - comp;
        const T t = q + y;
        comp = (t - q) - y;
        q = t;
    }
}

// Element r of a per-node array of one problem: a uniform base plus a 32-bit
// byte offset (a scalar-base load; node ids stay below 2^21).
template <class E> __device__ __forceinline__ E node_at(const E *base, int r)
{
    return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(base) +
                                        (uint32_t)r * (uint32_t)sizeof(E));
}

// Record r of a per-node array with S elements per node, the same way.
template <int S, class E> __device__ __forceinline__ E *node_rec(E *base, int r)
{
    return reinterpret_cast<E *>(reinterpret_cast<char *>(base) + (uint32_t)r * (uint32_t)(S * sizeof(E)));
}

// Inverse mass and mass of node r of the problem whose nodes start at nb.
template <class Prec, class T = typename Prec::T>
__device__ __forceinline__ void node_mass(const SolveArgs &A, int64_t nb, int r, T &im, double &m)
{
    if constexpr (Prec::kDisp) {
        im = node_at(A.invm32 + nb, r);
        m = (double)node_at(A.mass32 + nb, r);
    } else {
        im = node_at(A.invm + nb, r);
        m = node_at(A.mass + nb, r);
    }
}

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

// ---------------------------------------------------------------------------
// Force gather (Fig. 1, getInternalForces): g_i = sum over the node's fibers
// of T d / l, d pointing from node i to the neighbour, T = EA (l^2/L^2 - 1)/2
// = k (l^2 - L^2), k = EA / (2 L^2).
//
// The slice width is wave-uniform, so the row is walked in chunks of C
// incidences whose loads are unconditional: C neighbour ids and constants
// from L2, then the C neighbour states from LDS, then C independent chains.
// Entries past the node's own degree (padding up to the slice width) hold a
// valid neighbour id and are masked out by a select, never by a branch.
// Contributions are added in ascending incidence order.
// ---------------------------------------------------------------------------
template <int C, bool STRESS, class Pos>
__device__ __forceinline__ void chunk64(const SolveArgs &A, int64_t e, const Pos &pos, int k0,
                                        int d, double xi, double yi, double zi, double &gx,
                                        double &gy, double &gz, double *sf)
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
        double s = c[t].k * (l2 - c[t].L2) * rsq64(l2);
        s = (k0 + t < d) ? s : 0.0;
        axpy3(s, dx[t], dy[t], dz[t], gx, gy, gz);
        if (STRESS) {
            const double hs = 0.5 * s;
            const double dv[3] = {dx[t], dy[t], dz[t]};
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) sf[3 * p + q] = fma(hs * dv[p], dv[q], sf[3 * p + q]);
        }
    }
}

// FP32 state: q = u - (F - I) X, the displacement beyond the affine field
// (the smooth affine part would otherwise dominate |u| and round away the
// small differences between neighbours).  For a fiber with reference vector
// dX and dq = q_j - q_i:
//   d = F dX + dq,  l^2 - L^2 = dX.(F^T F - I) dX + 2 (F dX).dq + dq.dq,
// all of it well conditioned and exactly zero at the reference state.
struct Aff32 {
    float F[9]; // row-major F
    float C[6]; // F^T F - I: C00, C11, C22, 2 C01, 2 C02, 2 C12
};

template <int C, class Pos>
__device__ __forceinline__ void chunk32(const SolveArgs &A, const Aff32 &af, int64_t e,
                                        const Pos &pos, int k0, int d, float qi0, float qi1,
                                        float qi2, float &gx, float &gy, float &gz)
{
    int j[C];
    KL32 c[C];
#pragma unroll
    for (int t = 0; t < C; ++t) {
        j[t] = A.nbr[e + (int64_t)t * kWave];
        c[t] = A.kl32[e + (int64_t)t * kWave];
    }
    float dq0[C], dq1[C], dq2[C];
#pragma unroll
    for (int t = 0; t < C; ++t) {
        pos.load(j[t], dq0[t], dq1[t], dq2[t]);
        dq0[t] -= qi0; dq1[t] -= qi1; dq2[t] -= qi2;
    }
#pragma unroll
    for (int t = 0; t < C; ++t) {
        const float X0 = c[t].dx, X1 = c[t].dy, X2 = c[t].dz;
        const float f0 = fma(af.F[2], X2, fma(af.F[1], X1, af.F[0] * X0));
        const float f1 = fma(af.F[5], X2, fma(af.F[4], X1, af.F[3] * X0));
        const float f2 = fma(af.F[8], X2, fma(af.F[7], X1, af.F[6] * X0));
        const float eaff = fma(af.C[5] * X1, X2, fma(af.C[4] * X0, X2, fma(af.C[3] * X0, X1,
                           fma(af.C[2] * X2, X2, fma(af.C[1] * X1, X1, af.C[0] * X0 * X0)))));
        const float fdq = fma(f2, dq2[t], fma(f1, dq1[t], f0 * dq0[t]));
        const float ex = fma(2.0f, fdq, eaff) + sq3(dq0[t], dq1[t], dq2[t]);
        const float dx = f0 + dq0[t], dy = f1 + dq1[t], dz = f2 + dq2[t];
        const float l2 = sq3(dx, dy, dz);
        float s = c[t].k * ex * rsqrtf(l2);
        s = (k0 + t < d) ? s : 0.0f;
        axpy3(s, dx, dy, dz, gx, gy, gz);
    }
}

__device__ __forceinline__ Aff32 make_aff32(const double *F)
{
    Aff32 a;
#pragma unroll
    for (int k = 0; k < 9; ++k) a.F[k] = (float)F[k];
    double C[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            C[p][q] = F[p] * F[q] + F[3 + p] * F[3 + q] + F[6 + p] * F[6 + q] - (p == q ? 1.0 : 0.0);
    a.C[0] = (float)C[0][0]; a.C[1] = (float)C[1][1]; a.C[2] = (float)C[2][2];
    a.C[3] = (float)(2.0 * C[0][1]); a.C[4] = (float)(2.0 * C[0][2]); a.C[5] = (float)(2.0 * C[1][2]);
    return a;
}

template <class P, int CH, class Pos, class T = typename P::T>
__device__ __forceinline__ void gather(const SolveArgs &A, const Aff32 &af, const Row &row,
                                       const Pos &pos, int lane, int d, T qi0, T qi1, T qi2,
                                       T &gx, T &gy, T &gz)
{
    static_assert(CH == 1 || CH == 2 || CH == 4, "chunk of 1, 2 or 4 incidences");
    gx = 0; gy = 0; gz = 0;
    int64_t e = row.e0 + lane;
    int k0 = 0;
    if constexpr (P::kDisp) {
        for (; k0 + CH <= row.width; k0 += CH, e += CH * kWave)
            chunk32<CH>(A, af, e, pos, k0, d, qi0, qi1, qi2, gx, gy, gz);
        if (CH == 4 && k0 + 2 <= row.width) {
            chunk32<2>(A, af, e, pos, k0, d, qi0, qi1, qi2, gx, gy, gz);
            k0 += 2;
            e += 2 * kWave;
        }
        if (k0 < row.width) chunk32<1>(A, af, e, pos, k0, d, qi0, qi1, qi2, gx, gy, gz);
    } else {
        for (; k0 + CH <= row.width; k0 += CH, e += CH * kWave)
            chunk64<CH, false>(A, e, pos, k0, d, qi0, qi1, qi2, gx, gy, gz, nullptr);
        if (CH == 4 && k0 + 2 <= row.width) {
            chunk64<2, false>(A, e, pos, k0, d, qi0, qi1, qi2, gx, gy, gz, nullptr);
            k0 += 2;
            e += 2 * kWave;
        }
        if (k0 < row.width) chunk64<1, false>(A, e, pos, k0, d, qi0, qi1, qi2, gx, gy, gz, nullptr);
    }
}

// FP64 gather that also accumulates 1/2 (T / l) d (x) d into the fiber
// stress (each fiber is visited from both ends).
template <class Pos>
__device__ __forceinline__ void gather_stress(const SolveArgs &A, const Row &row, const Pos &pos,
                                              int lane, int d, double xi, double yi, double zi,
                                              double &gx, double &gy, double &gz, double *sf)
{
    gx = 0.0; gy = 0.0; gz = 0.0;
    int64_t e = row.e0 + lane;
    int k0 = 0;
    for (; k0 + 2 <= row.width; k0 += 2, e += 2 * kWave)
        chunk64<2, true>(A, e, pos, k0, d, xi, yi, zi, gx, gy, gz, sf);
    if (k0 < row.width) chunk64<1, true>(A, e, pos, k0, d, xi, yi, zi, gx, gy, gz, sf);
}

// ---------------------------------------------------------------------------
// Software-pipelined gather of the pass loops.  A wave's rows are walked as
// one stream of chunks of C incidences; the neighbour ids and constants of
// the next chunk are loaded before the current chunk's neighbour states are
// read and its forces formed.  Every entry of a row up to the slice width is
// summed: padding entries carry zero constants and point at a real
// neighbour of the node (a positive length), so they add exactly zero and
// need no per-lane mask; entries past the width (the last chunk of a row) are
// skipped by a wave-uniform test.  Loads use the problem's base pointers
// (uniform) and 32-bit per-lane offsets.
// ---------------------------------------------------------------------------
template <class Prec> struct KLof;
template <> struct KLof<P64> { using type = KL; };
template <> struct KLof<P32> { using type = KL32; };

template <class Prec, int C> struct Pref {
    int j[C];
    typename KLof<Prec>::type c[C];
};

// Header of one slice (wave-uniform): first entry relative to the problem's
// incidence base, and width (0: no such slice for this wave).
struct RowHdr {
    uint32_t off;
    int32_t w;
};

// A header read from LDS, made wave-uniform (scalar registers).
__device__ __forceinline__ RowHdr uniform_hdr(const RowHdr *p)
{
    const RowHdr h = *p;
    return RowHdr{(uint32_t)__builtin_amdgcn_readfirstlane((int)h.off),
                  __builtin_amdgcn_readfirstlane(h.w)};
}

// One problem's incidence arrays as buffer resources (base, size in bytes;
// 32-bit raw data), read with a uniform (scalar) offset for the entry and a
// per-lane offset that stays fixed: no per-lane address arithmetic in the
// loop, and an offset past the end reads zero instead of faulting.
constexpr int kBufWord3 = 0x00020000; // data format 32, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_of(const void *p, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kBufWord3);
}

template <class Prec> struct Topo {
    __amdgpu_buffer_rsrc_t nbr, kl;
};

template <class Prec>
__device__ __forceinline__ Topo<Prec> topo_of(const SolveArgs &A, const ProbDesc &P)
{
    using KLT = typename KLof<Prec>::type;
    static_assert(sizeof(KLT) == 16, "16-byte incidence constants");
    Topo<Prec> t;
    t.nbr = buf_of(A.nbr + P.inc_base, P.n_inc * 4);
    if constexpr (Prec::kDisp) t.kl = buf_of(A.kl32 + P.inc_base, P.n_inc * 16);
    else t.kl = buf_of(A.kl + P.inc_base, P.n_inc * 16);
    return t;
}

// Loads entries k0 .. k0+C-1 of a row (clamped to its last entry): the
// row's entry k starts at a uniform address, the lane indexes into it.
template <class Prec, int C>
__device__ __forceinline__ void pref_load(const Topo<Prec> &tp, RowHdr h, int k0, int lane,
                                          Pref<Prec, C> &pf)
{
    using KLT = typename KLof<Prec>::type;
    const int oj = lane * 4, oc = lane * 16;
#pragma unroll
    for (int t = 0; t < C; ++t) {
        const int k = k0 + t < h.w ? k0 + t : h.w - 1;
        const int e = (int)h.off + k * kWave; // uniform
        pf.j[t] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(tp.nbr, oj, e * 4, 0);
        pf.c[t] = __builtin_bit_cast(KLT, __builtin_amdgcn_raw_buffer_load_b128(tp.kl, oc, e * 16, 0));
    }
}

// Forces of the first nv (>= 1) entries of one chunk whose neighbour states
// px, py, pz are loaded, added in entry order.
template <int C>
__device__ __forceinline__ void force_pre(const KL (&c)[C], const double (&px)[C],
                                          const double (&py)[C], const double (&pz)[C],
                                          const Aff32 &, int nv, double xi, double yi, double zi,
                                          double &gx, double &gy, double &gz)
{
#pragma unroll
    for (int t = 0; t < C; ++t) {
        if (t > 0 && t >= nv) break;
        const double dx = px[t] - xi, dy = py[t] - yi, dz = pz[t] - zi;
        const double l2 = len2(dx, dy, dz);
        const double s = c[t].k * (l2 - c[t].L2) * rsq64(l2);
        axpy3(s, dx, dy, dz, gx, gy, gz);
    }
}

template <int C>
__device__ __forceinline__ void force_pre(const KL32 (&c)[C], const float (&px)[C],
                                          const float (&py)[C], const float (&pz)[C],
                                          const Aff32 &af, int nv, float qi0, float qi1, float qi2,
                                          float &gx, float &gy, float &gz)
{
#pragma unroll
    for (int t = 0; t < C; ++t) {
        if (t > 0 && t >= nv) break;
        const float dq0 = px[t] - qi0, dq1 = py[t] - qi1, dq2 = pz[t] - qi2;
        const float X0 = c[t].dx, X1 = c[t].dy, X2 = c[t].dz;
        const float f0 = fma(af.F[2], X2, fma(af.F[1], X1, af.F[0] * X0));
        const float f1 = fma(af.F[5], X2, fma(af.F[4], X1, af.F[3] * X0));
        const float f2 = fma(af.F[8], X2, fma(af.F[7], X1, af.F[6] * X0));
        const float eaff = fma(af.C[5] * X1, X2, fma(af.C[4] * X0, X2, fma(af.C[3] * X0, X1,
                           fma(af.C[2] * X2, X2, fma(af.C[1] * X1, X1, af.C[0] * X0 * X0)))));
        const float fdq = fma(f2, dq2, fma(f1, dq1, f0 * dq0));
        const float ex = fma(2.0f, fdq, eaff) + sq3(dq0, dq1, dq2);
        const float dx = f0 + dq0, dy = f1 + dq1, dz = f2 + dq2;
        const float l2 = sq3(dx, dy, dz);
        const float s = c[t].k * ex * rsqrtf(l2);
        axpy3(s, dx, dy, dz, gx, gy, gz);
    }
}

// Forces of one prefetched chunk on a node: neighbour states from pos, then
// force_pre.
template <class Prec, int C, class Pos, class T = typename Prec::T>
__device__ __forceinline__ void force_chunk(const Pref<Prec, C> &pf, const Aff32 &af,
                                            const Pos &pos, int nv, T qi0, T qi1, T qi2, T &gx,
                                            T &gy, T &gz)
{
    T px[C], py[C], pz[C];
#pragma unroll
    for (int t = 0; t < C; ++t) pos.load(pf.j[t], px[t], py[t], pz[t]);
    force_pre<C>(pf.c, px, py, pz, af, nv, qi0, qi1, qi2, gx, gy, gz);
}

// ---------------------------------------------------------------------------
// Per-slot set-up shared by the kernels
// ---------------------------------------------------------------------------
struct Slot {
    ProbDesc P;
    int slot, p, start; // start: dr_start of a new solve, or kResume
    int64_t sb;         // first running-state record of the problem (qbuf, wbuf)
    double F[9];
};

__device__ __forceinline__ Slot load_slot(const SolveArgs &A, int slot)
{
    Slot S;
    S.slot = slot;
    S.p = A.ids ? A.ids[slot] : slot;
    S.P = A.probs[S.p];
    S.sb = A.state_off[S.p];
    S.start = A.starts ? A.starts[slot] : A.start;
    const double *F = (S.start == kResume) ? A.F_cur + 9 * (int64_t)S.p : A.F + 9 * (int64_t)slot;
#pragma unroll
    for (int k = 0; k < 9; ++k) S.F[k] = F[k];
    return S;
}

// ((F - I) X)_a
__device__ __forceinline__ double affine_u(const double *F, const double *X, int a)
{
    return (F[3 * a] - (a == 0 ? 1.0 : 0.0)) * X[0] + (F[3 * a + 1] - (a == 1 ? 1.0 : 0.0)) * X[1] +
           (F[3 * a + 2] - (a == 2 ? 1.0 : 0.0)) * X[2];
}

// Start displacement of local node r (Fig. 1 step 4 and the initialisation):
// prescribed nodes u = (F - I) X; free nodes from the affine field, from
// u = 0, or warm (u_prev + (F - F_prev) X).
__device__ __forceinline__ void start_u(const SolveArgs &A, const Slot &S, int r, double u[3])
{
    const int64_t gi = S.P.node_base + r;
    const double X[3] = {A.X[3 * gi], A.X[3 * gi + 1], A.X[3 * gi + 2]};
    const bool warm = S.start == kStartWarm && A.has_state[S.p];
    const double *Fl = A.F_last + 9 * (int64_t)S.p;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r >= S.P.N_free || S.start == kStartAffine || (S.start == kStartWarm && !warm)) {
            u[a] = affine_u(S.F, X, a);
        } else if (S.start == kStartZero) {
            u[a] = 0.0;
        } else {
            const double dfx = (S.F[3 * a] - Fl[3 * a]) * X[0] +
                               (S.F[3 * a + 1] - Fl[3 * a + 1]) * X[1] +
                               (S.F[3 * a + 2] - Fl[3 * a + 2]) * X[2];
            u[a] = A.u[3 * gi + a] + dfx;
        }
    }
}

// State q of node r at the start of a solve: the position (FP64) or the
// displacement beyond the affine field (FP32, exactly zero on prescribed
// nodes and for the affine start).
template <class P, class T = typename P::T>
__device__ __forceinline__ void start_q(const SolveArgs &A, const Slot &S, int r, T q[3])
{
    double u[3];
    start_u(A, S, r, u);
    const int64_t gi = S.P.node_base + r;
    const double X[3] = {A.X[3 * gi], A.X[3 * gi + 1], A.X[3 * gi + 2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        q[a] = P::kDisp ? (T)(u[a] - affine_u(S.F, X, a)) : (T)(X[a] + u[a]);
}

// Displacement written back for node r at the end of a solve (prescribed
// nodes get their exact affine value).
template <class P, class T = typename P::T>
__device__ __forceinline__ void write_u(const SolveArgs &A, const Slot &S, int r, const T q[3])
{
    const int64_t gi = S.P.node_base + r;
    const double X[3] = {A.X[3 * gi], A.X[3 * gi + 1], A.X[3 * gi + 2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double u;
        if (r < S.P.N_free) u = P::kDisp ? (double)q[a] + affine_u(S.F, X, a) : (double)q[a] - X[a];
        else u = affine_u(S.F, X, a);
        A.u[3 * gi + a] = u;
    }
}

// Lane 0's value of a double, in every lane.
__device__ __forceinline__ double lane0(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Block-wide sums; every thread returns the same totals.  Each wave reduces
// its lanes and lane 0 posts the partials; after the barrier every wave
// reduces the NW partials over its lanes 0..NW-1 (the same inputs in the
// same lanes, so the same rounding in every wave) and takes lane 0's
// result, so all threads agree bit for bit.  The caller guarantees that no
// thread still reads the previous sums (a barrier since their last use).
template <int NW>
__device__ __forceinline__ void block_sum2(double *red, int lane, int wave, double &a, double &b)
{
    static_assert(NW <= 16, "the partials fit one 16-lane row");
    a = wave_sum(a); b = wave_sum(b);
    if (lane == 0) {
        red[wave * kRedStride + 0] = a;
        red[wave * kRedStride + 1] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
    if (lane < NW) {
        ta = red[lane * kRedStride + 0];
        tb = red[lane * kRedStride + 1];
    }
    a = lane0(row_sum(ta));
    b = lane0(row_sum(tb));
}

// The pass loops split a two-value block sum around their own barrier:
// wave_partials2 posts each wave's sums (lane 0), and after the barrier
// block_totals2 reduces the NW records over lanes 0..NW-1 of every wave
// (the same inputs in the same lanes, so the same rounding in every wave)
// and takes lane 0's result, so all threads hold the same bits.  The caller guarantees that no thread still reads the previous
// partials (a barrier since their last use).
template <int NW>
__device__ __forceinline__ void wave_partials2(double *red, int lane, int wave, double a, double b,
                                               bool has_a, bool has_b, int slot = 0)
{
    // a wave without free (resp. prescribed) nodes holds exact zeros: its
    // partial is 0 without the reduction (wave-uniform flags)
    a = has_a ? wave_sum(a) : 0.0;
    b = has_b ? wave_sum(b) : 0.0;
    if (lane == 0) {
        red[wave * kRedStride + slot] = a;
        red[wave * kRedStride + slot + 1] = b;
    }
}

// Whether the nodes r = i BLOCK + wave 64 + lane (i >= 0, r < N) of a wave
// include free ones (r < Nf) and prescribed ones (Nf <= r < N).
__device__ __forceinline__ bool wave_has_free(int wave, int Nf)
{
    return wave * kWave < Nf;
}

template <int BLOCK>
__device__ __forceinline__ bool wave_has_prescribed(int wave, int Nf, int N)
{
    const int base = wave * kWave;
    int i = Nf - base - (kWave - 1); // first i whose 64 nodes reach Nf
    i = i <= 0 ? 0 : (i + BLOCK - 1) / BLOCK;
    return Nf < N && i * BLOCK + base <= N - 1;
}

template <int NW>
__device__ __forceinline__ void block_totals2(const double *red, int lane, double &a, double &b,
                                              int slot = 0)
{
    static_assert(NW <= 16, "the partials fit one 16-lane row");
    double ta = 0.0, tb = 0.0;
    if (lane < NW) {
        ta = red[lane * kRedStride + slot];
        tb = red[lane * kRedStride + slot + 1];
    }
    a = lane0(row_sum(ta));
    b = lane0(row_sum(tb));
}

// One block-wide sum, with a barrier first (callable right after block_sum2).
template <int NW>
__device__ __forceinline__ double block_sum1(double *red, int lane, int wave, double a)
{
    static_assert(NW <= 16, "the partials fit one 16-lane row");
    __syncthreads();
    a = wave_sum(a);
    if (lane == 0) red[wave * kRedStride + 2] = a;
    __syncthreads();
    const double t = lane < NW ? red[lane * kRedStride + 2] : 0.0;
    return lane0(row_sum(t));
}

// Four block-wide sums, with a barrier first (slots 0..3 of each wave's record).
template <int NW>
__device__ __forceinline__ void block_sum4(double *red, int lane, int wave, double (&v)[4])
{
    static_assert(NW <= 16, "the partials fit one 16-lane row");
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) red[wave * kRedStride + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = lane < NW ? red[lane * kRedStride + k] : 0.0;
        v[k] = lane0(row_sum(t));
    }
}

// Energy balance (Fig. 1, the optional check).  Per free node and pass, with
// w_old / w_new the half-step velocities before / after the pass's velocity
// updates and g the pass's internal force:
//   e[0] += g . (w_old + w_new)   (x dt/2: the trapezoid work of g over the
//                                  displacement steps dt w_old and dt w_new)
//   e[1] += m |w_old|^2           (x c dt: damping work over the step)
//   e[2]  = g . w_new             (the forward half of the last pass)
// so W = dt/2 (sum e[0] - sum e[2]) and D = c dt sum e[1] once a solve has
// finished (while it runs, the forward half belongs to the next step).
__device__ __forceinline__ void energy_node(const SolveArgs &A, int64_t gi, double gdot,
                                            double mw2, double glast)
{
    double *e = A.enode + 4 * gi;
    e[0] += gdot;
    e[1] += mw2;
    e[2] = glast;
}

// The record update of one pass, from the force g and the half-step
// velocity w_old before the pass's velocity updates (recomputing w_new as
// those updates do).
template <class T>
__device__ __forceinline__ void energy_pass(const SolveArgs &A, int64_t gi, const T (&g)[3],
                                            const T (&wo)[3], T im, T cdamp, T hdt, double m)
{
    double gdot = 0.0, wo2 = 0.0, glast = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T wn = wo[a];
        vel_step(g[a], im, cdamp, hdt, wn);
        gdot = fma((double)g[a], (double)wo[a] + (double)wn, gdot);
        wo2 = fma((double)wo[a], (double)wo[a], wo2);
        glast = fma((double)g[a], (double)wn, glast);
    }
    energy_node(A, gi, gdot, m * wo2, glast);
}

// Work totals of a problem from the thread-summed records s = {sum e[0],
// sum e[1], sum e[2]} (block sums).
__device__ __forceinline__ void energy_totals(const ProbDesc &P, const double (&s)[4], bool finished,
                                              double &W, double &D)
{
    W = 0.5 * P.dt * (s[0] - (finished ? s[2] : 0.0));
    D = P.c * P.dt * s[1];
}

// The balance test of energy_tol: |KE - W + D| <= tol max(KE, |W|, D).
__device__ __forceinline__ bool energy_ok(double tol, double KE, double W, double D)
{
    const double scale = fmax(KE, fmax(fabs(W), D));
    return fabs(KE - W + D) <= tol * scale;
}

// Residual and stop test (Fig. 1: force residual, iteration count, until
// converged), plus the optional stall guard.  rho = |g_free| / max(|g_B|,
// s_floor) <= tol is tested in squared form, gf2 <= tol^2 max(gb2, s_floor^2),
// which needs no square root or division in the loop.  Returns true when the
// solve is finished.
__device__ __forceinline__ bool stop_test(const SolveArgs &A, const ProbDesc &P, double tol2,
                                          double gf2, double gb2, int64_t n, int &status,
                                          Progress &pg)
{
    const double fl2 = P.s_floor * P.s_floor;
    const double den2 = gb2 > fl2 ? gb2 : fl2;
    if (!isfinite(gf2) || !isfinite(gb2)) { status = kNonFinite; return true; }
    if (gf2 <= tol2 * den2) { status = kConverged; return true; }
    if (n >= A.max_iter) { status = kMaxIter; return true; }
    // progress (only with the stall guard on): rho^2 below (1 - 1e-3)^2 of
    // the best so far
    if (A.stall_window > 0) {
        if (gf2 < pg.best * den2 * 0.998001) {
            pg.best = gf2 / den2;
            pg.nbest = n;
        } else if (n - pg.nbest >= A.stall_window) {
            status = kStatusStalled;
            return true;
        }
    }
    return false;
}

// Reported residual ratio and kinetic energy of the last pass.
__device__ __forceinline__ void final_scalars(const ProbDesc &P, double gf2, double gb2,
                                              double ke2, double &rho, double &ke)
{
    double den = sqrt(gb2);
    if (den < P.s_floor) den = P.s_floor;
    rho = sqrt(gf2) / den;
    ke = 0.5 * ke2;
}

// Scalars of the problem after a launch (thread 0 writes).
__device__ __forceinline__ void record(const SolveArgs &A, const Slot &S, int64_t n, double rho,
                                       double ke, int status, const Progress &pg)
{
    A.iters[S.p] = n;
    A.rho_best[S.p] = pg.best;
    A.n_best[S.p] = pg.nbest;
    A.rho[S.p] = rho;
    A.ke[S.p] = ke;
    A.status[S.p] = status;
    if (status != kStatusRunning && status != kStatusAborted) {
        for (int k = 0; k < 9; ++k) A.F_last[9 * (int64_t)S.p + k] = S.F[k];
        A.has_state[S.p] = 1;
    }
}

// End of a problem's part of a launch with the tail hand-off on (thread 0
// writes): a solve drained to the group launch joins the tail list (with
// the pass count its launch started at, from which the budget counts); any
// other leaves the count of the launch's problems still running.
__device__ __forceinline__ void launch_done(const SolveArgs &A, const Slot &S, int64_t n_start,
                                            bool drained)
{
    if (A.tail_at <= 0) return;
    if (drained) {
        const int k = __hip_atomic_fetch_add(A.tail_count, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        A.tail_list[k] = S.p;
        A.n_begin[S.p] = n_start;
    } else {
        __hip_atomic_fetch_add(A.live, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Passes problem p may make in this launch.
__device__ __forceinline__ int64_t launch_budget(const SolveArgs &A, int p)
{
    return A.budgets ? A.budgets[p] : A.budget;
}

// Start of a new solve: F of the solve kept for resumes and the stress.
__device__ __forceinline__ void begin_solve(const SolveArgs &A, const Slot &S)
{
    for (int k = 0; k < 9; ++k) A.F_cur[9 * (int64_t)S.p + k] = S.F[k];
    A.status[S.p] = kStatusRunning;
}

// Thread sums of the energy records of its free nodes (nodes s * BLOCK + t,
// s < NPT, in the register variant; t, t + BLOCK, ... in the global one).
template <int NPT, int BLOCK>
__device__ __forceinline__ void energy_sum_reg(const SolveArgs &A, int64_t nb, int Nf, int t,
                                               double (&e)[4])
{
#pragma unroll
    for (int s = 0; s < NPT; ++s) {
        const int r = s * BLOCK + t;
        if (r < Nf) {
            const double *x = A.enode + 4 * (nb + r);
            e[0] += x[0];
            e[1] += x[1];
            e[2] += x[2];
        }
    }
}

__device__ __forceinline__ void energy_sum_glb(const SolveArgs &A, int64_t nb, int Nf, int t, int stride,
                                               double (&e)[4])
{
    for (int r = t; r < Nf; r += stride) {
        const double *x = A.enode + 4 * (nb + r);
        e[0] += x[0];
        e[1] += x[1];
        e[2] += x[2];
    }
}

// ---------------------------------------------------------------------------
// Register-resident variant
// ---------------------------------------------------------------------------
template <class Prec, int BLOCK, int NPT, int CH>
__global__ void __launch_bounds__(BLOCK) k_dr_reg(SolveArgs A)
{
    using T = typename Prec::T;
    extern __shared__ double smem[];
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id(tid);
    const Slot S = load_slot(A, A.order ? A.order[blockIdx.x] : (int)blockIdx.x);
    // a resume of a solve that is not running is a no-op (uniform per workgroup)
    if (S.start == kResume && A.status[S.p] != kStatusRunning) {
        if (tid == 0) launch_done(A, S, 0, false);
        return;
    }
    const Aff32 af = make_aff32(S.F);
    const ProbDesc &P = S.P;
    const int N = P.N, Nf = P.N_free;
    // node records first (LDS address = 24-bit product), the per-wave
    // reduction records after them
    const LdsQ<T> pos{reinterpret_cast<T *>(smem), N};
    double *red = smem + (3 * N * (int)sizeof(T) + 7) / 8;
    const T dt = (T)P.dt, hdt = (T)(0.5 * P.dt), cdamp = (T)P.c;
    const int64_t nb = P.node_base;
    constexpr int QS = kQStride<T>;
    // the saved state after pass k lives in buffer k & 1 of the two state
    // buffers the global variant alternates (same layout)
    T *const qbase = reinterpret_cast<T *>(A.qbuf) + QS * S.sb;
    const int64_t qhalf = A.qhalf * (int64_t)(sizeof(double) / sizeof(T));
    constexpr int WS = kWStride<T>;
    T *wsave = reinterpret_cast<T *>(A.wbuf) + WS * S.sb;

    // headers of this wave's NPT slices, read each pass from LDS
    static_assert(4 + NPT <= kRedStride, "row headers fit the wave's LDS record");
    RowHdr *hdr = reinterpret_cast<RowHdr *>(red + wave * kRedStride + 4);
    if (lane < NPT) {
        RowHdr h{0, 0};
        const int r0 = lane * BLOCK + wave * kWave;
        if (r0 < N) {
            const int q = r0 >> 6;
            h.w = A.slice_w[P.slice_base + q];
            h.off = (uint32_t)A.slice_off[P.slice_base + q];
        }
        hdr[lane] = h;
    }
    const Topo<Prec> topo = topo_of<Prec>(A, P);

    T w[NPT][3];
    T cmp[NPT][3]; // compensation of the FP32 state updates (unused in FP64)
    int64_t n = 0;
    if (S.start != kResume) {
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + tid;
            w[s][0] = w[s][1] = w[s][2] = 0;
            cmp[s][0] = cmp[s][1] = cmp[s][2] = 0;
            if (r < N) {
                T q[3];
                start_q<Prec>(A, S, r, q);
                pos.store(r, q[0], q[1], q[2]);
            }
        }
        if (tid == 0) begin_solve(A, S);
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
                    T qi[3], g[3];
                    pos.load(r, qi[0], qi[1], qi[2]);
                    gather<Prec, CH>(A, af, row, pos, lane, A.deg[nb + r], qi[0], qi[1], qi[2], g[0],
                                     g[1], g[2]);
                    const T im = Prec::kDisp ? (T)A.invm32[nb + r] : (T)A.invm[nb + r];
#pragma unroll
                    for (int a = 0; a < 3; ++a) w[s][a] = hdt * (g[a] * im);
                    if (A.energy_tol > 0.0) {
                        // the record starts afresh: w_old = 0
                        const double gw = (double)g[0] * (double)w[s][0] + (double)g[1] * (double)w[s][1] +
                                          (double)g[2] * (double)w[s][2];
                        double *e = A.enode + 4 * (nb + r);
                        e[0] = gw;
                        e[1] = 0.0;
                        e[2] = gw;
                    }
                }
            }
        }
    } else {
        n = A.iters[S.p];
        const T *const qsave = qbase + (n & 1) * qhalf;
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + tid;
            w[s][0] = w[s][1] = w[s][2] = 0;
            cmp[s][0] = cmp[s][1] = cmp[s][2] = 0;
            if (r < N) {
                pos.store(r, qsave[QS * r], qsave[QS * r + 1], qsave[QS * r + 2]);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    w[s][a] = wsave[WS * r + a];
                    if constexpr (Prec::kDisp) cmp[s][a] = qsave[QS * r + 4 + a];
                }
            }
        }
    }
    __syncthreads();

    const int64_t n0 = n;
    const int64_t budget = launch_budget(A, S.p);
    const double tol2 = A.tol * A.tol;
    double rho = 0.0, ke = 0.0, gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
    int status = kStatusRunning;
    bool drained = false;
    Progress pg{__builtin_huge_val(), n};
    const bool has_free = wave_has_free(wave, Nf), has_pres = wave_has_prescribed<BLOCK>(wave, Nf, N);
    if (S.start == kResume) {
        pg.best = A.rho_best[S.p];
        pg.nbest = A.n_best[S.p];
    }
    // displacement update of the free dof (the first step of a pass; it is
    // taken at the end of the previous pass, once the stop test has passed,
    // so that a finished solve keeps the state its residual belongs to)
    auto advance_all = [&](int t) {
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + t;
            if (r < Nf) {
                T x, y, z;
                pos.load(r, x, y, z);
                advance_q(x, dt, w[s][0], cmp[s][0]);
                advance_q(y, dt, w[s][1], cmp[s][1]);
                advance_q(z, dt, w[s][2], cmp[s][2]);
                pos.store(r, x, y, z);
            }
        }
    };
    advance_all(tid);
    __syncthreads();
    // Two barriers per pass: after the gather (the partial sums are posted)
    // and after the displacement update.
    for (;;) {
        // An opaque copy of the thread index: everything derived from it
        // (node ids, addresses) is recomputed each pass instead of being held
        // in registers across the loop, which would spill at 1024 threads.
        int tp = tid;
        asm volatile("" : "+v"(tp));
        gf2 = 0.0; gb2 = 0.0; ke2 = 0.0;
        Pref<Prec, CH> pf;
        {
            const RowHdr h0 = uniform_hdr(hdr);
            if (h0.w > 0) pref_load<Prec, CH>(topo, h0, 0, lane, pf);
        }
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + tp;
            const RowHdr h = uniform_hdr(hdr + s);
            RowHdr hn{0, 0};
            if (s + 1 < NPT) hn = uniform_hdr(hdr + s + 1);
            if (h.w > 0) {
                // node state and mass first, so their loads overlap the gather
                T qi[3] = {0, 0, 0};
                if (r < N) pos.load(r, qi[0], qi[1], qi[2]);
                T im = 0;
                double m = 0.0;
                if (r < Nf) node_mass<Prec>(A, nb, r, im, m);
                T g[3] = {0, 0, 0};
                for (int k0 = 0; k0 < h.w; k0 += CH) {
                    const Pref<Prec, CH> cur = pf;
                    // next chunk: the rest of this row, else the next row, else
                    // (end of the stream) this row's first chunk again
                    RowHdr nh = h;
                    int nk = 0;
                    if (k0 + CH < h.w) nk = k0 + CH;
                    else if (hn.w > 0) nh = hn;
                    pref_load<Prec, CH>(topo, nh, nk, lane, pf);
                    force_chunk<Prec, CH>(cur, af, pos, h.w - k0, qi[0], qi[1], qi[2], g[0], g[1], g[2]);
                }
                if (r < N) {
                    const double gg = sq3((double)g[0], (double)g[1], (double)g[2]);
                    if (r < Nf) {
                        if (A.energy_tol > 0.0)
                            energy_pass<T>(A, nb + r, g, w[s], im, cdamp, hdt, m);
                        double vv = 0.0;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            // damping force, acceleration, partial velocity updates
                            const T v = vel_step(g[a], im, cdamp, hdt, w[s][a]);
                            vv = fma((double)v, (double)v, vv);
                        }
                        gf2 += gg;
                        ke2 = fma(m, vv, ke2);
                    } else {
                        gb2 += gg;
                    }
                }
            } else if (hn.w > 0) {
                // an empty row (prescribed nodes without fibers): prime the next
                pref_load<Prec, CH>(topo, hn, 0, lane, pf);
            }
        }
        wave_partials2<NW>(red, lane, wave, gf2, gb2, has_free, has_pres);
        // every kDrainEvery passes thread 0 reads how many problems of the
        // launch are still running; all threads read its decision after the
        // barrier (before any later block sum reuses the slot)
        const bool drain_pass = A.tail_at > 0 && ((n + 1) & (kDrainEvery - 1)) == 0;
        if (drain_pass && tid == 0)
            red[kDrainSlotReg] = __hip_atomic_load(A.live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <=
                                         A.tail_at ? 1.0 : 0.0;
        __syncthreads();
        block_totals2<NW>(red, lane, gf2, gb2);
        const bool drain_now = drain_pass && red[kDrainSlotReg] != 0.0;
        ++n;
        if (stop_test(A, P, tol2, gf2, gb2, n, status, pg)) break;
        if (A.energy_tol > 0.0 && n % kEnergyEvery == 0) {
            double e[4] = {0.0, 0.0, 0.0, ke2};
            energy_sum_reg<NPT, BLOCK>(A, nb, Nf, tp, e);
            block_sum4<NW>(red, lane, wave, e);
            double W, D;
            energy_totals(P, e, false, W, D);
            if (!energy_ok(A.energy_tol, 0.5 * e[3], W, D)) {
                status = kStatusEnergy;
                break;
            }
        }
        if (drain_now) {
            drained = true; // the rest of this solve runs in a group launch
            break;
        }
        if (n - n0 >= budget) break;
        advance_all(tp);
        __syncthreads();
    }
    // kinetic energy of the last pass (reported only)
    ke2 = block_sum1<NW>(red, lane, wave, ke2);
    final_scalars(P, gf2, gb2, ke2, rho, ke);
    if (A.energy_tol > 0.0) {
        double e[4] = {0.0, 0.0, 0.0, 0.0};
        energy_sum_reg<NPT, BLOCK>(A, nb, Nf, tid, e);
        block_sum4<NW>(red, lane, wave, e);
        double W, D;
        energy_totals(P, e, status != kStatusRunning, W, D);
        if (status != kStatusRunning && status != kStatusEnergy && status != kNonFinite &&
            !energy_ok(A.energy_tol, ke, W, D))
            status = kStatusEnergy;
        if (tid == 0) {
            A.e_work[S.p] = W;
            A.e_damp[S.p] = D;
        }
    }

    if (status != kStatusRunning) {
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + tid;
            if (r < N) {
                T q[3];
                pos.load(r, q[0], q[1], q[2]);
                write_u<Prec>(A, S, r, q);
            }
        }
    } else {
        // budget spent: save the exact state for the next launch
        T *const qsave = qbase + (n & 1) * qhalf;
#pragma unroll
        for (int s = 0; s < NPT; ++s) {
            const int r = s * BLOCK + tid;
            if (r < N) {
                T q[3];
                pos.load(r, q[0], q[1], q[2]);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    qsave[QS * r + a] = q[a];
                    wsave[WS * r + a] = w[s][a];
                    if constexpr (Prec::kDisp) qsave[QS * r + 4 + a] = cmp[s][a];
                }
            }
        }
    }
    if (tid == 0) {
        record(A, S, n, rho, ke, status, pg);
        launch_done(A, S, n0, drained);
    }
}

// Workgroup groups.  A problem too slow for one compute unit (a large
// network, or the last networks of a batch still running) is shared by G
// workgroups of a cooperative launch, co-resident by construction.  The
// group works as one virtual workgroup of G * BLOCK threads: member m owns
// the nodes i * G * BLOCK + m * BLOCK + tid, i.e. the same node -> row ->
// wave layout as one workgroup of G * BLOCK threads, so every node's
// arithmetic is the same as in the other kernels.  Once per pass the
// members meet at a barrier in device memory: thread 0 of each posts its
// workgroup's partial sums, releases its writes (agent scope), counts itself
// in and waits for the other members, then acquires; every thread then sums
// the G partials in member order (the same lanes and order in every wave of
// every member, so all take the same stop decision).  The wait is bounded:
// a member that waits longer than kGroupTimeoutTicks marks the group
// aborted and every member leaves its loop, so every kernel ends.  Release
// and acquire are at agent scope (on this chip an L2 write-back before the
// arrival and an L2 invalidate after the wait).
struct GroupCtx {
    uint32_t *bar;  // arrival counter of the group (0 at the launch)
    int32_t *abort; // nonzero once a member's wait timed out
    double *part;   // [2][kGroupMax][4] partial sums by barrier parity and member
    int G, member;
    uint32_t nbar;  // group barriers passed in this launch
};

// 2 s of the 100 MHz wall clock.
constexpr uint64_t kGroupTimeoutTicks = 200000000ull;

// Barrier of the group's members; false when the group was aborted.  Every
// thread calls it; flag is an LDS word of the workgroup.
__device__ __forceinline__ bool group_barrier(GroupCtx &gc, int *flag)
{
    __syncthreads(); // the workgroup's writes of this phase are done
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(gc.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = (gc.nbar + 1u) * (uint32_t)gc.G;
        int ok = 1;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(gc.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(gc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            if (wall_clock64() - t0 > kGroupTimeoutTicks) {
                __hip_atomic_store(gc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag = ok;
    }
    __syncthreads();
    ++gc.nbar;
    return *flag != 0;
}

// A value another member posted before the last group barrier.
__device__ __forceinline__ double group_load(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums K <= 4 workgroup totals (equal in every thread of a member) over the
// group's members in member order; every thread of every member gets the
// same bits.  Returns false when the group was aborted.
template <int K>
__device__ __forceinline__ bool group_sum(GroupCtx &gc, int *flag, int lane, double (&v)[K])
{
    static_assert(K <= 4, "at most 4 sums per barrier");
    double *mine = gc.part + ((gc.nbar & 1u) * kGroupMax + gc.member) * 4;
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) mine[k] = v[k];
    const bool ok = group_barrier(gc, flag);
    const double *all = gc.part + ((gc.nbar - 1u) & 1u) * kGroupMax * 4;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // member m's value in lane m (G <= 16: one 16-lane row), zeros elsewhere
        double t = 0.0;
        if (lane < gc.G) t = group_load(all + lane * 4 + k);
        v[k] = lane0(row_sum(t));
    }
    return ok;
}

// Whether the nodes r = i VB + base + lane (i >= 0, r < N) of a wave whose
// first node is base include prescribed ones (Nf <= r < N); VB = threads of
// the (virtual) workgroup.
__device__ __forceinline__ bool wave_has_prescribed_vb(int base, int VB, int Nf, int N)
{
    int i = Nf - base - (kWave - 1); // first i whose 64 nodes reach Nf
    i = i <= 0 ? 0 : (i + VB - 1) / VB;
    return Nf < N && i * VB + base <= N - 1;
}

// ---------------------------------------------------------------------------
// Global-placement variant: state and half-step velocities in device memory
// (L2-resident for one problem), any problem size.
//
// The gather of a pass walks each wave's rows as one stream of chunks of C
// incidences in a two-stage software pipeline: while chunk c is formed, the
// neighbour states of chunk c+1 and the topology of chunk c+2 are in
// flight, and a row's own node data (state, degree, mass, velocity) is
// loaded when its first chunk enters the pipeline.  The slice headers of
// the workgroup's rows sit in LDS.
//
// GRP = false: one workgroup per slot (blockIdx).  GRP = true: G workgroups
// per problem (A.group), the problems taken from the tail list that the
// preceding launch of the batch filled (A.tail_list / A.tail_count); the
// members of one group are blockIdx values of one residue modulo 8, i.e.
// one XCD (workgroups are dealt to the 8 XCDs round robin), so they share
// that XCD's L2.
// ---------------------------------------------------------------------------
// A node's data for the force phase.
template <class T> struct NodeData {
    T q[3];
    T c[3]; // compensation terms of the FP32 state (zero in FP64)
    T w[3];
    T im;
    double m;
};

template <class Prec, int BLOCK, int C, bool GRP = false>
__global__ void __launch_bounds__(BLOCK) k_dr_glb(SolveArgs A)
{
    using T = typename Prec::T;
    extern __shared__ double smem[];
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = wave_id(tid);
    // The FP64 1024-thread build stages tiles: the staged records first
    // (kTile + the batch's largest halo, 24 bytes each), then the reduction
    // records, a flag word for the group barrier and the slice headers.
    constexpr bool kTileBuild = Prec::kDisp == false && sizeof(T) == 8 && BLOCK == kTile && C == 1;
    const int toff = kTileBuild && A.tile_hmax > 0 ? 3 * (kTile + A.tile_hmax) : 0;
    double *const tq = smem;
    double *red = smem + toff;
    int *gflag = reinterpret_cast<int *>(smem + toff + NW * kRedStride);
    RowHdr *hdr_lds = reinterpret_cast<RowHdr *>(smem + toff + NW * kRedStride + 2);
    GroupCtx gc{nullptr, nullptr, nullptr, 1, 0, 0u};
    Slot S;
    if constexpr (GRP) {
        const int b = blockIdx.x, G = A.group;
        const int g = ((b >> 3) / G) * 8 + (b & 7);
        if (g >= *A.tail_count) return; // uniform per workgroup
        gc.G = G;
        gc.member = (b >> 3) % G;
        gc.bar = A.gbar + g;
        gc.abort = A.gabort + g;
        gc.part = A.gpart + (int64_t)g * 2 * kGroupMax * 4;
        // a drained solve resumes from its saved state
        S.slot = -1;
        S.p = A.tail_list[g];
        S.P = A.probs[S.p];
        S.sb = A.state_off[S.p];
        S.start = kResume;
#pragma unroll
        for (int k = 0; k < 9; ++k) S.F[k] = A.F_cur[9 * (int64_t)S.p + k];
    } else {
        S = load_slot(A, A.order ? A.order[blockIdx.x] : (int)blockIdx.x);
    }
    // a resume of a solve that is not running is a no-op (uniform per workgroup)
    if (S.start == kResume && A.status[S.p] != kStatusRunning) {
        if (tid == 0 && gc.member == 0) launch_done(A, S, 0, false);
        return;
    }
    const Aff32 af = make_aff32(S.F);
    const ProbDesc &P = S.P;
    const int N = P.N, Nf = P.N_free;
    const int64_t nb = P.node_base;
    constexpr int QS = kQStride<T>;
    // virtual workgroup: G members of BLOCK threads; this thread's virtual
    // index and its wave's first node
    const int VB = gc.G * BLOCK;
    const int vt = gc.member * BLOCK + tid;
    const int vbase = (gc.member * NW + wave) * kWave;
    // Two state buffers: the state after pass k lives in buffer k & 1, so a
    // pass can write each node's next state as soon as its velocity is known
    // while the other waves still read this pass's state (no separate
    // displacement sweep, one barrier per pass).  A record holds the FP64
    // position, or the FP32 state and, at +4, its compensation terms.
    T *const qbase = reinterpret_cast<T *>(A.qbuf) + QS * S.sb;
    const int64_t qhalf = A.qhalf * (int64_t)(sizeof(double) / sizeof(T));
    auto qbuf_of = [&](int64_t k) { return qbase + (k & 1) * qhalf; };
    GlbQ<T> pos{qbase}; // the state this pass reads
    constexpr int WS = kWStride<T>;
    T *W = reinterpret_cast<T *>(A.wbuf) + WS * S.sb;
    const T dt = (T)P.dt, hdt = (T)(0.5 * P.dt), cdamp = (T)P.c;
    using KLT = typename KLof<Prec>::type;
    bool alive = true; // false once the group was aborted

    // headers of this workgroup's slices: row i of wave w is slice
    // (i * G + member) * NW + w (the host admits at most kGlbHdrMax slices
    // per problem and sizes the LDS for them)
    {
        const int rows = (P.n_slices + gc.G * NW - 1) / (gc.G * NW);
        for (int t = tid; t < rows * NW; t += BLOCK) {
            const int q = ((t / NW) * gc.G + gc.member) * NW + t % NW;
            hdr_lds[t] = q < P.n_slices ? RowHdr{(uint32_t)A.slice_off[P.slice_base + q],
                                                 A.slice_w[P.slice_base + q]}
                                        : RowHdr{0, 0};
        }
    }
    const Topo<Prec> tpg = topo_of<Prec>(A, P);
    // rows of this wave: i = 0 .. nrow-1 (node i * VB + vt)
    const int nrow = N > vbase ? (N - vbase + VB - 1) / VB : 0;
    auto hdr_of = [&](int i) -> RowHdr { return uniform_hdr(hdr_lds + i * NW + wave); };
    // stream cursor: row i, first incidence k0 of the chunk, row width w;
    // i >= nrow = end of the stream
    struct Cur {
        int i, k0, w;
    };
    auto first_from = [&](int i) -> Cur {
        int w = 0;
        while (i < nrow && (w = hdr_of(i).w) == 0) ++i;
        return Cur{i, 0, w};
    };
    auto next = [&](Cur c) -> Cur {
        if (c.i >= nrow) return c;
        if (c.k0 + C < c.w) return Cur{c.i, c.k0 + C, c.w};
        return first_from(c.i + 1);
    };
    auto topo = [&](Cur c, Cur dummy, Pref<Prec, C> &pf) {
        const Cur x = c.i < nrow ? c : dummy;
        pref_load<Prec, C>(tpg, hdr_of(x.i), x.k0, lane, pf);
    };
    auto node_data = [&](int i, NodeData<T> &nd) {
        const int r = i * VB + vt;
        nd.q[0] = nd.q[1] = nd.q[2] = 0;
        nd.c[0] = nd.c[1] = nd.c[2] = 0;
        nd.w[0] = nd.w[1] = nd.w[2] = 0;
        nd.im = 0;
        nd.m = 0.0;
        if (r < N) {
            pos.load(r, nd.q[0], nd.q[1], nd.q[2]);
            if constexpr (Prec::kDisp)
                if (r < Nf)
#pragma unroll
                    for (int a = 0; a < 3; ++a) nd.c[a] = node_rec<QS>(pos.base + 4, r)[a];
            if (r < Nf) {
                node_mass<Prec>(A, nb, r, nd.im, nd.m);
#pragma unroll
                for (int a = 0; a < 3; ++a) nd.w[a] = node_rec<WS>(W, r)[a];
            }
        }
    };
    // sums over the problem: the workgroup's (block_sum4, equal in all
    // threads), then over the group's members
    auto problem_sum4 = [&](double (&v)[4]) {
        block_sum4<NW>(red, lane, wave, v);
        if constexpr (GRP) alive = group_sum<4>(gc, gflag, lane, v) && alive;
    };

    int64_t n = 0;
    if (S.start != kResume) {
        for (int r = vt; r < N; r += VB) {
            T q[3];
            start_q<Prec>(A, S, r, q);
            pos.store(r, q[0], q[1], q[2]); // buffer 0: the state after pass 0
            if constexpr (Prec::kDisp)
                for (int a = 0; a < 3; ++a) node_rec<QS>(qbase + 4, r)[a] = 0;
        }
        if (tid == 0 && gc.member == 0) begin_solve(A, S);
        if constexpr (GRP) alive = group_barrier(gc, gflag);
        else __syncthreads();
        for (int r = vt; r < Nf; r += VB) {
            T qi[3], g[3];
            pos.load(r, qi[0], qi[1], qi[2]);
            gather<Prec, 4>(A, af, node_row(A, P, r), pos, lane, A.deg[nb + r], qi[0], qi[1], qi[2], g[0],
                         g[1], g[2]);
            const T im = Prec::kDisp ? (T)A.invm32[nb + r] : (T)A.invm[nb + r];
            T wn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) node_rec<WS>(W, r)[a] = wn[a] = hdt * (g[a] * im);
            if (A.energy_tol > 0.0) {
                // the record starts afresh: w_old = 0
                const double gw = (double)g[0] * (double)wn[0] + (double)g[1] * (double)wn[1] +
                                  (double)g[2] * (double)wn[2];
                double *e = A.enode + 4 * (nb + r);
                e[0] = gw;
                e[1] = 0.0;
                e[2] = gw;
            }
        }
    } else {
        n = A.iters[S.p];
    }
    __syncthreads();

    const int64_t n0 = n;
    // passes this launch may make: the budget counts from the first launch
    // of the batch call (a drained solve continues within the same budget)
    const int64_t nlim = (GRP ? A.n_begin[S.p] : n0) + launch_budget(A, S.p);
    const double tol2 = A.tol * A.tol;
    double rho = 0.0, ke = 0.0, gf2 = 0.0, gb2 = 0.0, ke2 = 0.0;
    int status = kStatusRunning;
    bool drained = false;
    Progress pg{__builtin_huge_val(), n};
    const bool has_free = vbase < Nf, has_pres = wave_has_prescribed_vb(vbase, VB, Nf, N);
    if (S.start == kResume) {
        pg.best = A.rho_best[S.p];
        pg.nbest = A.n_best[S.p];
    }
    // The first displacement update of this launch, from the state after
    // pass k (buffer k & 1) into buffer (k + 1) & 1; prescribed nodes are
    // copied, so that both buffers hold them.  Later passes update their
    // nodes' states as they finish them.
    auto advance_from = [&](int64_t k) {
        const GlbQ<T> src{qbuf_of(k)}, dst{qbuf_of(k + 1)};
        for (int r = vt; r < N; r += VB) {
            T q[3], c[3] = {0, 0, 0};
            src.load(r, q[0], q[1], q[2]);
            if constexpr (Prec::kDisp)
                for (int a = 0; a < 3; ++a) c[a] = node_rec<QS>(src.base + 4, r)[a];
            if (r < Nf)
#pragma unroll
                for (int a = 0; a < 3; ++a) advance_q(q[a], dt, node_rec<WS>(W, r)[a], c[a]);
            dst.store(r, q[0], q[1], q[2]);
            if constexpr (Prec::kDisp)
                for (int a = 0; a < 3; ++a) node_rec<QS>(dst.base + 4, r)[a] = c[a];
        }
    };
    advance_from(n);
    if constexpr (GRP) alive = group_barrier(gc, gflag) && alive;
    else __syncthreads();
    while (alive) {
        // pass n + 1 reads the state after pass n + 1's displacement update
        // (buffer (n + 1) & 1) and writes the next one into buffer n & 1;
        // the reduction slots alternate with the pass as well (one barrier
        // per pass separates a pass's reads from the next pass's writes)
        pos.base = qbuf_of(n + 1);
        const GlbQ<T> qnext{qbuf_of(n)};
        const int rslot = 2 * (int)(n & 1);
        gf2 = 0.0; gb2 = 0.0; ke2 = 0.0;
        const Cur cfirst = first_from(0);
        bool staged = false;
        if constexpr (kTileBuild) staged = P.n_tiles > 0;
        if constexpr (kTileBuild) if (staged) {
            // Staged gather: row i of this wave is tile i G + member (nodes
            // t kTile + tid).  The tile's records and its halo are copied into LDS, the
            // incidences name their neighbour's slot there; each node's
            // arithmetic is that of the streamed gather below.
            const int32_t *toffs = A.tile_halo + P.tile_base;
            const int32_t *hids = A.halo_ids + P.halo_base;
            const uint16_t *ls = A.lslot + P.inc_base;
            const KL *klp = A.kl + P.inc_base;
            const LdsQ<double> tpos{reinterpret_cast<double *>(tq), 0};
            // row i of the (virtual) workgroup is tile i G + member
            const int nit = (P.n_tiles + gc.G - 1) / gc.G;
            for (int i = 0; i < nit; ++i) {
                const int t = i * gc.G + gc.member;
                const int lo = t * kTile;
                const int h0 = t < P.n_tiles ? toffs[t] : 0;
                const int ns = t < P.n_tiles ? kTile + toffs[t + 1] - h0 : 0;
                for (int s = tid; s < ns; s += BLOCK) {
                    const int j = s < kTile ? lo + s : hids[h0 + s - kTile];
                    if (j < N) {
                        double x, y, z;
                        pos.load(j, x, y, z);
                        tpos.store(s, x, y, z);
                    }
                }
                __syncthreads();
                if (i < nrow) {
                    const RowHdr h = hdr_of(i);
                    const int r = lo + tid;
                    if (h.w > 0 && r < N) {
                        // the node's state from the staged tile, its velocity and mass
                        NodeData<T> nd;
                        tpos.load(tid, nd.q[0], nd.q[1], nd.q[2]);
                        nd.im = 0;
                        nd.m = 0.0;
                        nd.w[0] = nd.w[1] = nd.w[2] = 0;
                        if (r < Nf) {
                            node_mass<Prec>(A, nb, r, nd.im, nd.m);
#pragma unroll
                            for (int a = 0; a < 3; ++a) nd.w[a] = node_rec<WS>(W, r)[a];
                        }
                        double g[3] = {0.0, 0.0, 0.0};
                        int64_t e = (int64_t)h.off + lane;
                        int s0 = ls[e];
                        KL c0 = klp[e];
                        for (int k = 0; k < h.w; ++k, e += kWave) {
                            int s1 = 0;
                            KL c1{0.0, 0.0};
                            if (k + 1 < h.w) {
                                s1 = ls[e + kWave];
                                c1 = klp[e + kWave];
                            }
                            KL cc[1] = {c0};
                            double px[1], py[1], pz[1];
                            tpos.load(s0, px[0], py[0], pz[0]);
                            force_pre<1>(cc, px, py, pz, af, 1, nd.q[0], nd.q[1], nd.q[2], g[0], g[1], g[2]);
                            s0 = s1;
                            c0 = c1;
                        }
                        // the node's damped acceleration, velocity updates and norm shares
                        const double gg = sq3(g[0], g[1], g[2]);
                        if (r < Nf) {
                            if (A.energy_tol > 0.0)
                                energy_pass<T>(A, nb + r, g, nd.w, nd.im, cdamp, hdt, nd.m);
                            double vv = 0.0;
                            T qn[3];
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                T wa = nd.w[a];
                                const T v = vel_step(g[a], nd.im, cdamp, hdt, wa);
                                vv = fma((double)v, (double)v, vv);
                                node_rec<WS>(W, r)[a] = wa;
                                qn[a] = nd.q[a];
                                T cn = 0;
                                advance_q(qn[a], dt, wa, cn);
                            }
                            qnext.store(r, qn[0], qn[1], qn[2]);
                            gf2 += gg;
                            ke2 = fma(nd.m, vv, ke2);
                        } else {
                            gb2 += gg;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (!staged && cfirst.i < nrow) {
            // prologue: topology and neighbour states of chunk c0, topology of c1
            Cur c0 = cfirst;
            Pref<Prec, C> t0, t1;
            topo(c0, cfirst, t0);
            Cur c1 = next(c0);
            topo(c1, cfirst, t1);
            NodeData<T> n0, n1;
            node_data(c0.i, n0);
            KLT k0c[C];
            T px0[C], py0[C], pz0[C];
#pragma unroll
            for (int t = 0; t < C; ++t) {
                pos.load(t0.j[t], px0[t], py0[t], pz0[t]);
                k0c[t] = t0.c[t];
            }
            T g[3] = {0, 0, 0};
            for (;;) {
                // stage 1: neighbour states (and new row's node data) of c1
                KLT k1c[C];
                T px1[C], py1[C], pz1[C];
#pragma unroll
                for (int t = 0; t < C; ++t) {
                    pos.load(t1.j[t], px1[t], py1[t], pz1[t]);
                    k1c[t] = t1.c[t];
                }
                const bool c1_valid = c1.i < nrow;
                const bool c1_new_row = c1_valid && c1.i != c0.i;
                if (c1_new_row) node_data(c1.i, n1);
                // stage 2: topology of c2
                const Cur c2 = next(c1);
                topo(c2, cfirst, t1);
                // stage 3: forces of c0
                force_pre<C>(k0c, px0, py0, pz0, af, c0.w - c0.k0, n0.q[0], n0.q[1], n0.q[2], g[0],
                             g[1], g[2]);
                if (!c1_valid || c1_new_row) {
                    // c0 was the last chunk of its row: the node's damped
                    // acceleration, velocity updates and norm shares
                    const int r = c0.i * VB + vt;
                    if (r < N) {
                        const double gg = sq3((double)g[0], (double)g[1], (double)g[2]);
                        if (r < Nf) {
                            if (A.energy_tol > 0.0)
                                energy_pass<T>(A, nb + r, g, n0.w, n0.im, cdamp, hdt, n0.m);
                            double vv = 0.0;
                            T qn[3], cn[3];
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                T wa = n0.w[a];
                                const T v = vel_step(g[a], n0.im, cdamp, hdt, wa);
                                vv = fma((double)v, (double)v, vv);
                                node_rec<WS>(W, r)[a] = wa;
                                // the displacement update of the next pass
                                qn[a] = n0.q[a];
                                cn[a] = n0.c[a];
                                advance_q(qn[a], dt, wa, cn[a]);
                            }
                            qnext.store(r, qn[0], qn[1], qn[2]);
                            if constexpr (Prec::kDisp)
#pragma unroll
                                for (int a = 0; a < 3; ++a) node_rec<QS>(qnext.base + 4, r)[a] = cn[a];
                            gf2 += gg;
                            ke2 = fma(n0.m, vv, ke2);
                        } else {
                            gb2 += gg;
                        }
                    }
                    g[0] = g[1] = g[2] = 0;
                    if (!c1_valid) break;
                    n0 = n1;
                }
                c0 = c1;
                c1 = c2;
#pragma unroll
                for (int t = 0; t < C; ++t) {
                    k0c[t] = k1c[t];
                    px0[t] = px1[t]; py0[t] = py1[t]; pz0[t] = pz1[t];
                }
            }
        }
        wave_partials2<NW>(red, lane, wave, gf2, gb2, has_free, has_pres, rslot);
        // every kDrainEvery passes thread 0 reads how many problems of the
        // launch are still running; all threads read its decision after the
        // barrier
        const bool drain_pass = !GRP && A.tail_at > 0 && ((n + 1) & (kDrainEvery - 1)) == 0;
        if (drain_pass && tid == 0)
            red[kDrainSlotGlb] = __hip_atomic_load(A.live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <=
                                         A.tail_at ? 1.0 : 0.0;
        __syncthreads();
        block_totals2<NW>(red, lane, gf2, gb2, rslot);
        const bool drain_now = drain_pass && red[kDrainSlotGlb] != 0.0;
        if constexpr (GRP) {
            double v[2] = {gf2, gb2};
            if (!group_sum<2>(gc, gflag, lane, v)) { alive = false; break; }
            gf2 = v[0]; gb2 = v[1];
        }
        ++n;
        if (stop_test(A, P, tol2, gf2, gb2, n, status, pg)) break;
        if (A.energy_tol > 0.0 && n % kEnergyEvery == 0) {
            double e[4] = {0.0, 0.0, 0.0, ke2};
            energy_sum_glb(A, nb, Nf, vt, VB, e);
            problem_sum4(e);
            __syncthreads(); // its slots are read before the next pass writes any
            if (!alive) break;
            double Wk, D;
            energy_totals(P, e, false, Wk, D);
            if (!energy_ok(A.energy_tol, 0.5 * e[3], Wk, D)) {
                status = kStatusEnergy;
                break;
            }
        }
        if (drain_now) {
            drained = true; // the rest of this solve runs in a group launch
            break;
        }
        if (n >= nlim) break;
    }
    if (!alive) status = kStatusAborted;
    pos.base = qbuf_of(n); // the state after the last pass
    // kinetic energy of the last pass (reported only)
    if (alive) {
        double k4[4] = {ke2, 0.0, 0.0, 0.0};
        problem_sum4(k4);
        ke2 = k4[0];
    }
    final_scalars(P, gf2, gb2, ke2, rho, ke);
    if (A.energy_tol > 0.0 && alive) {
        double e[4] = {0.0, 0.0, 0.0, 0.0};
        energy_sum_glb(A, nb, Nf, vt, VB, e);
        problem_sum4(e);
        double Wk, D;
        energy_totals(P, e, status != kStatusRunning, Wk, D);
        if (status != kStatusRunning && status != kStatusEnergy && status != kNonFinite &&
            !energy_ok(A.energy_tol, ke, Wk, D))
            status = kStatusEnergy;
        if (tid == 0 && gc.member == 0) {
            A.e_work[S.p] = Wk;
            A.e_damp[S.p] = D;
        }
    }

    if (status != kStatusRunning && status != kStatusAborted) {
        for (int r = vt; r < N; r += VB) {
            T q[3];
            pos.load(r, q[0], q[1], q[2]);
            write_u<Prec>(A, S, r, q);
        }
    }
    if (tid == 0 && gc.member == 0) {
        record(A, S, n, rho, ke, status, pg);
        launch_done(A, S, n0, drained);
    }
}


// ---------------------------------------------------------------------------
// Launch helpers shared by the translation units that instantiate kernels
// ---------------------------------------------------------------------------
template <class K>
static inline int launch(K kernel, int grid, int block, int lds, hipStream_t st, const SolveArgs &a)
{
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, st, a);
    return (int)hipGetLastError();
}

// Register/LDS-resident launches, one translation unit per precision and
// workgroup size (dr_k_reg_*.hip), and the global-placement launches, one
// per precision (dr_k_glb_*.hip).
int launch_reg_p64_256(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);
int launch_reg_p64_512(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);
int launch_reg_p64_1024(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);
int launch_reg_p32_256(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);
int launch_reg_p32_512(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);
int launch_reg_p32_1024(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);
int launch_glb_p64(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);
int launch_glb_p32(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st);

// Instantiates k_dr_reg<P, B, NPT, CH> for NPT 1..8 and CH 1, 2, 4.
template <class P, int B, int NP>
static inline int launch_reg_np(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    if (pl.chunk == 4) return launch(k_dr_reg<P, B, NP, 4>, a.n_solve, B, pl.lds_bytes, st, a);
    if (pl.chunk == 1) return launch(k_dr_reg<P, B, NP, 1>, a.n_solve, B, pl.lds_bytes, st, a);
    return launch(k_dr_reg<P, B, NP, 2>, a.n_solve, B, pl.lds_bytes, st, a);
}

template <class P, int B>
static inline int launch_reg(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    switch (pl.npt) {
    case 1: return launch_reg_np<P, B, 1>(a, pl, st);
    case 2: return launch_reg_np<P, B, 2>(a, pl, st);
    case 3: return launch_reg_np<P, B, 3>(a, pl, st);
    case 4: return launch_reg_np<P, B, 4>(a, pl, st);
    case 5: return launch_reg_np<P, B, 5>(a, pl, st);
    case 6: return launch_reg_np<P, B, 6>(a, pl, st);
    case 7: return launch_reg_np<P, B, 7>(a, pl, st);
    case 8: return launch_reg_np<P, B, 8>(a, pl, st);
    default: return -1000;
    }
}

// The 256-thread global variant is built with chunks of 1 only: its chunk-2
// and chunk-4 builds gave wrong states on multi-row problems while every
// other shape matched bit for bit (the host rejects those plans).
template <class P, int B>
static inline int launch_glb(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    if constexpr (B == 256) {
        if (pl.chunk != 1) return -1002;
        return launch(k_dr_glb<P, B, 1>, a.n_solve, B, pl.lds_bytes, st, a);
    } else {
        if (pl.chunk == 4) return launch(k_dr_glb<P, B, 4>, a.n_solve, B, pl.lds_bytes, st, a);
        if (pl.chunk == 1) return launch(k_dr_glb<P, B, 1>, a.n_solve, B, pl.lds_bytes, st, a);
        return launch(k_dr_glb<P, B, 2>, a.n_solve, B, pl.lds_bytes, st, a);
    }
}

// The group form of the global kernel, as a cooperative launch (the runtime
// refuses a grid whose workgroups cannot all be resident at once).
template <class P, int B, int C>
static inline int launch_group(const SolveArgs &a, const LaunchPlan &pl, int grid, hipStream_t st)
{
    const void *k = reinterpret_cast<const void *>(k_dr_glb<P, B, C, true>);
    if (pl.lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, pl.lds_bytes);
        if (e != hipSuccess) return (int)e;
    }
    SolveArgs arg = a;
    void *args[] = {&arg};
    hipError_t e = hipLaunchCooperativeKernel(k, dim3(grid), dim3(B), args, (unsigned)pl.lds_bytes, st);
    if (e != hipSuccess) return (int)e;
    return (int)hipGetLastError();
}

template <class P, int B, int C>
static inline int group_occupancy(int lds_bytes, int *blocks_per_cu)
{
    const void *k = reinterpret_cast<const void *>(k_dr_glb<P, B, C, true>);
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return (int)e;
    }
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, B, (size_t)lds_bytes);
}

int launch_group_p64(const SolveArgs &a, const LaunchPlan &pl, int grid, hipStream_t st);
int launch_group_p32(const SolveArgs &a, const LaunchPlan &pl, int grid, hipStream_t st);
int group_capacity_p64(int block, int lds_bytes, int *blocks_per_cu);
int group_capacity_p32(int block, int lds_bytes, int *blocks_per_cu);

template <class P>
static inline int launch_glb_all(const SolveArgs &a, const LaunchPlan &pl, hipStream_t st)
{
    switch (pl.block) {
    case 256: return launch_glb<P, 256>(a, pl, st);
    case 512: return launch_glb<P, 512>(a, pl, st);
    case 1024: return launch_glb<P, 1024>(a, pl, st);
    default: return -1001;
    }
}

} // namespace drk
