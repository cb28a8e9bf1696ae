/*
 * Plain, slow, FP64 CPU oracle for dynamic relaxation (DR) of one
 * pin-jointed fiber network.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  The
 * product path never calls it and shares no code, header, table or helper
 * with it.
 *
 * What it computes (Merson & Shephard, "Using Hierarchical Parallelism to
 * Accelerate the Solution of Many Small Partial Differential Equations"):
 *   - section II: the microscale sub-problem is a static equilibrium of an
 *     athermal fiber network, reached by dynamic relaxation, i.e. a damped
 *     explicit pseudo-dynamics whose force residual is monitored;
 *   - section III, Fig. 1 ("Dynamic relaxation algorithm"): the set-up
 *     (boundary conditions, lumped mass, initial internal force and
 *     acceleration) and the loop (time step, half velocity update,
 *     displacement update, internal forces, damping force, force residual,
 *     acceleration, second half velocity update, energy, iteration count,
 *     until the residual has converged), taken in that order;
 *   - section I: the sub-problem returns constitutive information to the
 *     macroscale, here the volume-averaged Cauchy stress.
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes of the repository):
 *   R1 fiber law: axial force T = EA (lambda^2 - 1) / 2, lambda = l / L,
 *      acting along the current fiber direction, in tension and compression.
 *   R2 lumped mass: m_i = 1/2 sum_{f at i} L_f (unit mass per length).
 *   R3 time step: constant per solve, dt = s * 2 / w, with
 *      w^2 = max over free nodes i of (2 / m_i) sum_{f at i} 1.1 EA_f / L_f
 *      (a Gershgorin bound on M^-1 K with 10 % stretch headroom);
 *      "compute next time step" is then t <- t + dt.
 *   R4 damping force: f_d = -c m v with c = beta * w (mass proportional).
 *   R5 start: u_B = (F - I) X_B on prescribed nodes; free nodes start from
 *      the affine field (F - I) X (default), from zero, or warm from a
 *      previous solution u_prev + (F - F_prev) X; v = 0, n = 0, t = 0.
 *   R6 residual: rho = |g_free| / max(|g_B|, s_floor), 2-norms of the
 *      internal force on free and on prescribed degrees of freedom (the
 *      damping force excluded), s_floor = 1e-4 mean(EA) sqrt(3 max(N_B,1)).
 *      The loop is repeat-until, so at least one pass is made.
 *   R7 stress: sigma = 1/(J V0) sum_{b prescribed} r_b (x) (x_b - F c0),
 *      r_b = -g_b, J = det F, V0 = 1, c0 = (1/2, 1/2, 1/2), row-major with
 *      sigma_ij = sum r_i y_j.  The fiber form
 *      sigma_fib = 1/(J V0) sum_f T_f d_f (x) d_f / l_f is returned beside it.
 *   R16 "compute next time step" taken literally (optional, dt_rule = 1): at
 *      the top of each pass the pass's step is computed from the current
 *      state, dt_n = min(dt_{n-1}, s * 2 / w(u)), starting from dt_0 = the
 *      constant step of R3, with w(u)^2 = max over free nodes i of
 *      (2 / m_i) sum_{f at i} k_f(u),
 *      k_f = EA l / L^2, the fiber's axial tangent stiffness at its current
 *      length.  (Its transverse, geometric stiffness T / l is smaller in
 *      tension and negative in compression, where it drives buckling, a
 *      growth that no step size removes, so it does not bound the step.)
 *      Both half velocity updates of the pass use the step.  The step never
 *      grows back: a step that follows the stiffness up and down from pass to
 *      pass pumps energy into a violent transient (a parametric excitation)
 *      and made solves diverge that converge with the constant step.
 *      Where the current stiffness stays within R3's headroom every step is
 *      dt0 and the iteration is the constant-step one exactly.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so the
 * rounding follows the source order).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_CONVERGED 0
#define OR_MAX_ITER 1
#define OR_NONFINITE 2
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define OR_START_AFFINE 0
#define OR_START_ZERO 1
#define OR_START_WARM 2

/* Fiber lengths in the reference configuration; -1 if any is not > 0. */
static int fiber_lengths(int M, const int *fib, const double *X, double *L)
{
    for (int f = 0; f < M; ++f) {
        int a = fib[2 * f], b = fib[2 * f + 1];
        double dx = X[3 * b] - X[3 * a];
        double dy = X[3 * b + 1] - X[3 * a + 1];
        double dz = X[3 * b + 2] - X[3 * a + 2];
        L[f] = sqrt(dx * dx + dy * dy + dz * dz);
        if (!(L[f] > 0.0)) return -1;
    }
    return 0;
}

/*
 * getInternalForces (Fig. 1): g_i = sum over fibers f at i of T_f d_f / l_f,
 * with d_f pointing from i to the other end, i.e. the force the fibers exert
 * on node i (minus the gradient of the stored energy).  Evaluated for every
 * node, prescribed ones included.
 */
void oracle_internal_force(int N, const double *X, const double *u, int M,
                           const int *fib, const double *EA, const double *L,
                           double *g)
{
    for (int i = 0; i < 3 * N; ++i) g[i] = 0.0;
    for (int f = 0; f < M; ++f) {
        int a = fib[2 * f], b = fib[2 * f + 1];
        double d[3];
        for (int k = 0; k < 3; ++k)
            d[k] = (X[3 * b + k] + u[3 * b + k]) - (X[3 * a + k] + u[3 * a + k]);
        double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double lam = l / L[f];
        double T = EA[f] * (lam * lam - 1.0) / 2.0;
        for (int k = 0; k < 3; ++k) {
            double fk = T * d[k] / l;
            g[3 * a + k] += fk;
            g[3 * b + k] -= fk;
        }
    }
}

/* Stored energy W = sum_f EA L (lambda^3 - 3 lambda + 2) / 6 (integral of R1). */
double oracle_energy(int N, const double *X, const double *u, int M,
                     const int *fib, const double *EA, const double *L)
{
    (void)N;
    double W = 0.0;
    for (int f = 0; f < M; ++f) {
        int a = fib[2 * f], b = fib[2 * f + 1];
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double dk = (X[3 * b + k] + u[3 * b + k]) - (X[3 * a + k] + u[3 * a + k]);
            d2 += dk * dk;
        }
        double lam = sqrt(d2) / L[f];
        W += EA[f] * L[f] * (lam * lam * lam - 3.0 * lam + 2.0) / 6.0;
    }
    return W;
}

/* Step of R16 at displacement u: min(dt0, s 2 / w(u)) (dt0 when no free
 * node carries stiffness), dt0 the previous pass's step. */
static double step_at(int N, const double *X, const double *u, int M, const int *fib,
                      const double *EA, const double *L, const unsigned char *fixed,
                      const double *m, double dt0, double dt_safety, double *ksum)
{
    for (int i = 0; i < N; ++i) ksum[i] = 0.0;
    for (int f = 0; f < M; ++f) {
        int a = fib[2 * f], b = fib[2 * f + 1];
        double d[3];
        for (int k = 0; k < 3; ++k)
            d[k] = (X[3 * b + k] + u[3 * b + k]) - (X[3 * a + k] + u[3 * a + k]);
        double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double kf = EA[f] * l / (L[f] * L[f]);
        ksum[a] += kf;
        ksum[b] += kf;
    }
    double w2 = 0.0;
    for (int i = 0; i < N; ++i) {
        if (fixed[i]) continue;
        double wi = 2.0 / m[i] * ksum[i];
        if (wi > w2) w2 = wi;
    }
    if (!(w2 > 0.0)) return dt0;
    double dt = dt_safety * 2.0 / sqrt(w2);
    return dt < dt0 ? dt : dt0;
}

static double det3(const double *F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7])
         - F[1] * (F[3] * F[8] - F[5] * F[6])
         + F[2] * (F[3] * F[7] - F[4] * F[6]);
}

/* Derived per-network data: masses (R2), time step and damping (R3, R4),
 * residual floor (R6).  Returns OR_EINVAL on bad input. */
int oracle_derived(int N, const double *X, int M, const int *fib, const double *EA,
                   const unsigned char *fixed, double beta, double dt_safety,
                   double *L, double *m, double *dt, double *c, double *s_floor)
{
    for (int f = 0; f < M; ++f) {
        int a = fib[2 * f], b = fib[2 * f + 1];
        if (a < 0 || b < 0 || a >= N || b >= N || a == b) return OR_EINVAL;
        if (!(EA[f] > 0.0) || !isfinite(EA[f])) return OR_EINVAL;
    }
    for (int i = 0; i < 3 * N; ++i)
        if (!isfinite(X[i])) return OR_EINVAL;
    if (fiber_lengths(M, fib, X, L) != 0) return OR_EINVAL;

    double *ksum = (double *)calloc((size_t)N > 0 ? (size_t)N : 1, sizeof(double));
    if (!ksum) return OR_ENOMEM;
    for (int i = 0; i < N; ++i) m[i] = 0.0;
    for (int f = 0; f < M; ++f) {
        int a = fib[2 * f], b = fib[2 * f + 1];
        m[a] += 0.5 * L[f];
        m[b] += 0.5 * L[f];
        double kh = 1.1 * EA[f] / L[f];
        ksum[a] += kh;
        ksum[b] += kh;
    }
    double w2 = 0.0;
    int n_fixed = 0;
    for (int i = 0; i < N; ++i) {
        if (fixed[i]) { ++n_fixed; continue; }
        if (!(m[i] > 0.0)) { free(ksum); return OR_EINVAL; } /* free node, no fiber */
        double wi = 2.0 / m[i] * ksum[i];
        if (wi > w2) w2 = wi;
    }
    free(ksum);
    double w = sqrt(w2);
    *dt = (w > 0.0) ? dt_safety * 2.0 / w : 0.0;
    *c = beta * w;
    double ea_mean = 0.0;
    for (int f = 0; f < M; ++f) ea_mean += EA[f];
    ea_mean = (M > 0) ? ea_mean / M : 0.0;
    *s_floor = 1e-4 * ea_mean * sqrt(3.0 * (n_fixed > 1 ? n_fixed : 1));
    return 0;
}

/* Volume-averaged Cauchy stress, boundary (R7) and fiber forms. */
static void stress(int N, const double *X, const double *u, int M, const int *fib,
                   const double *EA, const double *L, const unsigned char *fixed,
                   const double *g, const double *F, double *sigma, double *sigma_fib)
{
    double J = det3(F);
    double Fc0[3];
    for (int r = 0; r < 3; ++r) Fc0[r] = 0.5 * (F[3 * r] + F[3 * r + 1] + F[3 * r + 2]);
    for (int k = 0; k < 9; ++k) { sigma[k] = 0.0; sigma_fib[k] = 0.0; }
    for (int i = 0; i < N; ++i) {
        if (!fixed[i]) continue;
        double r[3], y[3];
        for (int k = 0; k < 3; ++k) {
            r[k] = -g[3 * i + k];
            y[k] = X[3 * i + k] + u[3 * i + k] - Fc0[k];
        }
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) sigma[3 * p + q] += r[p] * y[q];
    }
    for (int f = 0; f < M; ++f) {
        int a = fib[2 * f], b = fib[2 * f + 1];
        double d[3];
        for (int k = 0; k < 3; ++k)
            d[k] = (X[3 * b + k] + u[3 * b + k]) - (X[3 * a + k] + u[3 * a + k]);
        double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double lam = l / L[f];
        double T = EA[f] * (lam * lam - 1.0) / 2.0;
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) sigma_fib[3 * p + q] += T * d[p] * d[q] / l;
    }
    for (int k = 0; k < 9; ++k) { sigma[k] /= J; sigma_fib[k] /= J; }
}

/*
 * The residual and the stress of a given state (R6, R7): rho of the
 * displacement u[3N] (prescribed nodes included as given) and both stress
 * forms under F.  Returns 0, or a negative error.  This evaluates the
 * definitions the solve stops on and returns; it does not iterate.
 */
int oracle_evaluate(int N, const double *X, const double *u, int M, const int *fib,
                    const double *EA, const unsigned char *fixed, const double *F,
                    double *rho_out, double *sigma, double *sigma_fib)
{
    if (N < 1 || M < 0) return OR_EINVAL;
    double *L = (double *)malloc(((size_t)M > 0 ? (size_t)M : 1) * sizeof(double));
    double *m = (double *)malloc((size_t)N * sizeof(double));
    double *g = (double *)calloc(3 * (size_t)N, sizeof(double));
    if (!L || !m || !g) {
        free(L); free(m); free(g);
        return OR_ENOMEM;
    }
    double dt, c, s_floor;
    int rc = oracle_derived(N, X, M, fib, EA, fixed, 0.0, 1.0, L, m, &dt, &c, &s_floor);
    if (rc == 0) {
        oracle_internal_force(N, X, u, M, fib, EA, L, g);
        double gf2 = 0.0, gb2 = 0.0;
        for (int i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) {
                double gk = g[3 * i + k];
                if (fixed[i]) gb2 += gk * gk; else gf2 += gk * gk;
            }
        double den = sqrt(gb2);
        if (den < s_floor) den = s_floor;
        *rho_out = sqrt(gf2) / den;
        stress(N, X, u, M, fib, EA, L, fixed, g, F, sigma, sigma_fib);
    }
    free(L); free(m); free(g);
    return rc;
}

/*
 * One dynamic-relaxation solve (Fig. 1).
 *
 * Inputs: N nodes with reference coordinates X[3N] (xyz interleaved), M
 * fibers fib[2M] (node ids), EA[M] > 0, fixed[N] (1 = prescribed), F[9]
 * row-major.  start_mode: OR_START_AFFINE / OR_START_ZERO / OR_START_WARM
 * (the last uses F_prev[9] and u_prev[3N]).
 * Outputs: u[3N], sigma[9], sigma_fib[9], iteration count, final residual,
 * kinetic energy, and the dt / c that were used.  Optional trace: when
 * rho_trace is not NULL, the residual of pass n is stored at rho_trace[n-1]
 * for n <= trace_len.  dt_rule: 0 = the constant step of R3, 1 = the
 * per-pass step of R16.  work_out (optional): the internal and damping work,
 * then the smallest step used.
 * Returns OR_CONVERGED / OR_MAX_ITER / OR_NONFINITE, or a negative error.
 */
int oracle_solve(int N, const double *X, int M, const int *fib, const double *EA,
                 const unsigned char *fixed, const double *F,
                 int start_mode, const double *F_prev, const double *u_prev,
                 double tol, long max_iter, double beta, double dt_safety,
                 double *u, double *sigma, double *sigma_fib, long *iters,
                 double *rho_out, double *ke_out, double *dt_out, double *c_out,
                 double *rho_trace, long trace_len, double *work_out, int dt_rule)
{
    if (N < 1 || M < 0 || max_iter < 1) return OR_EINVAL;
    size_t n3 = 3 * (size_t)N;
    double *L = (double *)malloc(((size_t)M > 0 ? (size_t)M : 1) * sizeof(double));
    double *m = (double *)malloc((size_t)N * sizeof(double));
    double *v = (double *)calloc(n3, sizeof(double));
    double *a = (double *)calloc(n3, sizeof(double));
    double *g = (double *)calloc(n3, sizeof(double));
    double *g_prev = (double *)calloc(n3, sizeof(double));
    double *ksum = (double *)calloc((size_t)N, sizeof(double));
    if (!L || !m || !v || !a || !g || !g_prev || !ksum) {
        free(L); free(m); free(v); free(a); free(g); free(g_prev); free(ksum);
        return OR_ENOMEM;
    }
    double dt0, c, s_floor;
    int rc = oracle_derived(N, X, M, fib, EA, fixed, beta, dt_safety, L, m, &dt0, &c, &s_floor);
    if (rc != 0) {
        free(L); free(m); free(v); free(a); free(g); free(g_prev); free(ksum);
        return rc;
    }
    double dt = dt0, dt_min = dt0;

    /* Set displacement boundary conditions and the start state (R5). */
    for (int i = 0; i < N; ++i) {
        for (int r = 0; r < 3; ++r) {
            double FmI_X = 0.0;   /* ((F - I) X_i)_r */
            double dF_X = 0.0;    /* ((F - F_prev) X_i)_r */
            for (int s = 0; s < 3; ++s) {
                double Frs = F[3 * r + s] - (r == s ? 1.0 : 0.0);
                FmI_X += Frs * X[3 * i + s];
                if (start_mode == OR_START_WARM)
                    dF_X += (F[3 * r + s] - F_prev[3 * r + s]) * X[3 * i + s];
            }
            if (fixed[i] || start_mode == OR_START_AFFINE)
                u[3 * i + r] = FmI_X;
            else if (start_mode == OR_START_ZERO)
                u[3 * i + r] = 0.0;
            else
                u[3 * i + r] = u_prev[3 * i + r] + dF_X;
        }
    }

    /* Initial internal force and acceleration (v = 0: no damping yet). */
    oracle_internal_force(N, X, u, M, fib, EA, L, g);
    for (int i = 0; i < N; ++i) {
        if (fixed[i]) continue;
        for (int k = 0; k < 3; ++k) a[3 * i + k] = g[3 * i + k] / m[i];
    }

    long n = 0;
    double t = 0.0, rho = 0.0, ke = 0.0;
    /* Energy balance (Fig. 1, the optional check): work done by the internal
     * forces, sum over passes of 1/2 (g_{n-1} + g_n) . du_n (trapezoid), and
     * work dissipated by the damping force, sum of c m |v_half|^2 dt (the
     * damping force acts with the half-step velocity, over du = dt v_half).
     * With v = 0 at the start, KE - work_int + work_damp stays near zero. */
    double work_int = 0.0, work_damp = 0.0;
    int status = OR_MAX_ITER;
    do {
        /* compute next time step: constant (R3), or from the current
         * state (R16) */
        if (dt_rule) {
            dt = step_at(N, X, u, M, fib, EA, L, fixed, m, dt, dt_safety, ksum);
            if (dt < dt_min) dt_min = dt;
        }
        /* partial velocity update (free dof) */
        for (int i = 0; i < N; ++i) {
            if (fixed[i]) continue;
            for (int k = 0; k < 3; ++k) v[3 * i + k] += 0.5 * dt * a[3 * i + k];
        }
        /* update displacements (free dof) */
        for (int i = 0; i < N; ++i) {
            if (fixed[i]) continue;
            for (int k = 0; k < 3; ++k) u[3 * i + k] += dt * v[3 * i + k];
        }
        /* getInternalForces(u) */
        memcpy(g_prev, g, n3 * sizeof(double));
        oracle_internal_force(N, X, u, M, fib, EA, L, g);
        /* work of the internal and the damping forces over this step */
        for (int i = 0; i < N; ++i) {
            if (fixed[i]) continue;
            for (int k = 0; k < 3; ++k) {
                double du = dt * v[3 * i + k];
                work_int += 0.5 * (g_prev[3 * i + k] + g[3 * i + k]) * du;
                work_damp += c * m[i] * v[3 * i + k] * du;
            }
        }
        /* damping force, force residual, accelerations (free dof) */
        double gf2 = 0.0, gb2 = 0.0;
        for (int i = 0; i < N; ++i) {
            for (int k = 0; k < 3; ++k) {
                double gk = g[3 * i + k];
                if (fixed[i]) gb2 += gk * gk; else gf2 += gk * gk;
            }
        }
        double den = sqrt(gb2);
        if (den < s_floor) den = s_floor;
        rho = sqrt(gf2) / den;
        for (int i = 0; i < N; ++i) {
            if (fixed[i]) continue;
            for (int k = 0; k < 3; ++k) {
                double fd = -c * m[i] * v[3 * i + k];
                a[3 * i + k] = (g[3 * i + k] + fd) / m[i];
            }
        }
        /* partial velocity update (free dof) */
        for (int i = 0; i < N; ++i) {
            if (fixed[i]) continue;
            for (int k = 0; k < 3; ++k) v[3 * i + k] += 0.5 * dt * a[3 * i + k];
        }
        /* energy (kinetic part reported) */
        ke = 0.0;
        for (int i = 0; i < N; ++i) {
            if (fixed[i]) continue;
            double vv = 0.0;
            for (int k = 0; k < 3; ++k) vv += v[3 * i + k] * v[3 * i + k];
            ke += 0.5 * m[i] * vv;
        }
        /* update iteration count */
        ++n;
        t += dt;
        if (rho_trace && n <= trace_len) rho_trace[n - 1] = rho;
        if (!isfinite(rho) || !isfinite(ke)) { status = OR_NONFINITE; break; }
        if (rho <= tol) { status = OR_CONVERGED; break; }
    } while (n < max_iter);

    stress(N, X, u, M, fib, EA, L, fixed, g, F, sigma, sigma_fib);
    *iters = n;
    *rho_out = rho;
    *ke_out = ke;
    *dt_out = dt0;
    *c_out = c;
    if (work_out) {
        work_out[0] = work_int;
        work_out[1] = work_damp;
        work_out[2] = dt_min;
    }
    (void)t;
    free(L); free(m); free(v); free(a); free(g); free(g_prev); free(ksum);
    return status;
}
