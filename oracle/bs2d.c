/*
 * bs2d.c -- plain FP64 reference solver for the two-asset Black-Scholes
 * equation and the Parareal iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the HIP path is checked
 * against.  It shares no code, header, table or helper with the product
 * library; only tests, the smoke check and the CPU-baseline leg of the bench
 * may load it.  It is compiled with -O3 -ffp-contract=off (no fast-math) so every operation
 * below is one IEEE double rounding in the order written.
 *
 * What it computes (paper: "Space-time parallel scaling of Parareal with a
 * physics-informed Fourier Neural Operator coarse propagator applied to the
 * Black-Scholes equation"):
 *   - the PDE in time-to-maturity form, Eq. (bse_change_variable), Sec. 3.2;
 *   - the centred finite-difference operator of Eq. (fd), Sec. 3.2 (second
 *     differences in x and y, the four-corner mixed difference, centred first
 *     differences, reaction -r u), written with x_i = i*h so that h cancels;
 *   - explicit Euler in time (the fine propagator used here; the paper
 *     uses implicit Euler, Eq. (fd), which is a later extension);
 *   - the coarse propagator G = B o P o Gc o R (injection, coarse explicit
 *     steps, bilinear prolongation, exact Dirichlet ring);
 *   - the Parareal iteration, Eq. (parareal), Sec. 3.1.
 * Every routine is the plain definition: no blocking, fusion or reordering.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_PAYOFF_BASKET = 0, ORC_PAYOFF_EXCHANGE = 1 };
enum { ORC_BC_FORWARD_INTRINSIC = 0, ORC_BC_DISCOUNTED_PAYOFF = 1, ORC_BC_EXACT = 2 };

/* One grid + model + payoff.  M nodes per side on [0, s_max]^2, both
 * boundaries included; node (i, j) is at x = i*h (asset 1), y = j*h (asset 2),
 * stored row-major u[i*M + j]. */
typedef struct {
    int32_t M;
    int32_t payoff_kind;
    int32_t bc_kind;
    int32_t pad_;
    double s_max;
    double sigma1, sigma2, rho, r;
    double w1, w2, strike;
} orc_problem;

static double orc_h(const orc_problem* p) { return p->s_max / (double)(p->M - 1); }

/* Standard normal CDF through erfc. */
static double ncdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

/* Payoff at maturity (tau = 0).  Basket call max(w1 x + w2 y - K, 0);
 * exchange max(x - y, 0). */
double orc_payoff(const orc_problem* p, double x, double y)
{
    if (p->payoff_kind == ORC_PAYOFF_EXCHANGE) {
        double v = x - y;
        return v > 0.0 ? v : 0.0;
    }
    double v = p->w1 * x + p->w2 * y - p->strike;
    return v > 0.0 ? v : 0.0;
}

/* Margrabe's price of the exchange option max(S1 - S2, 0); r cancels. */
double orc_margrabe(double x, double y, double tau, double s1, double s2, double rho)
{
    if (tau <= 0.0) { double v = x - y; return v > 0.0 ? v : 0.0; }
    if (x <= 0.0) return 0.0;
    if (y <= 0.0) return x;
    double var = s1 * s1 + s2 * s2 - 2.0 * rho * s1 * s2;
    double sd = sqrt(var * tau);
    double d1 = (log(x / y) + 0.5 * var * tau) / sd;
    double d2 = d1 - sd;
    return x * ncdf(d1) - y * ncdf(d2);
}

/* One-asset Black-Scholes call on S with strike K, rate r, volatility s. */
double orc_bs_call(double S, double K, double r, double s, double tau)
{
    if (tau <= 0.0) { double v = S - K; return v > 0.0 ? v : 0.0; }
    if (S <= 0.0) return 0.0;
    double sd = s * sqrt(tau);
    double d1 = (log(S / K) + (r + 0.5 * s * s) * tau) / sd;
    double d2 = d1 - sd;
    return S * ncdf(d1) - K * exp(-r * tau) * ncdf(d2);
}

/* Dirichlet data g(x, y, tau) on the boundary ring.
 *  FORWARD_INTRINSIC : basket max(w.S - K e^{-r tau}, 0); exchange max(x-y,0).
 *  DISCOUNTED_PAYOFF : e^{-r tau} * payoff(x, y).
 *  EXACT             : Margrabe for the exchange; for a basket with w2 = 0,
 *                      w1 * C_BS(x; K/w1) (the one-asset reduction).       */
double orc_bc(const orc_problem* p, double x, double y, double tau)
{
    if (p->bc_kind == ORC_BC_DISCOUNTED_PAYOFF)
        return exp(-p->r * tau) * orc_payoff(p, x, y);
    if (p->bc_kind == ORC_BC_EXACT) {
        if (p->payoff_kind == ORC_PAYOFF_EXCHANGE)
            return orc_margrabe(x, y, tau, p->sigma1, p->sigma2, p->rho);
        return p->w1 * orc_bs_call(x, p->strike / p->w1, p->r, p->sigma1, tau);
    }
    if (p->payoff_kind == ORC_PAYOFF_EXCHANGE) {
        double v = x - y;
        return v > 0.0 ? v : 0.0;
    }
    double v = p->w1 * x + p->w2 * y - p->strike * exp(-p->r * tau);
    return v > 0.0 ? v : 0.0;
}

/* u(tau = 0) = payoff at every node. */
void orc_init(const orc_problem* p, double* u)
{
    const int M = p->M;
    const double h = orc_h(p);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j)
            u[(size_t)i * M + j] = orc_payoff(p, i * h, j * h);
}

/* Overwrite the boundary ring (i or j in {0, M-1}) with g(., ., tau). */
void orc_set_boundary(const orc_problem* p, double tau, double* u)
{
    const int M = p->M;
    const double h = orc_h(p);
    for (int k = 0; k < M; ++k) {
        u[(size_t)0 * M + k] = orc_bc(p, 0.0, k * h, tau);
        u[(size_t)(M - 1) * M + k] = orc_bc(p, (M - 1) * h, k * h, tau);
        u[(size_t)k * M + 0] = orc_bc(p, k * h, 0.0, tau);
        u[(size_t)k * M + (M - 1)] = orc_bc(p, k * h, (M - 1) * h, tau);
    }
}

/* (L_h u)_{ij} at one interior node, Eq. (fd) spatial part with the signs of
 * Eq. (bse_change_variable) moved to the right-hand side:
 *   L_h u = 1/2 s1^2 x^2 D_xx u + 1/2 s2^2 y^2 D_yy u + rho s1 s2 x y D_xy u
 *         + r x D_x u + r y D_y u - r u.
 * With x_i = i h, y_j = j h every h cancels:
 *   1/2 s1^2 x_i^2 / h^2 = 1/2 s1^2 i^2, rho s1 s2 x_i y_j / (4 h^2) = rho s1 s2 i j / 4,
 *   r x_i / (2 h) = r i / 2. */
static double lh_at(const orc_problem* p, const double* u, int i, int j)
{
    const int M = p->M;
    const double s1 = p->sigma1, s2 = p->sigma2, rho = p->rho, r = p->r;
    const double fi = (double)i, fj = (double)j;
    const double* c = u + (size_t)i * M + j;
    double uxx = c[M] - 2.0 * c[0] + c[-M];                 /* (i+1) - 2 (i) + (i-1) */
    double uyy = c[1] - 2.0 * c[0] + c[-1];                 /* (j+1) - 2 (j) + (j-1) */
    double uxy = c[M + 1] + c[-M - 1] - c[M - 1] - c[-M + 1];
    double ux = c[M] - c[-M];
    double uy = c[1] - c[-1];
    return 0.5 * s1 * s1 * fi * fi * uxx
         + 0.5 * s2 * s2 * fj * fj * uyy
         + 0.25 * rho * s1 * s2 * fi * fj * uxy
         + 0.5 * r * fi * ux
         + 0.5 * r * fj * uy
         - r * c[0];
}

/* L_h u at every interior node; boundary entries of Lu are not written. */
void orc_apply_operator(const orc_problem* p, const double* u, double* Lu)
{
    const int M = p->M;
    for (int i = 1; i < M - 1; ++i)
        for (int j = 1; j < M - 1; ++j) Lu[(size_t)i * M + j] = lh_at(p, u, i, j);
}

/* One explicit Euler step at interior nodes: out = u + dt * L_h u.
 * The boundary ring of out is not written; out must not alias u. */
void orc_euler_step(const orc_problem* p, double dt, const double* u, double* out)
{
    const int M = p->M;
    /* rows in parallel (each node is the same independent expression; inside
     * the slice-parallel Parareal driver this region runs on one thread) */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (M > 64)
#endif
    for (int i = 1; i < M - 1; ++i)
        for (int j = 1; j < M - 1; ++j) {
            size_t k = (size_t)i * M + j;
            out[k] = u[k] + dt * lh_at(p, u, i, j);
        }
}

/* Fine propagator over one slice: m explicit steps of size dt starting at
 * tau0; after step q the ring is set to g(tau0 + (q+1) dt).  in and out may
 * alias. */
void orc_fine(const orc_problem* p, int m, double dt, double tau0, const double* in, double* out)
{
    const size_t n = (size_t)p->M * p->M;
    double* a = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    memcpy(a, in, sizeof(double) * n);
    for (int q = 0; q < m; ++q) {
        orc_euler_step(p, dt, a, b);
        orc_set_boundary(p, tau0 + (double)(q + 1) * dt, b);
        double* t = a; a = b; b = t;
    }
    memcpy(out, a, sizeof(double) * n);
    free(a);
    free(b);
}

/* Largest stable explicit-Euler step by Gershgorin's theorem.  Row (i,j) of
 * the update matrix has diagonal entry 1 + dt*c with c = -(s1^2 i^2 + s2^2 j^2
 * + r) and off-diagonal entries dt*(a_i +- m_i), dt*(b_j +- n_j),
 * +-dt*g_ij; every eigenvalue of L_h lies in a disc of centre c and radius
 * R = |a+m| + |a-m| + |b+n| + |b-n| + 4|g|, so |1 + dt lambda| <= 1 whenever
 * dt <= 2 / (|c| + R).  The bound is the minimum over interior nodes. */
double orc_stable_dt(const orc_problem* p)
{
    const int M = p->M;
    const double s1 = p->sigma1, s2 = p->sigma2, rho = p->rho, r = p->r;
    double worst = 0.0;
    for (int i = 1; i < M - 1; ++i)
        for (int j = 1; j < M - 1; ++j) {
            double a = 0.5 * s1 * s1 * i * i, b = 0.5 * s2 * s2 * j * j;
            double mi = 0.5 * r * i, nj = 0.5 * r * j;
            double g = 0.25 * rho * s1 * s2 * i * j;
            double c = 2.0 * a + 2.0 * b + r;
            double R = fabs(a + mi) + fabs(a - mi) + fabs(b + nj) + fabs(b - nj) + 4.0 * fabs(g);
            if (c + R > worst) worst = c + R;
        }
    return 2.0 / worst;
}

/* Steps per slice so that dt = dT/m <= cfl * dt_stable. */
int32_t orc_steps_for(const orc_problem* p, double dT, double cfl)
{
    double lim = cfl * orc_stable_dt(p);
    return (int32_t)ceil(dT / lim);
}

/* Injection: coarse node (I,J) takes fine node (I*q, J*q), q = (Mf-1)/(Mc-1). */
void orc_restrict(int Mf, int Mc, const double* fine, double* coarse)
{
    const int q = (Mf - 1) / (Mc - 1);
    for (int I = 0; I < Mc; ++I)
        for (int J = 0; J < Mc; ++J)
            coarse[(size_t)I * Mc + J] = fine[(size_t)(I * q) * Mf + (J * q)];
}

/* Bilinear prolongation: fine node (i,j) lies in coarse cell (I,J) with
 * fractional offsets a = (i - I q)/q, b = (j - J q)/q. */
void orc_prolong(int Mc, int Mf, const double* coarse, double* fine)
{
    const int q = (Mf - 1) / (Mc - 1);
    for (int i = 0; i < Mf; ++i)
        for (int j = 0; j < Mf; ++j) {
            int I = i / q, J = j / q;
            if (I > Mc - 2) I = Mc - 2;
            if (J > Mc - 2) J = Mc - 2;
            double a = (double)(i - I * q) / (double)q;
            double b = (double)(j - J * q) / (double)q;
            const double* c = coarse + (size_t)I * Mc + J;
            fine[(size_t)i * Mf + j] = (1.0 - a) * (1.0 - b) * c[0] + (1.0 - a) * b * c[1]
                                     + a * (1.0 - b) * c[Mc] + a * b * c[Mc + 1];
        }
}

/* Numerical coarse propagator over one slice:
 *   G(u) = B_{tau0 + m dt}( P( Gc( R u ) ) ),
 * Gc = m explicit steps on the coarse problem pc, B = exact Dirichlet ring
 * of the fine problem pf at the slice end. */
void orc_coarse(const orc_problem* pf, const orc_problem* pc, int m, double dt, double tau0,
                const double* in, double* out)
{
    const int Mf = pf->M, Mc = pc->M;
    double* c = (double*)malloc(sizeof(double) * (size_t)Mc * Mc);
    orc_restrict(Mf, Mc, in, c);
    orc_fine(pc, m, dt, tau0, c, c);
    orc_prolong(Mc, Mf, c, out);
    orc_set_boundary(pf, tau0 + (double)m * dt, out);
    free(c);
}

/* ---------------------------------------------------------------------------
 * Same-grid coarse propagator: locally one-dimensional implicit Euler.
 *
 * The paper's numerical coarse propagator is implicit Euler on the fine grid
 * with a larger time step (Sec. 3.2: coarse step 0.1, fine step a third of
 * it).  Here each implicit step is split by direction (locally one-
 * dimensional, LOD):
 *   Lx = alpha D_xx + mu D_x - r/2,   Ly = beta D_yy + nu D_y - r/2,
 *   Lxy = gamma D_xy (the four-corner mixed difference), L = Lx + Ly + Lxy,
 *   v   = u + dt Lxy u                            (explicit mixed term)
 *   (I - dt Lx) w  = v      along each interior column j (x lines)
 *   (I - dt Ly) u+ = w      along each interior row i    (y lines)
 * with u+ = g(tau1) on the ring, and on the two ring rows of the x stage the
 * end values w = (I - dt Ly) g(tau1), so that the step solves exactly
 *   (I - dt Ly)(I - dt Lx) u+ = u + dt Lxy u   at interior nodes.
 * Every line system is tridiagonal and solved by the Thomas algorithm.
 * ------------------------------------------------------------------------- */

/* Solve a_k x_{k-1} + b_k x_k + c_k x_{k+1} = d_k, k = 0..n-1, with x_{-1} =
 * xlo and x_n = xhi given; d is overwritten by the solution. */
static void thomas(int n, const double* a, const double* b, const double* c, double* d,
                   double xlo, double xhi, double* cp)
{
    d[0] -= a[0] * xlo;
    d[n - 1] -= c[n - 1] * xhi;
    cp[0] = c[0] / b[0];
    d[0] = d[0] / b[0];
    for (int k = 1; k < n; ++k) {
        double den = b[k] - a[k] * cp[k - 1];
        cp[k] = c[k] / den;
        d[k] = (d[k] - a[k] * d[k - 1]) / den;
    }
    for (int k = n - 2; k >= 0; --k) d[k] -= cp[k] * d[k + 1];
}

/* One LOD step from u (ring at the old time) to out; ring1 holds the ring
 * values at the new time (only its ring entries are read). */
void orc_lod_step_ring(const orc_problem* p, double dt, const double* u, const double* ring1,
                       double* out)
{
    const int M = p->M, n = M - 2;
    const double a1 = 0.5 * p->sigma1 * p->sigma1, a2 = 0.5 * p->sigma2 * p->sigma2;
    const double g12 = 0.25 * p->rho * p->sigma1 * p->sigma2, hr = 0.5 * p->r, r = p->r;
    double* v = (double*)malloc(sizeof(double) * (size_t)M * M);
    double *la = (double*)malloc(sizeof(double) * n), *lb = (double*)malloc(sizeof(double) * n);
    double *lc = (double*)malloc(sizeof(double) * n), *ld = (double*)malloc(sizeof(double) * n);
    double* cp = (double*)malloc(sizeof(double) * n);
    /* v = u + dt Lxy u */
    for (int i = 1; i < M - 1; ++i)
        for (int j = 1; j < M - 1; ++j) {
            const double* c = u + (size_t)i * M + j;
            v[(size_t)i * M + j] = c[0] + dt * g12 * i * j * (c[M + 1] + c[-M - 1] - c[M - 1] - c[-M + 1]);
        }
    /* (I - dt Ly) g(tau1) on the ring rows i = 0 and i = M-1 */
    double* wlo = (double*)malloc(sizeof(double) * M);
    double* whi = (double*)malloc(sizeof(double) * M);
    for (int j = 1; j < M - 1; ++j) {
        const double be = a2 * j * j, nu = hr * j;
        const double* g0 = ring1 + j;
        const double* g1 = ring1 + (size_t)(M - 1) * M + j;
        wlo[j] = g0[0] - dt * (be * (g0[1] - 2.0 * g0[0] + g0[-1]) + nu * (g0[1] - g0[-1]) - 0.5 * r * g0[0]);
        whi[j] = g1[0] - dt * (be * (g1[1] - 2.0 * g1[0] + g1[-1]) + nu * (g1[1] - g1[-1]) - 0.5 * r * g1[0]);
    }
    /* x lines: (I - dt Lx) w = v, unknowns i = 1..M-2 */
    for (int j = 1; j < M - 1; ++j) {
        for (int k = 0; k < n; ++k) {
            const int i = k + 1;
            const double al = a1 * i * i, mu = hr * i;
            la[k] = -dt * (al - mu);
            lb[k] = 1.0 + dt * (2.0 * al + 0.5 * r);
            lc[k] = -dt * (al + mu);
            ld[k] = v[(size_t)i * M + j];
        }
        thomas(n, la, lb, lc, ld, wlo[j], whi[j], cp);
        for (int k = 0; k < n; ++k) v[(size_t)(k + 1) * M + j] = ld[k];   /* v now holds w */
    }
    /* y lines: (I - dt Ly) u+ = w, unknowns j = 1..M-2 */
    for (int i = 1; i < M - 1; ++i) {
        for (int k = 0; k < n; ++k) {
            const int j = k + 1;
            const double be = a2 * j * j, nu = hr * j;
            la[k] = -dt * (be - nu);
            lb[k] = 1.0 + dt * (2.0 * be + 0.5 * r);
            lc[k] = -dt * (be + nu);
            ld[k] = v[(size_t)i * M + j];
        }
        thomas(n, la, lb, lc, ld, ring1[(size_t)i * M], ring1[(size_t)i * M + M - 1], cp);
        for (int k = 0; k < n; ++k) out[(size_t)i * M + k + 1] = ld[k];
    }
    for (int k = 0; k < M; ++k) {
        out[k] = ring1[k];
        out[(size_t)(M - 1) * M + k] = ring1[(size_t)(M - 1) * M + k];
        out[(size_t)k * M] = ring1[(size_t)k * M];
        out[(size_t)k * M + M - 1] = ring1[(size_t)k * M + M - 1];
    }
    free(v); free(la); free(lb); free(lc); free(ld); free(cp); free(wlo); free(whi);
}

/* LOD coarse propagator over one slice: m steps of dt from tau0, ring g. */
void orc_lod(const orc_problem* p, int m, double dt, double tau0, const double* in, double* out)
{
    const size_t n = (size_t)p->M * p->M;
    double* a = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    double* ring = (double*)malloc(sizeof(double) * n);
    memcpy(a, in, sizeof(double) * n);
    for (int q = 0; q < m; ++q) {
        orc_set_boundary(p, tau0 + (double)(q + 1) * dt, ring);
        orc_lod_step_ring(p, dt, a, ring, b);
        double* t = a; a = b; b = t;
    }
    memcpy(out, a, sizeof(double) * n);
    free(a); free(b); free(ring);
}

/* ---------------------------------------------------------------------------
 * Parareal, Eq. (parareal), Sec. 3.1, for a generic state of `len` doubles and
 * propagators given as callbacks prop(ctx, n, in, out) over slice n.
 *
 *   initialisation : U^0_0 = u0, U^0_{n+1} = G(U^0_n)
 *   iteration k    : f_n = F(U^k_n)              (independent in n: OpenMP)
 *                    U^{k+1}_0 = u0
 *                    U^{k+1}_{n+1} = f_n + (G(U^{k+1}_n) - G(U^k_n))   serial in n
 *   increment      : d^{k+1} = max_{n>=1} max |U^{k+1}_n - U^k_n|
 *   stop           : d < tol (tol_relative: d < tol * max |U^{k+1}_N|),
 *                    or k+1 == N (U^N_n = F^n u0 exactly), or k+1 == max_iters.
 * The bracket is evaluated first so that identical coarse inputs cancel to an
 * exact zero.  U holds (N+1)*len doubles; on return U[n] = U^K_n.
 * increments[k] = d^{k+1}; returns K, or -1 when an increment is not finite.
 * ------------------------------------------------------------------------- */
typedef void (*orc_prop_fn)(void* ctx, int32_t n, const double* in, double* out);

int32_t orc_parareal(int64_t len, int32_t N, const double* u0, orc_prop_fn F, void* ctxF,
                     orc_prop_fn G, void* ctxG, int32_t max_iters, double tol, int32_t tol_relative,
                     double* U, double* increments)
{
    const size_t L = (size_t)len;
    double* Gold = (double*)malloc(sizeof(double) * L * N);
    double* f = (double*)malloc(sizeof(double) * L * N);
    double* Unew = (double*)malloc(sizeof(double) * L * (N + 1));
    double* gnew = (double*)malloc(sizeof(double) * L);

    memcpy(U, u0, sizeof(double) * L);
    for (int n = 0; n < N; ++n) {
        G(ctxG, n, U + L * n, Gold + L * n);
        memcpy(U + L * (n + 1), Gold + L * n, sizeof(double) * L);
    }
    int32_t K = 0;
    int finite = 1;
    for (int k = 0; k < max_iters && k < N; ++k) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
        for (int n = 0; n < N; ++n)
            F(ctxF, n, U + L * n, f + L * n);
        memcpy(Unew, u0, sizeof(double) * L);
        for (int n = 0; n < N; ++n) {
            G(ctxG, n, Unew + L * n, gnew);
            double* dst = Unew + L * (n + 1);
            const double* fn = f + L * n;
            double* go = Gold + L * n;
            for (size_t e = 0; e < L; ++e) dst[e] = fn[e] + (gnew[e] - go[e]);
            memcpy(go, gnew, sizeof(double) * L);
        }
        double d = 0.0, scale = 0.0;
        for (size_t e = L; e < L * (N + 1); ++e) {
            double a = fabs(Unew[e] - U[e]);
            if (!(a == a) || isinf(a)) finite = 0;
            if (a > d) d = a;
        }
        for (size_t e = L * N; e < L * (N + 1); ++e) {
            double s = fabs(Unew[e]);
            if (s > scale) scale = s;
        }
        memcpy(U, Unew, sizeof(double) * L * (N + 1));
        increments[k] = finite ? d : NAN;
        K = k + 1;
        if (!finite) break;
        double thr = tol_relative ? tol * scale : tol;
        if (d < thr) break;
    }
    free(Gold);
    free(f);
    free(Unew);
    free(gnew);
    return finite ? K : -1;
}

/* ---------------------------------------------------------------------------
 * The Black-Scholes instance of the driver above.
 * ------------------------------------------------------------------------- */
enum { ORC_G_NUMERICAL = 0, ORC_G_FINE = 1, ORC_G_LOD = 2 };

typedef struct {
    orc_problem fine, coarse;
    int32_t N, mF, mG, coarse_kind;
    double T;
} orc_bs_ctx;

static void bs_F(void* ctx, int32_t n, const double* in, double* out)
{
    const orc_bs_ctx* c = (const orc_bs_ctx*)ctx;
    double dT = c->T / c->N;
    orc_fine(&c->fine, c->mF, dT / c->mF, n * dT, in, out);
}

static void bs_G(void* ctx, int32_t n, const double* in, double* out)
{
    const orc_bs_ctx* c = (const orc_bs_ctx*)ctx;
    double dT = c->T / c->N;
    if (c->coarse_kind == ORC_G_FINE)
        orc_fine(&c->fine, c->mF, dT / c->mF, n * dT, in, out);
    else if (c->coarse_kind == ORC_G_LOD)
        orc_lod(&c->fine, c->mG, dT / c->mG, n * dT, in, out);
    else
        orc_coarse(&c->fine, &c->coarse, c->mG, dT / c->mG, n * dT, in, out);
}

/* Serial fine solution: u <- F(u) for n = 0..N-1, starting from the payoff.
 * Output: the fine state at tau = T (price today). */
void orc_serial_fine(const orc_problem* p, int32_t N, double T, int32_t mF, double* out)
{
    const double dT = T / N;
    orc_init(p, out);
    for (int n = 0; n < N; ++n) orc_fine(p, mF, dT / mF, n * dT, out, out);
}

/* Parareal on the Black-Scholes problem.  out = U^K_N (fine grid); returns K
 * (>= 1) or -1 on a non-finite increment. */
int32_t orc_parareal_bs(const orc_problem* fine, const orc_problem* coarse, int32_t N, double T,
                        int32_t mF, int32_t mG, int32_t coarse_kind, int32_t max_iters, double tol,
                        int32_t tol_relative, double* out, double* increments)
{
    orc_bs_ctx c;
    c.fine = *fine;
    c.coarse = *coarse;
    c.N = N;
    c.mF = mF;
    c.mG = mG;
    c.coarse_kind = coarse_kind;
    c.T = T;
    const size_t L = (size_t)fine->M * fine->M;
    double* u0 = (double*)malloc(sizeof(double) * L);
    double* U = (double*)malloc(sizeof(double) * L * (N + 1));
    orc_init(fine, u0);
    int32_t K = orc_parareal((int64_t)L, N, u0, bs_F, &c, bs_G, &c, max_iters, tol, tol_relative, U,
                             increments);
    memcpy(out, U + L * N, sizeof(double) * L);
    free(u0);
    free(U);
    return K;
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
