/* parareal3.h -- C ABI of Parareal for the three-asset Black-Scholes equation
 * on gfx950: the n-asset generalisation, Eq. (bse_general) (Sec. 3.2), with
 * n = 3, discretised by the centred differences of Eq. (fd) in every axis and
 * every pair of axes (a 19-point stencil), explicit Euler in time, FP64.
 *
 * The problem: V(S1, S2, S3, tau) on [0, s_max]^3 with n nodes per axis (both
 * boundaries included, h = s_max / (n - 1)), in time to maturity tau = T - t,
 *
 *   V_tau = 1/2 sum_{d,e} rho_de s_d s_e S_d S_e V_de + r sum_d S_d V_d - r V,
 *
 * payoff the basket call max(w . S - K, 0), and on the six faces the forward
 * intrinsic value max(w . S - K e^{-r tau}, 0) at every step (an exact
 * solution of the equation where the max is active).  Parareal (Eq. (parareal),
 * Sec. 3.1): F is explicit Euler on the n^3 grid, G the same scheme on a
 * coarse grid of nc nodes per axis ((n - 1) divisible by (nc - 1)) with
 * injection and trilinear prolongation, the faces of G's output set to the fine
 * boundary data.  Step counts follow the Gershgorin bound of explicit Euler on
 * each grid (cfl times it), unless given.
 *
 * Memory: the caller passes one device workspace of pr3_workspace_bytes(), a
 * hipStream_t (NULL: the null stream) and device output arrays; the library
 * allocates no device memory.  States are stored as interior nodes only, k
 * (the S3 index) contiguous with a row pitch of a multiple of 64 elements.
 * Errors: the pr_status codes of parareal.h; argument errors return
 * PR_EINVAL before anything runs.
 */
#ifndef PARAREAL3_H
#define PARAREAL3_H

#include <stdint.h>

#include "parareal.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;             /* fine nodes per axis, 5 .. 513 */
    int32_t coarse_n;      /* coarse nodes per axis, >= 3, (n - 1) % (coarse_n - 1) == 0 */
    int32_t n_slices;      /* N, 1 .. PR_MAX_SLICES */
    int32_t max_iters;     /* 0 => N */
    int32_t fine_steps;    /* explicit steps per slice on the fine grid; 0 => from cfl */
    int32_t coarse_steps;  /* explicit steps per slice on the coarse grid; 0 => from cfl */
    double s_max;          /* > 0 */
    double T;              /* maturity, > 0 */
    double tol;            /* stop when max |U^k - U^{k-1}| < tol (absolute); 0 => run to K = N */
    double cfl;            /* fraction of the stability bound, (0, 1]; 0 => 0.9 */
    double sigma[3];       /* volatilities, > 0 */
    double rho[3];         /* correlations (rho12, rho13, rho23); the matrix must be
                              positive semi-definite */
    double r;              /* interest rate, >= 0 */
    double w[3];           /* basket weights */
    double strike;         /* K */
} pr3_problem;

typedef struct {
    int32_t iters;              /* Parareal iterations K */
    int32_t fine_steps;         /* steps per slice used by F */
    int32_t coarse_steps;       /* steps per slice used by G */
    int32_t pad_;
    double last_increment;
    double increments[PR_MAX_SLICES + 1];
    double t_fine_ms;           /* GPU time of the fine sweeps (HIP events) */
    double t_coarse_ms;         /* GPU time of G, the corrections and the norms */
    double t_total_ms;          /* host wall time of the call */
    int64_t fine_point_steps;   /* interior node-steps of F in this call */
} pr3_stats;

typedef struct pr3_solver pr3_solver; /* opaque */

/* Step counts the solver would use (PR_EUNSTABLE if a given count exceeds the
 * stability bound). */
pr_status pr3_plan(const pr3_problem* p, int32_t* fine_steps, int32_t* coarse_steps);
/* Device workspace needed (0 if the problem is invalid). */
uint64_t pr3_workspace_bytes(const pr3_problem* p);
/* Validate, carve the workspace (device pointer, 256-byte aligned, owned by the
 * caller, at least pr3_workspace_bytes) and return a solver bound to the stream. */
pr_status pr3_create(const pr3_problem* p, void* workspace, uint64_t workspace_bytes,
                     void* hip_stream, pr3_solver** out);
/* Parareal from the payoff to tau = T; v_out: device array of n^3 doubles
 * (index (i, j, k) at (i n + j) n + k, faces included); st may be NULL.
 * Returns when the result is written.  PR_ENOTCONV: max_iters reached above
 * tol (the result is still written). */
pr_status pr3_solve(pr3_solver* s, double* v_out, pr3_stats* st);
/* F over all slices in order from the payoff (the reference of Parareal). */
pr_status pr3_serial_fine(pr3_solver* s, double* v_out, pr3_stats* st);
/* One fine sweep over every slice at once from the payoff broadcast to all of
 * them (the step kernel's throughput at the solver's shape); *ms receives the
 * GPU time of the step launches. */
pr_status pr3_fine_sweep_probe(pr3_solver* s, double* ms, int64_t* point_steps);
pr_status pr3_destroy(pr3_solver* s);
const char* pr3_last_error(const pr3_solver* s);

#ifdef __cplusplus
}
#endif

#endif /* PARAREAL3_H */
