/*
 * parareal.h -- C ABI of the MI355X (gfx950) Parareal solver for the
 * two-asset Black-Scholes equation.
 *
 * The method: Parareal, Eq. (parareal) of Sec. 3.1 ("Space-time parallel
 * scaling of Parareal with a physics-informed Fourier Neural Operator coarse
 * propagator applied to the Black-Scholes equation", Ibrahim, Goetschel,
 * Ruprecht), applied to the two-asset Black-Scholes equation in
 * time-to-maturity form, Eq. (bse_change_variable) of Sec. 3.2, discretised
 * in space by the centred finite differences of Eq. (fd).  Time stepping of
 * the fine propagator F is explicit Euler; the coarse propagator G is the same
 * scheme on a coarser grid with injection and bilinear prolongation, or G := F
 * for tests.
 *
 * Conventions shared by every entry point:
 *  - Grids are n x n nodes on [0, s_max]^2 including both boundaries; node
 *    (i, j) sits at S1 = i*h, S2 = j*h with h = s_max/(n-1).  A full grid is
 *    n*n doubles, row-major, index i*n + j (j = S2 index contiguous).
 *  - Time runs as tau = T - t from tau = 0 (the payoff) to tau = T (today).
 *    Slice k covers [k*T/N, (k+1)*T/N].
 *  - "Device pointer" means memory allocated on the GPU the solver was
 *    created on (e.g. a torch CUDA/HIP tensor's data_ptr()).  "Host pointer"
 *    means ordinary CPU memory.
 *  - The caller owns every buffer it passes (workspace, outputs, stream);
 *    the library never frees caller memory and allocates no device memory
 *    of its own.  Structs passed to parareal_create are copied.
 *  - Every call returns a pr_status; no C++ exception crosses the boundary.
 *    parareal_last_error() gives a message for the last failing call on a
 *    solver.  A solver is not thread-safe; distinct solvers on distinct
 *    streams are independent.
 *  - All GPU work is enqueued on the stream given at create time.  Calls
 *    that return results to the host (solve, serial_fine) synchronise that
 *    stream before returning.
 */
#ifndef PARAREAL_H
#define PARAREAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_ABI_VERSION 2
#define PR_MAX_SLICES 1024

typedef struct pr_solver pr_solver; /* opaque */

typedef enum {
    PR_OK = 0,
    PR_EINVAL = 1,       /* an argument is out of range or inconsistent */
    PR_EUNSTABLE = 2,    /* the requested explicit step exceeds the stability bound */
    PR_ENOMEM = 3,       /* the workspace is smaller than parareal_workspace_bytes() */
    PR_EDEVICE = 4,      /* a HIP runtime call failed */
    PR_ENOTCONV = 5,     /* max_iters reached above tolerance (result still written) */
    PR_ENONFINITE = 6,   /* a non-finite value appeared in the iteration */
    PR_EMODEL = 7,       /* coarse model unavailable */
    PR_EBUSY = 8         /* pr_server_submit: the bounded queue of waiting requests is full */
} pr_status;

/* Payoff at maturity (tau = 0). */
enum { PR_PAYOFF_BASKET_CALL = 0,    /* max(w1 S1 + w2 S2 - K, 0) */
       PR_PAYOFF_EXCHANGE = 1,       /* max(S1 - S2, 0) */
       PR_PAYOFF_CASH_OR_NOTHING = 2 /* the paper's benchmark option (Sec. 3.2): cash if
                                        S1 >= strike and S2 >= strike2, else 0; ring kinds
                                        PR_BC_EXACT (Eq. (solution), |rho| <= 0.925) or
                                        PR_BC_DISCOUNTED_PAYOFF */ };

/* Dirichlet data on the boundary ring at time-to-maturity tau. */
enum { PR_BC_FORWARD_INTRINSIC = 0, /* basket: max(w1 S1 + w2 S2 - K e^{-r tau}, 0);
                                       exchange: max(S1 - S2, 0) */
       PR_BC_DISCOUNTED_PAYOFF = 1, /* e^{-r tau} * payoff(S1, S2) */
       PR_BC_EXACT = 2              /* exchange: Margrabe's formula; basket with w2 = 0:
                                       w1 * BlackScholesCall(S1; K/w1); cash-or-nothing:
                                       cash e^{-r tau} B(d1, d2; rho), Eq. (solution), with the
                                       bivariate normal CDF B by Plackett's identity and a
                                       20-point Gauss-Legendre rule */ };

/* Coarse propagator. */
enum { PR_G_NUMERICAL = 0, /* explicit Euler on a coarse grid, injection + bilinear */
       PR_G_FNO = 1,       /* the Fourier neural operator of Sec. 3.4 on a 64 x 64 grid, reached
                              through sine (DST-I) transfers of V - B(tau), B the Coons patch of
                              the ring values: G(u) = B(tau_{n+1}) + P_s(w + out_scale *
                              FNO(w, sigma1, sigma2, rho, r)), w = R_s(u - B(tau_n)), with w
                              replaced by the base of the operator's PR_FNO_BASE_*.  Needs
                              n >= 64 and an operator attached with parareal_attach_fno.  If the
                              increment is non-finite or grows in two consecutive iterations, the
                              solve restarts with PR_G_LOD (coarse_steps, default 4) and reports
                              pr_stats.coarse_fallback = 1; the solver keeps PR_G_LOD after that */
       PR_G_FINE = 2,      /* G := F (test mode: Parareal stops after one iteration) */
       PR_G_LOD = 3,       /* implicit Euler on the fine grid with coarse_steps steps per
                              slice (default 2), split by direction: the explicit mixed
                              term, then tridiagonal x lines and y lines (Sec. 3.2's
                              coarse propagator is implicit Euler with a larger step) */
       PR_G_IMPLICIT = 4   /* the paper's numerical G (Sec. 3.2): implicit Euler of
                              Eq. (fd) on the fine grid with coarse_steps steps per slice
                              (default 1), each solved by the BiCGStab of PR_FINE_IMPLICIT
                              (krylov_tol, krylov_max_iters); needs PR_FP64 */ };

/* Option flags.  PR_FLAG_TIME_STEPS: bracket runs of 8 consecutive explicit
 * fine-step launches (a run also ends with its sweep) with HIP events on the
 * solver's stream and report their summed durations in
 * pr_stats.t_step_kernels_ms, the launches and their algorithmic bytes in
 * timed_step_launches / timed_step_bytes (without the flag the field brackets
 * the whole run of step launches, gaps included).  A run's duration over its
 * launches is their launch-to-launch time: the dispatch delay of a run's first
 * launch is spread over the run. */
#define PR_FLAG_TIME_STEPS 1u
/* PR_FLAG_GRAPH: capture the initial sweep and each Parareal iteration k (its
 * fine sweep, coarse chain, correction and norm) into a HIP graph once, on a
 * private capture stream, and replay it on the solver's stream; graphs are
 * cached per k and reused by later solves of the same solver.  Phase timings
 * then cover whole iterations (t_fine_ms) and PR_FLAG_TIME_STEPS is ignored. */
#define PR_FLAG_GRAPH 2u
/* PR_FLAG_NO_FALLBACK: PR_G_FNO keeps the neural propagator even when the
 * increments grow (a non-finite increment then ends the solve with
 * PR_ENONFINITE, as for the other propagators). */
#define PR_FLAG_NO_FALLBACK 4u
/* PR_FLAG_SERIAL_CHAIN: run each iteration's coarse chain and correction after
 * its whole fine sweep, on the solver's stream.  By default (explicit F with the
 * numerical G, no PR_FLAG_GRAPH) the active slices are split in phases: while
 * at least 32 slices are active, a phase fixes a boundary B (about two thirds
 * of the active slices into the first group) and its iterations run two groups
 * of consecutive slices, [k, B) and [B, N).  The fine sweep runs group by group
 * on the solver's stream; each group's gather, chain and correction run on a
 * second stream of the solver as soon as its sweep ends, so the first group's
 * chain overlaps the second group's sweep; and the next iteration's first-group
 * sweep, which needs only states the first group's correction has written,
 * starts beside the second group's chain (it is discarded if the iteration
 * stops there).  The chain of the second group restarts from the corrected
 * state at its first slice, which equals the chain's own value there bitwise.
 * Results are bitwise those of the serial schedule.  In pr_stats, t_fine_ms
 * covers the fine sweeps, t_chain_ms the chain and correction time left after
 * the last sweep (the exposed part), t_correct_ms 0. */
#define PR_FLAG_SERIAL_CHAIN 8u

/* Time stepping of the fine propagator F.  PR_FINE_EXPLICIT: explicit Euler
 * (the planner keeps dt below the stability bound).  PR_FINE_IMPLICIT: implicit
 * Euler exactly as Eq. (fd) (Sec. 3.2): every step solves (I - dt L_h) u+ = u on
 * the interior with the ring of u+ at the new time, by Jacobi-preconditioned
 * BiCGStab on the GPU (matrix-free, all slices of a sweep together) to the
 * relative residual krylov_tol; it needs PR_FP64 and fine_steps >= 1, and is not
 * available with PR_FLAG_GRAPH or through the server (the solver polls the
 * iteration on the host). */
enum { PR_FINE_EXPLICIT = 0, PR_FINE_IMPLICIT = 1 };

/* Arithmetic of the fine and numerical coarse propagators. */
enum { PR_FP64 = 0, /* everything in FP64 */
       PR_FP32 = 1  /* FP32 increments over an FP64 slice base; correction and norm FP64 */ };

typedef struct {
    int32_t n;       /* nodes per side, >= 5 */
    int32_t pad_;
    double s_max;    /* domain [0, s_max]^2, > 0 */
} pr_grid;

typedef struct {
    double sigma1, sigma2; /* volatilities, > 0 */
    double rho;            /* correlation, |rho| < 1 */
    double r;              /* risk-free rate, >= 0 */
    double T;              /* maturity, > 0 */
} pr_model;

typedef struct {
    int32_t kind;    /* PR_PAYOFF_* */
    int32_t bc_kind; /* PR_BC_* */
    double w1, w2;   /* basket weights (basket call only) */
    double strike;   /* K (basket call); K1 (cash-or-nothing) */
    double strike2;  /* K2 (cash-or-nothing only) */
    double cash;     /* cash amount c (cash-or-nothing only) */
} pr_payoff;

typedef struct {
    int32_t n_slices;       /* N, 1..PR_MAX_SLICES */
    int32_t max_iters;      /* cap on Parareal iterations K; 0 => N */
    double tol;             /* stop when the max increment is below tol ... */
    int32_t tol_relative;   /* ... (1: times max |U^k_N| over all nodes) */
    int32_t precision;      /* PR_FP64 or PR_FP32 */
    int32_t fine_steps;     /* explicit steps per slice; 0 => planned from cfl */
    int32_t coarse_kind;    /* PR_G_* */
    int32_t coarse_n;       /* PR_G_NUMERICAL: coarse nodes per side, 3..257;
                               (n-1) % (coarse_n-1) == 0 */
    int32_t coarse_steps;   /* coarse steps per slice; 0 => planned from cfl (PR_G_LOD: 2) */
    double cfl;             /* planned dt = dT / ceil(dT / (cfl * dt_stable)); (0, 1] */
    uint32_t flags;         /* PR_FLAG_* bits */
    int32_t fine_scheme;    /* PR_FINE_* */
    double krylov_tol;      /* PR_FINE_IMPLICIT: relative residual ||r|| / ||b||; 0 => 1e-12 */
    int32_t krylov_max_iters; /* PR_FINE_IMPLICIT: BiCGStab iterations per step;
                                 0 => max(1000, 10 (n - 2)) */
    int32_t pad2_;
} pr_options;

typedef struct {
    int32_t status;             /* pr_status of the call */
    int32_t iters;              /* Parareal iterations performed (K) */
    int32_t fine_steps;         /* explicit fine steps per slice */
    int32_t coarse_steps;       /* coarse steps per slice */
    double last_increment;      /* max |U^K_n - U^{K-1}_n| */
    double scale;               /* max |U^K_N| over all nodes */
    double increments[PR_MAX_SLICES + 1]; /* increments[k] after iteration k+1 */
    double t_total_ms;          /* wall time of the call, host clock */
    double t_fine_ms;           /* GPU time of the fine sweeps (HIP events) */
    double t_chain_ms;          /* GPU time of the coarse chains; with a fine-grid G
                                   (LOD, FNO, FINE) the chain applies G and the
                                   correction slice by slice, so this includes the
                                   corrections and t_correct_ms is 0 */
    double t_correct_ms;        /* GPU time of the corrections + norms (coarse-grid G) */
    int64_t fine_point_steps;   /* interior node updates performed by F */
    int64_t fine_step_launches; /* explicit-step kernel launches */
    double fine_step_bytes;     /* algorithmic bytes moved by those launches */
    double t_step_kernels_ms;   /* GPU time of those launches (HIP events, see PR_FLAG_TIME_STEPS) */
    uint64_t workspace_bytes;   /* bytes of workspace the solver uses */
    int32_t coarse_fallback;    /* 1 when PR_G_FNO fell back to PR_G_LOD in this solve */
    int32_t pad_;
    int64_t timed_step_launches; /* step launches bracketed by events (PR_FLAG_TIME_STEPS) */
    double timed_step_bytes;     /* their algorithmic bytes (t_step_kernels_ms covers them) */
    int64_t krylov_iters;        /* PR_FINE_IMPLICIT: BiCGStab iterations summed over steps
                                    (a step runs until its last slice converges) */
    int32_t krylov_max_step;     /* most iterations one step took */
    int32_t krylov_unconverged;  /* slice-steps stopped at krylov_max_iters or by a breakdown */
} pr_stats;

/* Explicit-Euler stability bound and the planned step counts (host only, no
 * GPU).  dt_stable = 2 / max over interior nodes of (|c| + R), where c and R
 * are the centre and radius of the Gershgorin disc of the operator of
 * Eq. (fd) at that node.  Writes fine and coarse steps per slice (the given
 * counts, or the cfl plan when they are 0) and the two bounds.  Returns
 * PR_EINVAL on bad arguments, PR_EUNSTABLE if a given step count exceeds the
 * bound. */
pr_status parareal_plan(const pr_grid* grid, const pr_model* model, const pr_options* opt,
                        int32_t* fine_steps, int32_t* coarse_steps, double* dt_stable_fine,
                        double* dt_stable_coarse);

/* Bytes of device workspace a solver with these options needs (host only).
 * Returns 0 when the arguments are invalid. */
uint64_t parareal_workspace_bytes(const pr_grid* grid, const pr_options* opt);

/* Create a solver.  device_workspace: device pointer to at least
 * parareal_workspace_bytes() bytes, 256-byte aligned, owned by the caller and
 * borrowed until parareal_destroy.  hip_stream: a hipStream_t (NULL = the
 * default stream).  Validation happens before any GPU call. */
pr_status parareal_create(const pr_grid* grid, const pr_model* model, const pr_payoff* payoff,
                          const pr_options* opt, void* device_workspace, uint64_t workspace_bytes,
                          void* hip_stream, pr_solver** out);

/* Run Parareal, Eq. (parareal), from the payoff at tau = 0 to tau = T and
 * write U^K_N (n*n doubles, device pointer) to v_out.  Initialisation:
 * U^0_0 = payoff, U^0_{k+1} = G(U^0_k).  Iterates until the max increment is
 * below the tolerance, K = N (then the result equals serial F exactly) or
 * K = max_iters (PR_ENOTCONV, result still written).  stats (host pointer,
 * may be NULL) receives the iteration history and timings. */
pr_status parareal_solve(pr_solver* s, double* v_out, pr_stats* stats);

/* Serial fine solution: u <- F(u) for slices 0..N-1 from the payoff; writes
 * the state at tau = T (n*n doubles, device pointer) to v_out. */
pr_status parareal_serial_fine(pr_solver* s, double* v_out, pr_stats* stats);

/* Apply one propagator over slice k to a full grid: op = PR_OP_FINE (F) or
 * PR_OP_COARSE (G); in and out are device pointers to n*n doubles (may not
 * alias).  The input's boundary ring is taken as g(tau_k) whatever it holds;
 * the output's ring is g(tau_{k+1}). */
enum { PR_OP_FINE = 0, PR_OP_COARSE = 1 };
pr_status parareal_apply(pr_solver* s, int32_t op, int32_t slice, const double* in, double* out);

pr_status parareal_destroy(pr_solver* s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * solve, as parareal_create + parareal_solve + parareal_destroy, on a workspace
 * that is a static device array of PR_STATIC_SCRATCH_BYTES inside the library
 * (one copy per GPU, held until the process ends).  It calls no hipMalloc,
 * hipFree or other allocating routine and creates no event, stream or graph;
 * PR_FLAG_TIME_STEPS and PR_FLAG_GRAPH are ignored (phase timings stay 0).
 * The stream must belong to the current device; v_out (device, n*n doubles)
 * and stats (host, may be NULL) as in parareal_solve, and the same kernels run
 * with the same launch geometry, so the result equals parareal_solve's bitwise.
 * Errors: PR_ENOMEM when the problem's workspace (parareal_workspace_bytes)
 * exceeds PR_STATIC_SCRATCH_BYTES; PR_EINVAL for PR_G_FNO (it needs an attached
 * operator) and for the argument errors of parareal_create; PR_EDEVICE when the
 * scratch's device address cannot be obtained.  Every call on one GPU uses that
 * GPU's one array and keeps its contents after returning: calls that overlap on
 * one GPU (other threads, other streams) race and must be serialised by the
 * caller. */
#define PR_STATIC_SCRATCH_BYTES (64ull << 20)
pr_status parareal_solve_static(const pr_grid* grid, const pr_model* model,
                                const pr_payoff* payoff, const pr_options* opt, void* hip_stream,
                                double* v_out, pr_stats* stats);

/* PR_G_FNO solvers: attach the operator (borrowed, not owned; it must outlive
 * the solver's use of it and is used on the solver's stream, one solve at a
 * time).  PR_EINVAL for solvers of another coarse kind. */
typedef struct pr_fno pr_fno;
pr_status parareal_attach_fno(pr_solver* s, pr_fno* f);

/* PR_G_FNO solvers: one training pair of the operator from two fine states,
 * v0 at tau_slice and v1 at tau_{slice+1} (n*n doubles each, device).  Writes
 * four 64 x 64 FP32 planes (device) [w_in, B1, V_in, V_tgt]: w_in = R_s(v0 -
 * B(tau_slice)) with zero ring, B1 = the Coons patch of g(tau_{slice+1}) on the
 * 64 x 64 grid (base PR_FNO_BASE_LOD: plus the 64 x 64 LOD prediction's w;
 * PR_FNO_BASE_FINE_LOD: plus R_s(LOD(v0) - B(tau_{slice+1})) of the fine LOD), V_in =
 * B0 + w_in and V_tgt = B1 + R_s(v1 - B(tau_{slice+1})) with the Coons B1. */
pr_status parareal_fno_pair(pr_solver* s, int32_t slice, const double* v0, const double* v1,
                            int32_t base, float* pair_out);

/* PR_G_FNO solvers: the training pairs of one whole trajectory.  Runs serial F
 * from the payoff over all N slices and writes, for every slice n, the pair of
 * parareal_fno_pair from the F states at tau_n and tau_{n+1}: pairs_out
 * (device) receives N x 4 x 64 x 64 floats. */
pr_status parareal_fno_pairs(pr_solver* s, int32_t base, float* pairs_out);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent Parareal solves (no counterpart
 * in the paper; the solves are those of parareal_solve).
 *
 * A server owns nothing but its streams and a small pinned host pool: the
 * caller hands it one device arena, and every admitted request gets its
 * workspace carved out of that arena (first fit, 256-byte aligned) for as
 * long as it is resident.  Requests are admitted in submission order while
 * their workspace fits and fewer than max_resident are resident; each
 * resident request runs on one of n_streams HIP streams, so the kernels of
 * different requests overlap on the device.  pr_server_progress never blocks:
 * it looks at which in-flight iterations have finished, decides stop or
 * continue for each from its 24-byte norm read-back, enqueues the next
 * iteration or the final write of the result, retires finished requests
 * (their workspace returns to the arena) and admits waiting ones.  Results
 * are bitwise those of parareal_solve on the same request.
 *
 * PR_SERVER_RAGGED_F: the fine sweeps (Eq. (parareal)'s F over the active
 * slices, Sec. 3.1) of every request that a progress pass makes ready for an
 * iteration run together at the end of that pass, as shared step launches:
 * sweeps of similar work per step (point-steps per step within a power of 4)
 * share launches that carry up to eight requests' slices, each with its own
 * grid, step size and launch geometry (a ragged launch), on one of up to four
 * extra streams taken in turn.  Each request's coarse chain and correction
 * follow on its own stream as soon as its own sweep has ended.  Requests
 * whose Dirichlet data are PR_BC_EXACT keep launches of their own in that
 * sequence.  Results are unchanged (bitwise).
 * ------------------------------------------------------------------------- */
typedef struct pr_server pr_server; /* opaque */

typedef struct {
    int32_t max_resident; /* cap on resident requests (>= 1) */
    int32_t n_streams;    /* HIP streams shared by resident requests (1..32) */
    uint32_t flags;       /* 0 or PR_SERVER_RAGGED_F */
    int32_t max_queued;   /* waiting (submitted, not yet admitted) requests held at
                             once; 0 = no bound.  Beyond it pr_server_submit
                             refuses the request with PR_EBUSY (load shedding). */
} pr_server_options;
#define PR_SERVER_RAGGED_F 1u

typedef struct {
    int32_t status;        /* pr_status of the solve */
    int32_t iters;         /* Parareal iterations K */
    double last_increment; /* max increment of the last iteration */
    double latency_ms;     /* submit -> result written (host clock) */
    double queue_ms;       /* submit -> admission */
    uint64_t workspace_bytes;
    int32_t coarse_fallback; /* 1: the neural G diverged and the solve restarted on
                                the LOD propagator (PR_G_FNO requests) */
    int32_t reserved_;
} pr_request_info;

/* Workspace a request needs inside the arena (0 when the arguments are invalid). */
uint64_t pr_server_footprint(const pr_grid* grid, const pr_options* opt);
/* arena: device pointer, 256-byte aligned, owned by the caller. */
pr_status pr_server_create(void* arena, uint64_t arena_bytes, const pr_server_options* opt,
                           pr_server** out);
/* Queue one solve; v_out: device pointer to n*n doubles, written when the request
 * completes.  Arguments are validated here (PR_EINVAL / PR_EUNSTABLE); a request
 * larger than the whole arena is rejected with PR_ENOMEM, and a request that
 * finds max_queued requests already waiting with PR_EBUSY (nothing is queued;
 * pr_server_rejected counts these refusals).  *id_out identifies it. */
pr_status pr_server_submit(pr_server* sv, const pr_grid* grid, const pr_model* model,
                           const pr_payoff* payoff, const pr_options* opt, double* v_out,
                           int64_t* id_out);
/* One non-blocking scheduling pass.  Counts are written when the pointers are
 * non-NULL.  Returns the first device or setup error of the pass (the request
 * concerned is retired with that status); a solve's own outcome (PR_ENOTCONV,
 * PR_ENONFINITE) is only the request's status in pr_server_poll. */
pr_status pr_server_progress(pr_server* sv, int32_t* n_resident, int32_t* n_queued,
                             int32_t* n_done);
/* *done = 1 once the request's result is written; info (may be NULL) is filled then. */
pr_status pr_server_poll(pr_server* sv, int64_t id, int32_t* done, pr_request_info* info);
/* Peak resident requests and peak arena bytes in use since creation. */
pr_status pr_server_peaks(const pr_server* sv, int32_t* peak_resident, uint64_t* peak_bytes);
/* Submissions refused with PR_EBUSY since creation. */
pr_status pr_server_rejected(const pr_server* sv, int64_t* n_rejected);
/* The neural operator of PR_G_FNO requests (Sec. 3.4; the network, its base
 * and output scale as created by pr_fno_create): such submissions are refused
 * with PR_EMODEL while none is attached, and the grid must suit the operator as
 * for parareal_attach_fno.  Every PR_G_FNO request runs on the server's first
 * stream, so the operator's activation workspace serves one request at a time;
 * the caller does not use the handle elsewhere while such requests are queued
 * or resident, and replacing or clearing it (f = NULL) then gives PR_EINVAL.
 * A request whose neural G diverges (a non-finite value, or two increments in
 * a row growing) restarts on the LOD propagator as parareal_solve does, unless
 * it carries PR_FLAG_NO_FALLBACK (pr_request_info.coarse_fallback). */
pr_status pr_server_attach_fno(pr_server* sv, pr_fno* f);
/* PR_SERVER_RAGGED_F: progress passes that issued shared fine sweeps, the
 * shared step launches, and the request entries those launches carried
 * (entries / launches = requests per launch).  Zeros without the flag; the
 * pointers may be NULL. */
pr_status pr_server_ragged_stats(const pr_server* sv, int64_t* ticks, int64_t* launches,
                                 int64_t* entries);
/* Blocks until all submitted work has drained, then releases the streams. */
pr_status pr_server_destroy(pr_server* sv);

/* ---------------------------------------------------------------------------
 * Fourier neural operator (Sec. 3.4) and its training with a PDE-residual
 * loss (Sec. 3.5).  Architecture: lift 7 -> 64 -> 32 with GELU, four Fourier
 * layers of width 32 (truncated DFT to modes kx in {0..11, -12..-1},
 * ky in {0..11}, a complex 32 x 32 multiplier per mode, inverse DFT, plus a
 * pointwise 32 x 32 path and bias, GELU after all but the last), projection
 * 32 -> 128 -> 1 with GELU, on a 64 x 64 grid.  GELU is the exact erf form.
 *
 * Per sample the input is one 64 x 64 plane w (x index major, y contiguous)
 * and four parameters meta = (sigma1, sigma2, rho, r); the network sees the
 * channels [w, sigma1, sigma2, rho, r, x/63, y/63] and returns one plane.
 *
 * Parameters are one flat FP32 vector of pr_fno_param_count() values, blocks
 * in this order (row-major within a block, "in x out" for dense weights):
 *   L1 (7,64) l1 (64) L2 (64,32) l2 (32),
 *   per layer: Rr (24,12,32,32) Ri (24,12,32,32) W (32,32) b (32)
 *              (multiplier of mode (kx index, ky) from input to output channel),
 *   P1 (32,128) p1 (128) P2 (128,1) p2 (1).
 *
 * A training pair is four consecutive 64 x 64 FP32 planes
 * [w_in, B1, V_in, V_tgt] (see pr_fno_loss).  The prediction of a pair is
 * V1 = B1 + w_in + out_scale * out (base PR_FNO_BASE_IDENTITY) or
 * V1 = B1 + out_scale * out (the other bases; with PR_FNO_BASE_LOD the pair's
 * B1 plane carries the LOD prediction) on the interior (the ring of the
 * network's output is ignored), and its loss is the mean over the 62 x 62 interior of
 * (V1 - V_tgt)^2 plus lam times the mean of R^2, where R is the discrete
 * Crank-Nicolson residual (V1 - V_in) - dT L_h((V1 + V_in) / 2) of the
 * operator of Eq. (fd) on the 64 x 64 grid (node (i, j) at index form i, j).
 *
 * Precision: PR_FNO_FP32 runs every contraction in FP32; PR_FNO_BF16 runs the
 * channel contractions (lift, pointwise, per-mode multipliers, projection and
 * their gradients) on bf16 matrix cores with FP32 accumulation, the DFTs in
 * FP32.  Master weights, gradients and Adam moments are FP32.
 *
 * All buffers are device pointers unless marked host.  An FNO handle owns
 * nothing but its caller-provided workspace (which holds the parameters,
 * gradients, Adam moments and the activations of up to max_batch samples);
 * its calls are enqueued on the stream given at create; a handle is used by
 * one caller at a time.
 * ------------------------------------------------------------------------- */
#define PR_FNO_GRID 64
#define PR_FNO_WIDTH 32
#define PR_FNO_MODES 12
#define PR_FNO_LAYERS 4
#define PR_FNO_CIN 7
#define PR_FNO_LIFT 64
#define PR_FNO_PROJ 128
#define PR_FNO_MAX_BATCH 512

enum { PR_FNO_FP32 = 0, PR_FNO_BF16 = 1 };

/* What the network's (scaled) output is added to, on the 62 x 62 interior of
 * the operator grid, to give the restricted state after the slice:
 *   PR_FNO_BASE_ZERO     nothing: the network predicts the new w;
 *   PR_FNO_BASE_IDENTITY w_in: the network predicts the change of w;
 *   PR_FNO_BASE_LOD      the LOD implicit propagator (PR_G_LOD's scheme) run on
 *                        the 64 x 64 grid itself over the slice (coarse_steps
 *                        steps, default 4) from B(tau_n) + w_in: the network
 *                        predicts the correction to that cheap, stable step;
 *   PR_FNO_BASE_FINE_LOD the LOD propagator on the fine grid itself (coarse_steps
 *                        steps, default 1): G(u) = LOD(u) + P_s(out_scale * FNO(w)),
 *                        the network predicts the restricted correction F - LOD. */
enum { PR_FNO_BASE_ZERO = 0, PR_FNO_BASE_IDENTITY = 1, PR_FNO_BASE_LOD = 2,
       PR_FNO_BASE_FINE_LOD = 3 };


typedef struct {
    int32_t max_batch;      /* samples per forward / training step, 1..PR_FNO_MAX_BATCH */
    int32_t precision;      /* PR_FNO_*: precision of the inference a solver's coarse propagator runs */
    double out_scale;       /* prediction = out_scale * network output, > 0 */
    int32_t base;           /* PR_FNO_BASE_*: what the prediction is added to */
    int32_t pad_;
} pr_fno_config;

/* Number of FP32 parameters (host only). */
uint64_t pr_fno_param_count(void);
/* Workspace bytes for max_batch samples; 0 when out of range (host only). */
uint64_t pr_fno_workspace_bytes(int32_t max_batch);
/* Create; ws: device, 256-byte aligned, >= pr_fno_workspace_bytes(max_batch),
 * borrowed until destroy.  Parameters start undefined: call pr_fno_set_params.
 * Errors: PR_EINVAL (config), PR_ENOMEM (workspace too small), PR_EDEVICE. */
pr_status pr_fno_create(const pr_fno_config* cfg, void* ws, uint64_t bytes, void* hip_stream,
                        pr_fno** out);
/* Copy the flat parameter vector in from / out to a device buffer; set also
 * clears the Adam moments. */
pr_status pr_fno_set_params(pr_fno* f, const float* src);
pr_status pr_fno_get_params(pr_fno* f, float* dst);
/* Copy the gradient vector of the last pr_fno_backward to a device buffer. */
pr_status pr_fno_get_grads(pr_fno* f, float* dst);
/* out (batch x 64 x 64) = network(w (batch x 64 x 64), meta (batch x 4)). */
pr_status pr_fno_forward(pr_fno* f, const float* w, const float* meta, int32_t batch,
                         int32_t precision, float* out);
/* Gradients of sum(gout * out) with respect to the parameters, for the
 * activations of the last pr_fno_forward (same batch and precision); the
 * gradient vector is overwritten. */
pr_status pr_fno_backward(pr_fno* f, const float* gout);
/* Loss of batch pairs (batch x 4 x 64 x 64) against the prediction `pred`
 * (batch x 64 x 64, scaled by `scale`, added to w_in when the handle's base
 * is PR_FNO_BASE_IDENTITY); gpred (may be NULL) receives
 * dLoss/dpred (zero on the ring); host_loss (host, may be NULL; the call then
 * synchronises) receives [loss, data term, residual term]. */
pr_status pr_fno_loss(pr_fno* f, const float* pred, const float* pairs, const float* meta,
                      int32_t batch, double scale, double dT, double lam, float* gpred,
                      double* host_loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the current
 * gradients; step counts from 1. */
pr_status pr_fno_adam(pr_fno* f, double lr, int32_t step);
/* Forward, loss (scale = out_scale), backward and Adam on the pairs
 * idx[0..batch) (device int32 indices into pairs (n_pairs x 4 x 64 x 64) and
 * meta (n_pairs x 4); an index outside [0, n_pairs) is clamped into it).
 * host_loss as in pr_fno_loss. */
pr_status pr_fno_train_step(pr_fno* f, const float* pairs, const float* meta, int64_t n_pairs,
                            const int32_t* idx, int32_t batch, double dT, double lam, double lr,
                            int32_t step, int32_t precision, double* host_loss);
/* Weight files: the trained network reused without retraining, across
 * processes and runs (Sec. 4.4 and Sec. 4.5 apply the trained operator to other
 * resolutions and parameters without retraining it).  A file holds a 96-byte
 * header (magic "PRFNOW01", version, the architecture constants above, base,
 * inference precision, out_scale, parameter count, a caller-chosen 64-bit hash
 * of the training configuration, an FNV-1a 64 checksum of header and weights)
 * followed by the flat FP32 master weights.
 *
 * pr_fno_save: copies the handle's parameters to the host (synchronises its
 * stream) and writes path atomically (path.tmp, then rename).  PR_EMODEL when
 * the file cannot be written.
 * pr_fno_check_file (host only, no GPU): validates a file (magic, version,
 * architecture, parameter count, field ranges, checksum, finite weights, no
 * trailing bytes) and fills info (may be NULL).  PR_EMODEL, with no further
 * detail, for a missing, truncated, corrupted or incompatible file.
 * pr_fno_load: validates as pr_fno_check_file, then requires the file's base and
 * out_scale to equal the handle's configuration (PR_EMODEL otherwise, with a
 * message in pr_fno_last_error), copies the weights in and clears the Adam
 * moments as pr_fno_set_params does; synchronises the handle's stream.  The
 * handle is unchanged when the call fails. */
typedef struct {
    uint32_t version;
    int32_t base;         /* PR_FNO_BASE_* the weights were trained for */
    int32_t precision;    /* PR_FNO_* inference precision of the saving handle */
    int32_t pad_;
    double out_scale;
    uint64_t param_count;
    uint64_t train_hash;  /* the value given to pr_fno_save */
} pr_fno_file_info;
pr_status pr_fno_save(pr_fno* f, const char* path, uint64_t train_hash);
pr_status pr_fno_check_file(const char* path, pr_fno_file_info* info);
pr_status pr_fno_load(pr_fno* f, const char* path, pr_fno_file_info* info);
pr_status pr_fno_destroy(pr_fno* f);
const char* pr_fno_last_error(const pr_fno* f);

const char* parareal_strerror(pr_status st);
const char* parareal_last_error(const pr_solver* s);
int32_t parareal_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PARAREAL_H */
