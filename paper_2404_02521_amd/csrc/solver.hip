// solver.hip -- host driver and C ABI of the Parareal solver (include/parareal.h).
//
// One solve on one GPU:
//   init   : U_0 = payoff; coarse sweep c_{n+1} = Gc(c_n); U_{n+1} = P(c_{n+1})
//   iter k : F sweep over the active slices n = k..N-1 (all slices in one
//            launch per explicit step), coarse chain over n = k..N-1,
//            correction + norm over n = k..N-1, 24-byte read-back of the norms.
// Slices n <= k are converged after iteration k (U^k_n = F^n u0) and are
// neither propagated nor corrected again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/parareal.h"
#include "internal.hpp"

namespace pr {
hipError_t launch_fine_prep(const double*, float*, float*, const StepArgs&, hipStream_t);
hipError_t launch_fine_tb_f32(const float*, const float*, float*, const float*, const StepArgs&, int,
                              hipStream_t);
hipError_t launch_fine_tb_f64(const double*, double*, const double*, const StepArgs&, int,
                              hipStream_t);
hipError_t launch_row_weights(void*, int, const Coef&, double, int, hipStream_t);
hipError_t launch_fine_tb_batch(const TbBatch&, bool, int, hipStream_t);
void tb_geometry(StepArgs&, int, int, int, int, int);
int krylov_blocks_per_slice(const Grid&, int);
hipError_t krylov_step(double*, const KrylovBufs&, const KrylovArgs&, int, int, int*, int*,
                       hipStream_t);
hipError_t chain_set_lds(int);
hipError_t launch_chain(const double*, double*, double*, double*, float*, const ChainArgs&,
                        hipStream_t);
hipError_t launch_gather_coincident(const double*, const void*, double*, const Grid&, int, int,
                                    int, int, int, hipStream_t);
int chain_lds_bytes(int, int);
bool chain_state_in_lds(int, int);
hipError_t launch_correct(const double*, const void*, const double*, const double*, double*,
                          double*, unsigned long long*, const Grid&, int, int, int, int, int,
                          int, int, hipStream_t);
hipError_t launch_zero_red(unsigned long long*, hipStream_t);
hipError_t launch_payoff(double*, const Grid&, const Bc&, hipStream_t);
hipError_t launch_prolong(const double*, double*, const Grid&, int, int, int, int, hipStream_t);
hipError_t launch_pack(const double*, double*, const Grid&, hipStream_t);
hipError_t launch_unpack(const double*, double*, const Grid&, const Bc&, double, hipStream_t);
hipError_t launch_finalize(const double*, const float*, double*, const Grid&, hipStream_t);
hipError_t launch_lod_slice(const double*, double*, double*, double*, double*, const Grid&,
                            const Coef&, const Bc&, double, double, int, hipStream_t);
hipError_t lod_set_lds(int);
hipError_t launch_lift(const double*, double*, const Grid&, const Bc&, double, double, hipStream_t);
hipError_t launch_fno_in(const double*, float*, float*, const Bc&, hipStream_t);
hipError_t launch_fno_out(const double*, const float*, double, double*, hipStream_t);
hipError_t launch_pair(const double*, const double*, const double*, float*, const Bc&, double,
                       double, double, hipStream_t);
void sine_transfer_matrices(int nf, std::vector<double>& R, std::vector<double>& P);
namespace fno {
hipError_t infer(pr_fno* f, const float* w, const float* meta, int B, float* out, hipStream_t st);
double out_scale(const pr_fno* f);
int base(const pr_fno* f);
hipError_t gemm_f64(const double* A, long long ars, long long acs, const double* B, long long brs,
                    long long bcs, double* C, long long crs, int M, int N, int K, double beta,
                    hipStream_t st);
}  // namespace fno
constexpr int kFnoInt = 62;   // interior nodes per side of the 64 x 64 operator grid
}  // namespace pr

using namespace pr;

namespace {

constexpr uint64_t kAlign = 256;
uint64_t al(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

Grid make_grid(int n) {
    Grid g;
    g.n = n;
    g.nin = n - 2;
    g.pitch = (g.nin + kWave - 1) / kWave * kWave;
    g.stride = (long long)g.nin * g.pitch;
    return g;
}

// Gershgorin bound of explicit Euler for the operator of Eq. (fd) in index
// form: row (i, j) has centre c = -(2 alpha + 2 beta + r) and radius
// R = |alpha + mu| + |alpha - mu| + |beta + nu| + |beta - nu| + 4 |gamma|;
// |1 + dt lambda| <= 1 for every eigenvalue when dt <= 2 / (|c| + R).
double gershgorin_dt(int n, const pr_model& m) {
    const double a1 = 0.5 * m.sigma1 * m.sigma1, a2 = 0.5 * m.sigma2 * m.sigma2;
    const double g12 = 0.25 * m.rho * m.sigma1 * m.sigma2, hr = 0.5 * m.r;
    double worst = 0.0;
    for (int i = 1; i < n - 1; ++i) {
        const double al_ = a1 * i * i, mu = hr * i;
        const double rx = std::fabs(al_ + mu) + std::fabs(al_ - mu);
        for (int j = 1; j < n - 1; ++j) {
            const double be = a2 * j * j, nu = hr * j;
            const double ga = g12 * i * j;
            const double v = 2.0 * al_ + 2.0 * be + m.r + rx + std::fabs(be + nu) +
                             std::fabs(be - nu) + 4.0 * std::fabs(ga);
            worst = std::max(worst, v);
        }
    }
    return 2.0 / worst;
}

struct Layout {
    uint64_t Ua, Ub, dA, dB, Lb, wA, wB, wt, Gold, dcor, cst, lbc, Gf, tA, tB, tLb, twA, twB, tg, red,
        lw0, lw1, lwb, Sr, Sp, fwf, fT, fwc, fwc1, fTp, fin, fmeta, fout, fvc0, fvc1, flw0, flw1,
        flwb, fwb, gst, foldc, kB, kR, kRH, kP0, kP1, kV0, kV1, kS, kT, kpA, kpB, kpC, ksc, kdone, total;
};

bool valid_basic(const pr_grid* g, const pr_options* o, std::string* why) {
    auto fail = [&](const char* m) { if (why) *why = m; return false; };
    if (!g || !o) return fail("null argument");
    if (g->n < 5) return fail("grid.n must be >= 5");
    if (!(g->s_max > 0.0)) return fail("grid.s_max must be > 0");
    if (o->n_slices < 1 || o->n_slices > PR_MAX_SLICES) return fail("n_slices out of range");
    if (o->precision != PR_FP64 && o->precision != PR_FP32) return fail("unknown precision");
    if (o->coarse_kind != PR_G_NUMERICAL && o->coarse_kind != PR_G_FINE &&
        o->coarse_kind != PR_G_LOD && o->coarse_kind != PR_G_FNO &&
        o->coarse_kind != PR_G_IMPLICIT)
        return fail("unknown coarse_kind");
    if (o->coarse_kind == PR_G_IMPLICIT && o->precision != PR_FP64)
        return fail("PR_G_IMPLICIT runs in PR_FP64");
    if (o->coarse_kind == PR_G_IMPLICIT && (o->flags & PR_FLAG_GRAPH))
        return fail("PR_G_IMPLICIT cannot be graph-captured");
    if (o->coarse_kind == PR_G_FNO && g->n < 64)
        return fail("PR_G_FNO needs at least 64 nodes per side");
    if (o->coarse_kind == PR_G_NUMERICAL) {
        if (o->coarse_n < 3) return fail("coarse_n must be >= 3");
        if ((g->n - 1) % (o->coarse_n - 1) != 0)
            return fail("(n-1) must be divisible by (coarse_n-1)");
        if (o->coarse_n > kChainMaxN) return fail("coarse_n above 257 is not supported");
    }
    if (o->coarse_kind == PR_G_LOD && g->n - 2 > 2048)
        return fail("PR_G_LOD supports up to 2050 nodes per side");
    if (o->fine_steps < 0 || o->coarse_steps < 0) return fail("negative step count");
    if ((o->fine_steps == 0 || o->coarse_steps == 0) && !(o->cfl > 0.0 && o->cfl <= 1.0))
        return fail("cfl must be in (0, 1] when a step count is planned");
    if (o->max_iters < 0) return fail("max_iters must be >= 0");
    if (!(o->tol >= 0.0)) return fail("tol must be >= 0");
    if (o->fine_scheme != PR_FINE_EXPLICIT && o->fine_scheme != PR_FINE_IMPLICIT)
        return fail("unknown fine_scheme");
    if (o->fine_scheme == PR_FINE_IMPLICIT) {
        if (o->precision != PR_FP64) return fail("PR_FINE_IMPLICIT runs in PR_FP64");
        if (o->fine_steps < 1) return fail("PR_FINE_IMPLICIT needs fine_steps >= 1");
        if (o->flags & PR_FLAG_GRAPH) return fail("PR_FINE_IMPLICIT cannot be graph-captured");
    }
    if (o->fine_scheme == PR_FINE_IMPLICIT || o->coarse_kind == PR_G_IMPLICIT) {
        if (!(o->krylov_tol >= 0.0 && o->krylov_tol < 1.0)) return fail("krylov_tol must be in [0, 1)");
        if (o->krylov_max_iters < 0) return fail("krylov_max_iters must be >= 0");
    }
    return true;
}

Layout layout(const pr_grid* g, const pr_options* o) {
    const Grid fg = make_grid(g->n);
    const uint64_t N = o->n_slices;
    const uint64_t sd = (uint64_t)fg.stride * 8, sf = (uint64_t)fg.stride * 4;
    const bool fp32 = o->precision == PR_FP32;
    const bool gfine = o->coarse_kind == PR_G_FINE;
    const bool lod = o->coarse_kind == PR_G_LOD;
    const bool fno = o->coarse_kind == PR_G_FNO;
    const bool gimp = o->coarse_kind == PR_G_IMPLICIT;
    const bool fineg = gfine || lod || fno || gimp;   // G returns fine-grid states (chain over fine slices)
    const uint64_t nc = fineg ? 0 : (uint64_t)o->coarse_n;
    Layout L{};
    uint64_t p = 0;
    auto take = [&](uint64_t bytes) { uint64_t at = p; p = al(p + bytes); return at; };
    L.Ua = take((N + 1) * sd);
    L.Ub = take((N + 1) * sd);
    L.dA = take(fp32 ? N * sf : 0);
    L.dB = take(fp32 ? N * sf : 0);
    L.Lb = take(fp32 ? N * sf : 0);
    L.wA = take(fp32 ? 0 : N * sd);
    L.wB = take(fp32 ? 0 : N * sd);
    L.wt = take((uint64_t)g->n * 4 * 8);   // row weights of the step kernel
    L.Gold = take(N * nc * nc * 8);
    L.dcor = take(N * nc * nc * 8);
    L.cst = take(nc * nc * 8);
    L.foldc = take(N * nc * nc * 8);
    L.lbc = take(nc * nc * 4);
    // chain state in global memory when it does not fit in LDS
    L.gst = take(nc > 0 && !chain_state_in_lds((int)nc, fp32 ? 1 : 0) ? 2 * nc * nc * (fp32 ? 4 : 8)
                                                                       : 0);
    L.Gf = take(fineg ? N * sd : 0);
    L.tA = take(gfine && fp32 ? sf : 0);
    L.tB = take(gfine && fp32 ? sf : 0);
    L.tLb = take(gfine && fp32 ? sf : 0);
    L.twA = take((gfine || gimp) && !fp32 ? sd : 0);
    L.twB = take(gfine && !fp32 ? sd : 0);
    L.tg = take(fineg ? sd : 0);
    L.lw0 = take(lod || fno ? sd : 0);   // PR_G_FNO falls back to LOD
    L.lw1 = take(lod || fno ? sd : 0);
    L.lwb = take(lod || fno ? sd : 0);
    const uint64_t nf = fg.nin, mi = kFnoInt;
    L.Sr = take(fno ? mi * nf * 8 : 0);
    L.Sp = take(fno ? nf * mi * 8 : 0);
    L.fwf = take(fno ? sd : 0);
    L.fT = take(fno ? mi * nf * 8 : 0);
    L.fwc = take(fno ? mi * mi * 8 : 0);
    L.fwc1 = take(fno ? mi * mi * 8 : 0);
    L.fTp = take(fno ? nf * mi * 8 : 0);
    L.fin = take(fno ? 64 * 64 * 4 : 0);
    L.fmeta = take(fno ? 16 : 0);
    L.fout = take(fno ? 64 * 64 * 4 : 0);
    L.fvc0 = take(fno ? mi * mi * 8 : 0);   // PR_FNO_BASE_LOD: the 64 x 64 grid's own states
    L.fvc1 = take(fno ? mi * mi * 8 : 0);
    L.flw0 = take(fno ? mi * mi * 8 : 0);
    L.flw1 = take(fno ? mi * mi * 8 : 0);
    L.flwb = take(fno ? mi * mi * 8 : 0);
    L.fwb = take(fno ? mi * mi * 8 : 0);
    // implicit F: BiCGStab vectors (N slices each), partial sums (at most one
    // workgroup per row), per-slice scalars and the finished-slice counter
    const bool imp = o->fine_scheme == PR_FINE_IMPLICIT || gimp;
    L.kR = take(imp ? N * sd : 0);
    L.kB = take(imp ? N * sd : 0);
    L.kRH = take(imp ? N * sd : 0);
    L.kP0 = take(imp ? N * sd : 0);
    L.kP1 = take(imp ? N * sd : 0);
    L.kV0 = take(imp ? N * sd : 0);
    L.kV1 = take(imp ? N * sd : 0);
    L.kS = take(imp ? N * sd : 0);
    L.kT = take(imp ? N * sd : 0);
    L.kpA = take(imp ? N * nf * 8 : 0);
    L.kpB = take(imp ? N * nf * 16 : 0);
    L.kpC = take(imp ? N * nf * 16 : 0);
    L.ksc = take(imp ? N * sizeof(KScal) : 0);
    L.kdone = take(imp ? 64 : 0);
    L.red = take(64);
    L.total = p;
    return L;
}

}  // namespace

struct pr_solver {
    pr_grid grid{};
    pr_model model{};
    pr_payoff pay{};
    pr_options opt{};
    hipStream_t stream = nullptr;
    Grid fg{};
    Coef coef{};
    Bc bcf{}, bcc{};
    int N = 0, nc = 0, q = 1, mF = 0, mG = 0, maxit = 0;
    double dT = 0, dtF = 0, dtG = 0, ring_max_T = 0;
    bool fp32 = false, fineg = false, lod = false, fnog = false;
    pr_fno* fno = nullptr;             // PR_G_FNO: the attached operator (borrowed)
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    Layout L{};
    hipEvent_t ev[6]{};
    bool events = false;
    std::vector<hipEvent_t> step_ev;   // PR_FLAG_TIME_STEPS: a pair per step launch
    int step_ev_used = 0;
    int rows_override = 0;             // PR_STEP_ROWS (tuning): rows per wavefront chunk
    // Launch shape of the step kernel (measured on the 513^2 x 64 Parareal
    // solves with the phased chain overlap, whose sweeps cover 1 to 42
    // slices): six fused steps, five for sweeps of at most 16 slices and at
    // most kSmallSweepPoints interior nodes, at most 4096 wavefronts per
    // launch in row chunks of at least 24 rows (at 2049^2 x 32 slices, whose
    // row chunks reach the 128-row cap, six steps stay 9% faster than five).
    int fuse = 6;                      // explicit steps per launch (PR_STEP_FUSE, 1..8)
    int fuse_small = 5;                // ... when a sweep has few slices (PR_STEP_FUSE_SMALL)
    int small_count = 16;              // "few": at most this many slices (PR_STEP_SMALL_COUNT;
                                       // 0: every sweep uses `fuse`)
    bool weights_ready = false;        // row-weight table of the step kernel written
    bool implicit = false;             // PR_FINE_IMPLICIT
    bool implicit_g = false;           // PR_G_IMPLICIT
    int* kry_pin = nullptr;            // BiCGStab: 2 pinned slots for the finished-slice count
    hipEvent_t kry_ev[2]{};            // ... and their events (polls read one round late)
    int64_t kry_iters = 0;             // BiCGStab iterations of this call (summed over steps)
    int kry_max = 0;                   // most iterations of one step
    int kry_unconv = 0;                // slice-steps that stopped unconverged
    int wave_target = 4096;            // wavefronts a step launch aims for (PR_STEP_WAVES)
    int min_rows = 24;                 // shortest row chunk of a step launch (PR_STEP_MINROWS)
    int step_fit = 1;                  // PR_STEP_FIT: at most wave_target wavefronts per launch
    std::map<int, int64_t> graph_launches;   // step launches captured in graph k
    std::map<int, double> graph_bytes;
    int ev_every = 8;                  // PR_FLAG_TIME_STEPS: step launches per timed run
    int64_t timed_launches = 0;        // launches bracketed by events in this call
    double timed_bytes = 0;            // their algorithmic bytes
    int64_t sweep_launches = 0;        // step launches of the last fine_sweep
    double sweep_bytes = 0;            // their algorithmic bytes
    bool graph = false;                // PR_FLAG_GRAPH
    hipStream_t cap_stream = nullptr;  // capture vehicle (never executes work)
    // overlapped chain (see PR_FLAG_SERIAL_CHAIN): second stream, one event per
    // slice group plus the join, group count and smallest group
    bool pipe = false;
    hipStream_t chain_stream = nullptr;
    static constexpr int kPipeMaxGroups = 8;
    hipEvent_t pipe_ev[kPipeMaxGroups + 1]{};
    int pipe_groups = 2;               // PR_PIPE_GROUPS (1..8; 1 = off)
    int pipe_min = 16;                 // PR_PIPE_MIN: fewest slices per group
    int pipe_mode = 1;                 // PR_PIPE_MODE: 0 equal groups, 1 phases with an early sweep
    int pipe_split = 67;               // PR_PIPE_SPLIT: percent of a phase's slices in group 0
    int pipe_B = -1;                   // phased overlap: the current phase's group boundary
    int early_k = -1;                  // iteration whose first group was swept early
    const void* early_fold = nullptr;  // that sweep's result (as fine_sweep returns it)
    int pipe_min_rows = 24;            // PR_PIPE_MINROWS: shortest row chunk of a grouped sweep
    bool bracket_sweep = true;         // fine_sweep records ev[4] / ev[5] itself
    std::map<int, hipGraphExec_t> graphs;   // key -1: initial sweep, k: iteration k
    std::map<int, hipGraph_t> graph_defs;
    std::string err;

    template <class T> T* at(uint64_t off) { return reinterpret_cast<T*>(ws + off); }
    double* U(int which) { return at<double>(which ? L.Ub : L.Ua); }
    unsigned long long* red() { return at<unsigned long long>(L.red); }
};

namespace {

constexpr long long kSmallSweepPoints = 32LL * 511 * 511;   // 32 slices of 513^2

#define HIPCHK(expr)                                                                 \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            s->err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
            return PR_EDEVICE;                                                       \
        }                                                                            \
    } while (0)

StepArgs step_args(pr_solver* s, const Grid& g, const Bc& bc, double dt, int first, int count,
                   int step) {
    StepArgs a{};
    a.g = g;
    a.c = s->coef;
    a.bc = bc;
    a.dt = dt;
    a.dT = s->dT;
    a.first = first;
    a.count = count;
    a.step = step;
    a.nstrips = (g.nin + kWave - 1) / kWave;
    // rows per wavefront: enough wavefronts to fill 256 CUs several times over
    const long long per_slice_cols = (long long)a.nstrips * count;
    int rows = (int)std::min<long long>(64, std::max<long long>(8, (long long)g.nin * per_slice_cols / 16384));
    if (s->rows_override > 0) rows = std::min(s->rows_override, g.nin);
    a.rows = rows;
    a.nchunks = (g.nin + rows - 1) / rows;
    return a;
}

// Launch geometry of the temporally blocked step kernel (tb_geometry in
// kernels.hip): strips of 64 - 2S output columns, row chunks sized so that a
// launch has enough wavefronts to fill the chip.
StepArgs tb_args(pr_solver* s, const Grid& g, double dt, int first, int count, int step, int S) {
    StepArgs a = step_args(s, g, s->bcf, dt, first, count, step);
    tb_geometry(a, S, s->wave_target, s->min_rows, s->rows_override, s->step_fit);
    return a;
}

// Implicit-Euler F (Eq. (fd)) over slices [first, first+count): the FP64
// states start as copies of the bases and are stepped in place, each step a
// BiCGStab solve of every slice at once (tmp: the single-slice temporaries).
pr_status implicit_sweep(pr_solver* s, const double* Ubase, int first, int count, bool tmp,
                         const double** wres, double* step_ms, double dt, int steps) {
    const Grid& g = s->fg;
    if (step_ms && s->events) HIPCHK(hipEventRecord(s->ev[4], s->stream));
    const long long off = tmp ? 0 : (long long)first * g.stride;
    double* X = s->at<double>(tmp ? s->L.twA : s->L.wA) + off;
    HIPCHK(hipMemcpyAsync(X, Ubase + (long long)first * g.stride,
                          (size_t)count * g.stride * sizeof(double), hipMemcpyDeviceToDevice,
                          s->stream));
    KrylovBufs b{};
    b.B = s->at<double>(s->L.kB);
    b.R = s->at<double>(s->L.kR);
    b.RH = s->at<double>(s->L.kRH);
    b.P[0] = s->at<double>(s->L.kP0);
    b.P[1] = s->at<double>(s->L.kP1);
    b.V[0] = s->at<double>(s->L.kV0);
    b.V[1] = s->at<double>(s->L.kV1);
    b.S = s->at<double>(s->L.kS);
    b.T = s->at<double>(s->L.kT);
    b.partA = s->at<double>(s->L.kpA);
    b.partB = s->at<double>(s->L.kpB);
    b.partC = s->at<double>(s->L.kpC);
    b.sc = s->at<KScal>(s->L.ksc);
    b.ndone = s->at<int>(s->L.kdone);
    b.hpoll = s->kry_pin;
    b.pev[0] = s->kry_ev[0];
    b.pev[1] = s->kry_ev[1];
    KrylovArgs a{};
    a.g = g;
    a.c = s->coef;
    a.bc = s->bcf;
    a.dt = dt;
    a.dT = s->dT;
    a.first = first;
    a.count = count;
    a.nblk = krylov_blocks_per_slice(g, count);
    a.rows = (g.nin + a.nblk - 1) / a.nblk;
    a.nblk = (g.nin + a.rows - 1) / a.rows;
    const double tol = s->opt.krylov_tol > 0.0 ? s->opt.krylov_tol : 1e-12;
    a.tol2 = tol * tol;
    // default cap: Jacobi-preconditioned BiCGStab on the stiffest steps seen
    // (dt |L_h| ~ 1e3 at 301^2) takes up to ~3 n iterations, erratically
    const int maxit = s->opt.krylov_max_iters > 0 ? s->opt.krylov_max_iters
                                                   : std::max(1000, 10 * g.nin);
    for (int q = 0; q < steps; ++q) {
        a.step = q;
        int done = 0, its = 0;
        HIPCHK(krylov_step(X, b, a, maxit, 8, &done, &its, s->stream));
        s->kry_iters += its;
        s->kry_max = std::max(s->kry_max, its);
        s->kry_unconv += count - done;
        // a slice that stopped by breakdown counts as finished in `done`; its
        // residual is checked here so that it is reported
        std::vector<KScal> hs((size_t)count);
        HIPCHK(hipMemcpyAsync(hs.data(), b.sc, hs.size() * sizeof(KScal), hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        for (const KScal& k : hs)
            if (k.breakdown && !(k.rr <= a.tol2 * k.bb)) s->kry_unconv += 1;
    }
    if (step_ms && s->events) HIPCHK(hipEventRecord(s->ev[5], s->stream));
    *wres = X - off;
    return PR_OK;
}

// F over slices [first, first+count) from base U (interior layout, slice
// `first` at U + first*stride).  FP32: result increments land in *dres (dA or
// dB); FP64: the state lands in *wres.  `tmp` selects the single-slice
// temporaries (G = F chain) instead of the per-slice buffers.
pr_status fine_sweep(pr_solver* s, const double* Ubase, int first, int count, bool tmp,
                     const float** dres, const double** wres, double* step_ms) {
    const Grid& g = s->fg;
    const long long off = tmp ? 0 : (long long)first * g.stride;
    // optional: another fused-step count for sweeps over few slices (their
    // launches have few wavefronts; off by default, where it measured within
    // 1% of one count for every sweep)
    const bool small = count <= s->small_count &&
                       (long long)count * g.nin * g.nin <= kSmallSweepPoints;
    const int fuse = small ? s->fuse_small : s->fuse;
    if (s->implicit)
        return implicit_sweep(s, Ubase, first, count, tmp, wres, step_ms, s->dtF, s->mF);
    if (!s->weights_ready) {
        // stream-ordered before every step launch of this solver; under graph
        // capture the launch becomes part of the graph (which replays it before
        // its step launches) and the flag stays clear for eager sweeps
        HIPCHK(launch_row_weights(s->at<char>(s->L.wt), g.n, s->coef, s->dtF, s->fp32 ? 1 : 0,
                                  s->stream));
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIPCHK(hipStreamIsCapturing(s->stream, &cs));
        if (cs == hipStreamCaptureStatusNone) s->weights_ready = true;
    }
    // PR_FLAG_TIME_STEPS: runs of ev_every consecutive step launches (a run also
    // ends with the sweep) are bracketed by events; a run's elapsed time over its
    // launches is their launch-to-launch duration, the first launch's dispatch
    // delay spread over the run
    struct RunTimer {
        pr_solver* s;
        bool on;
        int n = 0;
        double bytes = 0;
        bool open = false;
        hipError_t begin() {
            if (!on || open || s->step_ev_used + 2 > (int)s->step_ev.size()) return hipSuccess;
            open = true;
            n = 0;
            bytes = 0;
            return hipEventRecord(s->step_ev[s->step_ev_used], s->stream);
        }
        hipError_t end(double b, bool last) {
            if (!open) return hipSuccess;
            n += 1;
            bytes += b;
            if (n < s->ev_every && !last) return hipSuccess;
            open = false;
            s->step_ev_used += 2;
            s->timed_launches += n;
            s->timed_bytes += bytes;
            return hipEventRecord(s->step_ev[s->step_ev_used - 1], s->stream);
        }
    } rt{s, step_ms != nullptr};
    if (s->fp32) {
        float* A = s->at<float>(tmp ? s->L.tA : s->L.dA) + off;
        float* B = s->at<float>(tmp ? s->L.tB : s->L.dB) + off;
        float* Lb = s->at<float>(tmp ? s->L.tLb : s->L.Lb) + off;
        StepArgs a = step_args(s, g, s->bcf, s->dtF, first, count, 0);
        HIPCHK(launch_fine_prep(Ubase + (long long)first * g.stride, Lb, A, a, s->stream));
        if (step_ms && s->events && s->bracket_sweep) HIPCHK(hipEventRecord(s->ev[4], s->stream));
        for (int q = 1; q < s->mF;) {
            const int S = std::min(fuse, s->mF - q);
            StepArgs b = tb_args(s, g, s->dtF, first, count, q, S);
            HIPCHK(rt.begin());
            HIPCHK(launch_fine_tb_f32(A, Lb, B, s->at<float>(s->L.wt), b, S, s->stream));
            const double bytes = 12.0 * S * (double)count * g.nin * g.nin;
            HIPCHK(rt.end(bytes, q + S >= s->mF));
            s->sweep_launches += 1;
            s->sweep_bytes += bytes;
            std::swap(A, B);
            q += S;
        }
        if (step_ms && s->events && s->bracket_sweep) HIPCHK(hipEventRecord(s->ev[5], s->stream));
        *dres = A - off;
    } else {
        double* A = s->at<double>(tmp ? s->L.twA : s->L.wA) + off;
        double* B = s->at<double>(tmp ? s->L.twB : s->L.wB) + off;
        if (step_ms && s->events && s->bracket_sweep) HIPCHK(hipEventRecord(s->ev[4], s->stream));
        for (int q = 0; q < s->mF;) {
            const int S = std::min(fuse, s->mF - q);
            StepArgs b = tb_args(s, g, s->dtF, first, count, q, S);
            HIPCHK(rt.begin());
            HIPCHK(launch_fine_tb_f64(q == 0 ? Ubase + (long long)first * g.stride : A,
                                      q == 0 ? A : B, s->at<double>(s->L.wt), b, S, s->stream));
            const double bytes = 16.0 * S * (double)count * g.nin * g.nin;
            HIPCHK(rt.end(bytes, q + S >= s->mF));
            s->sweep_launches += 1;
            s->sweep_bytes += bytes;
            if (q > 0) std::swap(A, B);
            q += S;
        }
        if (step_ms && s->events && s->bracket_sweep) HIPCHK(hipEventRecord(s->ev[5], s->stream));
        *wres = A - off;
    }
    return PR_OK;
}

// U_out (one slice) <- F result of slice `slice`.
pr_status fine_result_to_state(pr_solver* s, const double* Ubase_slice, const float* d,
                               const double* w, double* Uout_slice) {
    const Grid& g = s->fg;
    if (s->fp32)
        HIPCHK(launch_finalize(Ubase_slice, d, Uout_slice, g, s->stream));
    else
        HIPCHK(hipMemcpyAsync(Uout_slice, w, (size_t)g.stride * 8, hipMemcpyDeviceToDevice,
                              s->stream));
    return PR_OK;
}

// ---------------------------------------------------------------------------
// Ragged fine sweeps: the F work of several solvers in shared step launches.
// A solver's sweep is prepared on its own stream (row weights, the FP32
// preparation step), then the fused-step launches of all solvers run on one
// stream: per round, each solver takes min(fuse, steps left) steps, and the
// solvers with the same step count and precision share launches of up to
// kTbBatchMax entries.  Each entry keeps its solver's launch geometry, so the
// result is bitwise that of fine_sweep.
// ---------------------------------------------------------------------------
struct RaggedSweep {
    pr_solver* s = nullptr;
    int first = 0, count = 0;
    int q = 0;                  // step index of the next launch's input
    int fuse = 0;               // fused steps per launch
    long long off = 0;          // element offset of slice `first`
    const void* cur = nullptr;  // input of the next launch (the FP64 base at q = 0)
    void* bufA = nullptr;
    void* bufB = nullptr;
    const float* Lb = nullptr;  // FP32 increment form: dt L b
    hipEvent_t done = nullptr;  // recorded on the launch stream after this sweep's last launch
};

// Prepare the sweep of s over slices [first, first+count) from base Ubase (on
// s->stream); the step launches follow in ragged_run.
pr_status ragged_begin(pr_solver* s, const double* Ubase, int first, int count, RaggedSweep* j) {
    const Grid& g = s->fg;
    if (s->implicit) return PR_EINVAL;
    *j = RaggedSweep{};
    j->s = s;
    j->first = first;
    j->count = count;
    j->off = (long long)first * g.stride;
    const bool small = count <= s->small_count &&
                       (long long)count * g.nin * g.nin <= kSmallSweepPoints;
    j->fuse = small ? s->fuse_small : s->fuse;
    if (!s->weights_ready) {
        HIPCHK(launch_row_weights(s->at<char>(s->L.wt), g.n, s->coef, s->dtF, s->fp32 ? 1 : 0,
                                  s->stream));
        s->weights_ready = true;
    }
    if (s->fp32) {
        float* A = s->at<float>(s->L.dA) + j->off;
        float* Lb = s->at<float>(s->L.Lb) + j->off;
        StepArgs a = step_args(s, g, s->bcf, s->dtF, first, count, 0);
        HIPCHK(launch_fine_prep(Ubase + j->off, Lb, A, a, s->stream));
        j->bufA = A;
        j->bufB = s->at<float>(s->L.dB) + j->off;
        j->Lb = Lb;
        j->cur = A;
        j->q = 1;
    } else {
        j->bufA = s->at<double>(s->L.wA) + j->off;
        j->bufB = s->at<double>(s->L.wB) + j->off;
        j->cur = Ubase + j->off;
        j->q = 0;
    }
    return PR_OK;
}

// The step launches of every prepared sweep, on stream st (which must be
// ordered after each ragged_begin); a sweep's `done` event (when set) is
// recorded right after its last launch, so that its solver can go on while
// longer sweeps of the batch still run.  *launches / *entries count the
// shared launches and the entries they carried.
pr_status ragged_run(std::vector<RaggedSweep>& jobs, hipStream_t st, int64_t* launches,
                     int64_t* entries) {
    std::vector<char> finished(jobs.size(), 0);
    auto mark_done = [&]() -> pr_status {
        for (size_t i = 0; i < jobs.size(); ++i) {
            RaggedSweep& j = jobs[i];
            if (finished[i] || j.q < j.s->mF) continue;
            finished[i] = 1;
            if (j.done && hipEventRecord(j.done, st) != hipSuccess) {
                j.s->err = "ragged sweep: hipEventRecord failed";
                return PR_EDEVICE;
            }
        }
        return PR_OK;
    };
    for (;;) {
        const pr_status ms = mark_done();
        if (ms != PR_OK) return ms;
        std::map<std::pair<int, int>, std::vector<size_t>> groups;   // (fp32, S) -> jobs
        for (size_t i = 0; i < jobs.size(); ++i) {
            RaggedSweep& j = jobs[i];
            pr_solver* s = j.s;
            if (j.q >= s->mF) continue;
            const int S = std::min(j.fuse, s->mF - j.q);
            void* out = j.cur == j.bufA ? j.bufB : j.bufA;
            if (s->bcf.kind == PR_BC_EXACT) {
                // out-of-line closed-form ring: the solver's own launch
                StepArgs b = tb_args(s, s->fg, s->dtF, j.first, j.count, j.q, S);
                if (s->fp32)
                    HIPCHK(launch_fine_tb_f32(static_cast<const float*>(j.cur), j.Lb,
                                              static_cast<float*>(out), s->at<float>(s->L.wt), b,
                                              S, st));
                else
                    HIPCHK(launch_fine_tb_f64(static_cast<const double*>(j.cur),
                                              static_cast<double*>(out), s->at<double>(s->L.wt),
                                              b, S, st));
                j.cur = out;
                j.q += S;
                s->sweep_launches += 1;
                continue;
            }
            groups[{s->fp32 ? 1 : 0, S}].push_back(i);
        }
        if (groups.empty()) {
            bool left = false;
            for (const RaggedSweep& j : jobs) left = left || j.q < j.s->mF;
            if (!left) break;
            continue;   // only own launches this round
        }
        for (auto& kv : groups) {
            const bool fp32 = kv.first.first != 0;
            const int S = kv.first.second;
            const std::vector<size_t>& idx = kv.second;
            for (size_t c = 0; c < idx.size(); c += kTbBatchMax) {
                TbBatch b{};
                const size_t ce = std::min(idx.size(), c + (size_t)kTbBatchMax);
                for (size_t e = c; e < ce; ++e) {
                    RaggedSweep& j = jobs[idx[e]];
                    pr_solver* s = j.s;
                    TbEntry& en = b.e[b.n++];
                    en.a = tb_args(s, s->fg, s->dtF, j.first, j.count, j.q, S);
                    en.in = j.cur;
                    en.out = j.cur == j.bufA ? j.bufB : j.bufA;
                    en.lb = fp32 ? j.Lb : nullptr;
                    en.wt = s->at<char>(s->L.wt);
                    en.block0 = b.nblocks;
                    b.nblocks += (en.a.count * en.a.nchunks * en.a.nstrips + kBlock / kWave - 1) /
                                 (kBlock / kWave);
                }
                const hipError_t e = launch_fine_tb_batch(b, fp32, S, st);
                if (e != hipSuccess) {
                    jobs[idx[c]].s->err = std::string("ragged step launch: ") +
                                          hipGetErrorString(e);
                    return PR_EDEVICE;
                }
                for (int e2 = 0; e2 < b.n; ++e2) {
                    RaggedSweep& j = jobs[idx[c + e2]];
                    j.cur = b.e[e2].out;
                    j.q += S;
                    j.s->sweep_launches += 1;
                }
                if (launches) *launches += 1;
                if (entries) *entries += b.n;
            }
        }
    }
    // the sweeps whose last launch was an own launch of the final round
    return mark_done();
}

// The result of a finished ragged sweep, as fine_sweep returns it.
void ragged_end(const RaggedSweep& j, const float** dres, const double** wres) {
    if (j.s->fp32)
        *dres = static_cast<const float*>(j.cur) - j.off;
    else
        *wres = static_cast<const double*>(j.cur) - j.off;
}

ChainArgs chain_args(pr_solver* s, int k0, int k1, int init) {
    ChainArgs a{};
    a.fg = s->fg;
    a.nc = s->nc;
    a.q = s->q;
    a.k0 = k0;
    a.k1 = k1;
    a.steps = s->mG;
    a.init = init;
    a.fp32 = s->fp32 ? 1 : 0;
    a.c = s->coef;
    a.bc = s->bcc;
    a.dt = s->dtG;
    a.dT = s->dT;
    a.gstate = chain_state_in_lds(s->nc, a.fp32) ? nullptr : (void*)s->at<char>(s->L.gst);
    a.foldc = s->at<double>(s->L.foldc);
    return a;
}

double elapsed(pr_solver* s, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev[a], s->ev[b]) != hipSuccess) {
        (void)hipGetLastError();   // an unrecorded pair is not an error of the solve
        return 0.0;
    }
    return ms;
}

double host_ring_max(const pr_solver* s, double tau) {
    // max |g| over the fine ring at tau (host evaluation of the same closed forms)
    const Bc& b = s->bcf;
    if (b.payoff == 2) return std::fabs(b.cash);   // the option never pays more than c
    auto payoff = [&](double x, double y) {
        double v = (b.payoff == 1) ? (x - y) : (b.w1 * x + b.w2 * y - b.K);
        return v > 0 ? v : 0.0;
    };
    auto ncdf = [](double z) { return 0.5 * std::erfc(-z / std::sqrt(2.0)); };
    auto g = [&](double x, double y) {
        const double disc = std::exp(-b.r * tau);
        if (b.kind == PR_BC_DISCOUNTED_PAYOFF) return disc * payoff(x, y);
        if (b.kind == PR_BC_EXACT) {
            if (b.payoff == 1) {
                if (tau <= 0) return payoff(x, y);
                if (x <= 0) return 0.0;
                if (y <= 0) return x;
                double sd = std::sqrt((b.s1 * b.s1 + b.s2 * b.s2 - 2 * b.rho * b.s1 * b.s2) * tau);
                double d1 = (std::log(x / y) + 0.5 * sd * sd) / sd;
                return x * ncdf(d1) - y * ncdf(d1 - sd);
            }
            double S = x, K = b.K / b.w1;
            if (tau <= 0) return b.w1 * std::max(S - K, 0.0);
            if (S <= 0) return 0.0;
            double sd = b.s1 * std::sqrt(tau);
            double d1 = (std::log(S / K) + (b.r + 0.5 * b.s1 * b.s1) * tau) / sd;
            return b.w1 * (S * ncdf(d1) - K * std::exp(-b.r * tau) * ncdf(d1 - sd));
        }
        if (b.payoff == 1) return std::max(x - y, 0.0);
        return std::max(b.w1 * x + b.w2 * y - b.K * disc, 0.0);
    };
    const int n = s->fg.n;
    double m = 0;
    for (int k = 0; k < n; ++k) {
        const double t = k * b.h, e = (n - 1) * b.h;
        m = std::max({m, std::fabs(g(0, t)), std::fabs(g(e, t)), std::fabs(g(t, 0)),
                      std::fabs(g(t, e))});
    }
    return m;
}

void reset_krylov_stats(pr_solver* s) {
    s->kry_iters = 0;
    s->kry_max = 0;
    s->kry_unconv = 0;
}

void write_krylov_stats(const pr_solver* s, pr_stats* st) {
    st->krylov_iters = s->kry_iters;
    st->krylov_max_step = s->kry_max;
    st->krylov_unconverged = s->kry_unconv;
}

pr_status do_serial_fine(pr_solver* s, double* v_out, pr_stats* st) {
    const Grid& g = s->fg;
    double* U = s->U(0);
    reset_krylov_stats(s);
    s->sweep_launches = 0;
    s->sweep_bytes = 0;
    HIPCHK(launch_payoff(U, g, s->bcf, s->stream));
    for (int n = 0; n < s->N; ++n) {
        const float* d = nullptr;
        const double* w = nullptr;
        pr_status r = fine_sweep(s, U, n, 1, false, &d, &w, nullptr);
        if (r != PR_OK) return r;
        r = fine_result_to_state(s, U + (long long)n * g.stride,
                                 d ? d + (long long)n * g.stride : nullptr,
                                 w ? w + (long long)n * g.stride : nullptr,
                                 U + (long long)(n + 1) * g.stride);
        if (r != PR_OK) return r;
    }
    if (v_out) HIPCHK(launch_unpack(U + (long long)s->N * g.stride, v_out, g, s->bcf, s->N * s->dT, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (st) {
        st->fine_point_steps = (int64_t)s->N * s->mF * g.nin * g.nin;
        st->fine_step_launches = s->sweep_launches;
        st->fine_step_bytes = s->sweep_bytes;
        write_krylov_stats(s, st);
    }
    return PR_OK;
}

// R_s: fine interior state u at tau (interior layout) -> 62 x 62 coefficients
// field wc on the operator grid: wc = Sr (u - B(tau)) Sr^T.
pr_status fno_restrict(pr_solver* s, const double* u, double tau, double* wc) {
    const Grid& g = s->fg;
    const int nf = g.nin, mi = kFnoInt;
    double* wf = s->at<double>(s->L.fwf);
    double* T = s->at<double>(s->L.fT);
    const double* Sr = s->at<double>(s->L.Sr);
    HIPCHK(launch_lift(u, wf, g, s->bcf, tau, -1.0, s->stream));
    HIPCHK(fno::gemm_f64(Sr, nf, 1, wf, g.pitch, 1, T, nf, mi, nf, nf, 0.0, s->stream));
    HIPCHK(fno::gemm_f64(T, nf, 1, Sr, 1, nf, wc, mi, mi, mi, nf, 0.0, s->stream));
    return PR_OK;
}

// PR_FNO_BASE_LOD: the LOD propagator on the 64 x 64 grid itself over slice n
// from B(tau_n) + wc; wb = its result minus B(tau_{n+1}) (62 x 62 interior).
pr_status fno_lod_base(pr_solver* s, const double* wc, int n, double* wb) {
    const int mi = kFnoInt;
    const Grid g64{64, mi, mi, (long long)mi * mi};
    Bc bc = s->bcf;
    bc.h = s->grid.s_max / 63.0;
    const int m = s->opt.coarse_steps > 0 ? s->opt.coarse_steps : 4;
    double* v0 = s->at<double>(s->L.fvc0);
    double* v1 = s->at<double>(s->L.fvc1);
    HIPCHK(launch_lift(wc, v0, g64, bc, n * s->dT, 1.0, s->stream));
    HIPCHK(launch_lod_slice(v0, v1, s->at<double>(s->L.flw0), s->at<double>(s->L.flw1),
                            s->at<double>(s->L.flwb), g64, s->coef, bc, s->dT / m, n * s->dT, m,
                            s->stream));
    HIPCHK(launch_lift(v1, wb, g64, bc, (n + 1) * s->dT, -1.0, s->stream));
    return PR_OK;
}

// PR_FNO_BASE_FINE_LOD: out = the LOD propagator on the fine grid over slice n
// (coarse_steps steps, default 1) from the interior state u.
pr_status fno_fine_lod(pr_solver* s, const double* u, int n, double* out) {
    const int m = s->opt.coarse_steps > 0 ? s->opt.coarse_steps : 1;
    HIPCHK(launch_lod_slice(u, out, s->at<double>(s->L.lw0), s->at<double>(s->L.lw1),
                            s->at<double>(s->L.lwb), s->fg, s->coef, s->bcf, s->dT / m,
                            n * s->dT, m, s->stream));
    return PR_OK;
}

// Neural G over slice n: gout = B(tau_{n+1}) + P_s(base + scale * FNO(wc, params)),
// wc = R_s(U_n); the ring of gout is g(tau_{n+1}) by construction of B.
pr_status fno_g(pr_solver* s, const double* Uall, int n, double* gout) {
    const Grid& g = s->fg;
    const int nf = g.nin, mi = kFnoInt;
    double* wc = s->at<double>(s->L.fwc);
    double* wo = s->at<double>(s->L.fwc1);
    double* Tp = s->at<double>(s->L.fTp);
    const double* Sp = s->at<double>(s->L.Sp);
    const double* u = Uall + (long long)n * g.stride;
    pr_status r = fno_restrict(s, u, n * s->dT, wc);
    if (r != PR_OK) return r;
    float* fin = s->at<float>(s->L.fin);
    float* fmeta = s->at<float>(s->L.fmeta);
    float* fout = s->at<float>(s->L.fout);
    HIPCHK(launch_fno_in(wc, fin, fmeta, s->bcf, s->stream));
    HIPCHK(fno::infer(s->fno, fin, fmeta, 1, fout, s->stream));
    if (fno::base(s->fno) == PR_FNO_BASE_FINE_LOD) {
        // gout = LOD(u) on the fine grid, plus the prolonged correction
        r = fno_fine_lod(s, u, n, gout);
        if (r != PR_OK) return r;
        HIPCHK(launch_fno_out(nullptr, fout, fno::out_scale(s->fno), wo, s->stream));
        HIPCHK(fno::gemm_f64(Sp, mi, 1, wo, mi, 1, Tp, mi, nf, mi, mi, 0.0, s->stream));
        HIPCHK(fno::gemm_f64(Tp, mi, 1, Sp, 1, mi, gout, g.pitch, nf, nf, mi, 1.0, s->stream));
        return PR_OK;
    }
    const double* base = nullptr;
    if (fno::base(s->fno) == PR_FNO_BASE_IDENTITY) base = wc;
    if (fno::base(s->fno) == PR_FNO_BASE_LOD) {
        double* wb = s->at<double>(s->L.fwb);
        r = fno_lod_base(s, wc, n, wb);
        if (r != PR_OK) return r;
        base = wb;
    }
    HIPCHK(launch_fno_out(base, fout, fno::out_scale(s->fno), wo, s->stream));
    HIPCHK(fno::gemm_f64(Sp, mi, 1, wo, mi, 1, Tp, mi, nf, mi, mi, 0.0, s->stream));
    HIPCHK(fno::gemm_f64(Tp, mi, 1, Sp, 1, mi, gout, g.pitch, nf, nf, mi, 0.0, s->stream));
    HIPCHK(launch_lift(gout, gout, g, s->bcf, (n + 1) * s->dT, 1.0, s->stream));
    return PR_OK;
}

// The fine-grid G over slice n: g = G(U^{k+1}_n) into gout (one slice).
pr_status fine_g(pr_solver* s, const double* Uslice_base_all, int n, double* gout) {
    if (s->fnog) return fno_g(s, Uslice_base_all, n, gout);
    if (s->implicit_g) {
        const double* w = nullptr;
        pr_status r = implicit_sweep(s, Uslice_base_all, n, 1, true, &w, nullptr, s->dtG, s->mG);
        if (r != PR_OK) return r;
        HIPCHK(hipMemcpyAsync(gout, w, (size_t)s->fg.stride * 8, hipMemcpyDeviceToDevice, s->stream));
        return PR_OK;
    }
    if (s->lod) {
        HIPCHK(launch_lod_slice(Uslice_base_all + (long long)n * s->fg.stride, gout,
                                s->at<double>(s->L.lw0), s->at<double>(s->L.lw1),
                                s->at<double>(s->L.lwb), s->fg, s->coef, s->bcf, s->dtG,
                                n * s->dT, s->mG, s->stream));
        return PR_OK;
    }
    const float* d = nullptr;
    const double* w = nullptr;
    pr_status r = fine_sweep(s, Uslice_base_all, n, 1, true, &d, &w, nullptr);
    if (r != PR_OK) return r;
    return fine_result_to_state(s, Uslice_base_all + (long long)n * s->fg.stride, d, w, gout);
}

// Initial coarse sweep: U_0 = payoff, U_{n+1} = G(U_n) (stream-ordered, no host sync).
pr_status init_phase(pr_solver* s, double* Ucur, double* Unext) {
    const Grid& g = s->fg;
    const int N = s->N;
    HIPCHK(launch_payoff(Ucur, g, s->bcf, s->stream));
    HIPCHK(hipMemcpyAsync(Unext, Ucur, (size_t)g.stride * 8, hipMemcpyDeviceToDevice, s->stream));
    if (s->fineg) {
        double* Gf = s->at<double>(s->L.Gf);
        for (int n = 0; n < N; ++n) {
            pr_status r = fine_g(s, Ucur, n, Ucur + (long long)(n + 1) * g.stride);
            if (r != PR_OK) return r;
            HIPCHK(hipMemcpyAsync(Gf + (long long)n * g.stride, Ucur + (long long)(n + 1) * g.stride,
                                  (size_t)g.stride * 8, hipMemcpyDeviceToDevice, s->stream));
        }
    } else {
        ChainArgs ca = chain_args(s, 0, N, 1);
        HIPCHK(launch_chain(Ucur, s->at<double>(s->L.Gold), s->at<double>(s->L.dcor),
                            s->at<double>(s->L.cst), s->at<float>(s->L.lbc), ca, s->stream));
        HIPCHK(launch_prolong(s->at<double>(s->L.Gold), Ucur, g, s->nc, s->q, 0, N, s->stream));
    }
    return PR_OK;
}

// Iteration k with the chain overlapped (numerical G, explicit F): slices
// k..N-1 in G groups of gs consecutive slices.  Per group, on the solver's
// stream: the fine sweep; on the chain stream, once that sweep has ended: the
// gather of F at the coincident nodes, the chain over the group (the first
// group starts from U^k_k, a later one from the corrected U^{k+1} at its first
// slice, which the previous group's correction has written) and the correction
// + norm of the group.  The chain of group g thus runs while group g+1 is swept.
// The two streams touch disjoint slices of every buffer they share (F results,
// Lb, foldc, Gold, dcor, U), except the chain's own scratch, which only the
// chain stream uses.  The solver's stream waits for the chain stream at the
// end, so callers see one stream-ordered phase.
pr_status iteration_phase_overlapped(pr_solver* s, int k, double* Ucur, double* Unext,
                                     double* step_ms, int gs, int G) {
    const Grid& g = s->fg;
    const int N = s->N;
    const bool ev = step_ms != nullptr && s->events;
    hipStream_t cs = s->chain_stream;
    unsigned long long* red = s->red();
    HIPCHK(launch_zero_red(red, s->stream));
    if (k > 0)
        HIPCHK(hipMemcpyAsync(Unext + (long long)k * g.stride, Ucur + (long long)k * g.stride,
                              (size_t)g.stride * 8, hipMemcpyDeviceToDevice, s->stream));
    if (ev) HIPCHK(hipEventRecord(s->ev[4], s->stream));
    // a group's launches have 1/G of the wavefronts; longer row chunks keep
    // the temporally blocked kernel's recomputed halo rows a small share
    struct Restore {   // the sweep settings come back on every return
        pr_solver* s;
        int min_rows;
        ~Restore() {
            s->min_rows = min_rows;
            s->bracket_sweep = true;
        }
    } restore{s, s->min_rows};
    s->min_rows = std::max(restore.min_rows, s->pipe_min_rows);
    s->bracket_sweep = false;
    for (int gi = 0; gi < G; ++gi) {
        const int b0 = k + gi * gs, b1 = std::min(N, b0 + gs);
        const float* d = nullptr;
        const double* w = nullptr;
        pr_status r = fine_sweep(s, Ucur, b0, b1 - b0, false, &d, &w, step_ms);
        if (r != PR_OK) return r;
        const void* Fold = s->fp32 ? (const void*)d : (const void*)w;
        HIPCHK(hipEventRecord(s->pipe_ev[gi], s->stream));
        HIPCHK(hipStreamWaitEvent(cs, s->pipe_ev[gi], 0));
        HIPCHK(launch_gather_coincident(Ucur, Fold, s->at<double>(s->L.foldc), g, s->nc, s->q, b0,
                                        b1, s->fp32 ? 1 : 0, cs));
        ChainArgs ca = chain_args(s, b0, b1, 0);
        HIPCHK(launch_chain(gi == 0 ? Ucur : Unext, s->at<double>(s->L.Gold),
                            s->at<double>(s->L.dcor), s->at<double>(s->L.cst),
                            s->at<float>(s->L.lbc), ca, cs));
        HIPCHK(launch_correct(Ucur, Fold, s->at<double>(s->L.dcor), nullptr, nullptr, Unext, red,
                              g, b0, b1, N, s->nc, s->q, s->fp32, 0, cs));
    }
    if (ev) {
        HIPCHK(hipEventRecord(s->ev[5], s->stream));
        HIPCHK(hipEventRecord(s->ev[1], s->stream));
    }
    HIPCHK(hipEventRecord(s->pipe_ev[G], cs));
    HIPCHK(hipStreamWaitEvent(s->stream, s->pipe_ev[G], 0));
    if (ev) {
        HIPCHK(hipEventRecord(s->ev[2], s->stream));
        HIPCHK(hipEventRecord(s->ev[3], s->stream));
    }
    return PR_OK;
}

// Phased overlap (PR_PIPE_MODE 1).  A phase fixes a group boundary B for the
// iterations k < B (B - k0 = pipe_split percent of the N - k0 active slices at
// the phase's first iteration k0; a phase starts while at least 2 pipe_min
// slices are active, after that an iteration runs as one group): group 0 is
// [k, B) and shrinks by one slice per iteration, group 1 is [B, N).  As in iteration_phase_overlapped, group 0's chain and
// correction (chain stream) run beside group 1's fine sweep.  In addition, the
// next iteration's group-0 sweep [k+1, B) needs only U^{k+1}_{k+1..B}, which
// group 0's correction has just written, and touches no buffer that group 1
// still reads (its slices are below B): it is issued right after that
// correction and runs beside group 1's chain, the part of the chain that the
// equal-group schedule leaves exposed.  If the solve stops at k, that sweep is
// discarded.  The arithmetic of every slice is unchanged.
pr_status iteration_phase_phased(pr_solver* s, int k, double* Ucur, double* Unext,
                                 double* step_ms) {
    const Grid& g = s->fg;
    const int N = s->N;
    const int B = s->pipe_B;
    const bool ev = step_ms != nullptr && s->events;
    hipStream_t cs = s->chain_stream;
    unsigned long long* red = s->red();
    HIPCHK(launch_zero_red(red, s->stream));
    if (k > 0)
        HIPCHK(hipMemcpyAsync(Unext + (long long)k * g.stride, Ucur + (long long)k * g.stride,
                              (size_t)g.stride * 8, hipMemcpyDeviceToDevice, s->stream));
    if (ev) HIPCHK(hipEventRecord(s->ev[4], s->stream));
    struct Restore {   // the sweep settings come back on every return
        pr_solver* s;
        int min_rows;
        ~Restore() {
            s->min_rows = min_rows;
            s->bracket_sweep = true;
        }
    } restore{s, s->min_rows};
    s->min_rows = std::max(restore.min_rows, s->pipe_min_rows);
    s->bracket_sweep = false;
    auto fold = [&](const float* d, const double* w) {
        return s->fp32 ? (const void*)d : (const void*)w;
    };
    // group 0: [k, B), swept during the previous iteration when it could be
    const void* F0 = nullptr;
    if (s->early_k == k) {
        F0 = s->early_fold;
    } else {
        const float* d = nullptr;
        const double* w = nullptr;
        pr_status r = fine_sweep(s, Ucur, k, B - k, false, &d, &w, step_ms);
        if (r != PR_OK) return r;
        F0 = fold(d, w);
    }
    s->early_k = -1;
    HIPCHK(hipEventRecord(s->pipe_ev[0], s->stream));
    HIPCHK(hipStreamWaitEvent(cs, s->pipe_ev[0], 0));
    HIPCHK(launch_gather_coincident(Ucur, F0, s->at<double>(s->L.foldc), g, s->nc, s->q, k, B,
                                    s->fp32 ? 1 : 0, cs));
    ChainArgs c0 = chain_args(s, k, B, 0);
    HIPCHK(launch_chain(Ucur, s->at<double>(s->L.Gold), s->at<double>(s->L.dcor),
                        s->at<double>(s->L.cst), s->at<float>(s->L.lbc), c0, cs));
    HIPCHK(launch_correct(Ucur, F0, s->at<double>(s->L.dcor), nullptr, nullptr, Unext, red, g, k,
                          B, N, s->nc, s->q, s->fp32, 0, cs));
    HIPCHK(hipEventRecord(s->pipe_ev[2], cs));   // U^{k+1}_{k+1..B} written
    // group 1: [B, N)
    {
        const float* d = nullptr;
        const double* w = nullptr;
        pr_status r = fine_sweep(s, Ucur, B, N - B, false, &d, &w, step_ms);
        if (r != PR_OK) return r;
        const void* F1 = fold(d, w);
        HIPCHK(hipEventRecord(s->pipe_ev[1], s->stream));
        HIPCHK(hipStreamWaitEvent(cs, s->pipe_ev[1], 0));
        HIPCHK(launch_gather_coincident(Ucur, F1, s->at<double>(s->L.foldc), g, s->nc, s->q, B,
                                        N, s->fp32 ? 1 : 0, cs));
        ChainArgs c1 = chain_args(s, B, N, 0);
        HIPCHK(launch_chain(Unext, s->at<double>(s->L.Gold), s->at<double>(s->L.dcor),
                            s->at<double>(s->L.cst), s->at<float>(s->L.lbc), c1, cs));
        HIPCHK(launch_correct(Ucur, F1, s->at<double>(s->L.dcor), nullptr, nullptr, Unext, red,
                              g, B, N, N, s->nc, s->q, s->fp32, 0, cs));
    }
    // the next iteration's group 0, beside group 1's chain
    if (k + 1 < B && k + 1 < s->maxit) {
        HIPCHK(hipStreamWaitEvent(s->stream, s->pipe_ev[2], 0));
        const float* d = nullptr;
        const double* w = nullptr;
        pr_status r = fine_sweep(s, Unext, k + 1, B - k - 1, false, &d, &w, step_ms);
        if (r != PR_OK) return r;
        s->early_fold = fold(d, w);
        s->early_k = k + 1;
    }
    if (ev) {
        HIPCHK(hipEventRecord(s->ev[5], s->stream));
        HIPCHK(hipEventRecord(s->ev[1], s->stream));
    }
    HIPCHK(hipEventRecord(s->pipe_ev[3], cs));
    HIPCHK(hipStreamWaitEvent(s->stream, s->pipe_ev[3], 0));
    if (ev) {
        HIPCHK(hipEventRecord(s->ev[2], s->stream));
        HIPCHK(hipEventRecord(s->ev[3], s->stream));
    }
    return PR_OK;
}

pr_status iteration_after_sweep(pr_solver* s, int k, double* Ucur, double* Unext,
                                const void* Fold, bool ev);

// Iteration k: F sweep over slices k..N-1, coarse chain, correction + norm
// into Unext (stream-ordered, no host sync).  step_ms != nullptr enables the
// per-phase and per-launch timing events.
pr_status iteration_phase(pr_solver* s, int k, double* Ucur, double* Unext, double* step_ms) {
    const int N = s->N;
    if (s->pipe && !s->fineg && !s->implicit && s->pipe_mode == 1) {
        if (k >= s->pipe_B) {   // a new phase: split the active slices in two
            const int active = N - k;
            const int g0 = std::max(1, std::min(active - 1, active * s->pipe_split / 100));
            s->pipe_B = active >= 2 * s->pipe_min ? k + g0 : N;
        }
        if (s->pipe_B > k && s->pipe_B < N) return iteration_phase_phased(s, k, Ucur, Unext, step_ms);
    } else if (s->pipe && !s->fineg && !s->implicit) {
        const int active = N - k;
        const int gs = std::max(s->pipe_min, (active + s->pipe_groups - 1) / s->pipe_groups);
        const int G = (active + gs - 1) / gs;
        if (G > 1) return iteration_phase_overlapped(s, k, Ucur, Unext, step_ms, gs, G);
    }
    const float* d = nullptr;
    const double* w = nullptr;
    const bool ev = step_ms != nullptr && s->events;
    pr_status r = fine_sweep(s, Ucur, k, N - k, false, &d, &w, step_ms);
    if (r != PR_OK) return r;
    return iteration_after_sweep(s, k, Ucur, Unext, s->fp32 ? (const void*)d : (const void*)w,
                                 ev);
}

// Iteration k after its fine sweep (Fold: the sweep's result, increments or
// states): the coarse chain, or the same-grid G slice by slice, and the
// correction with its norm into Unext.
pr_status iteration_after_sweep(pr_solver* s, int k, double* Ucur, double* Unext,
                                const void* Fold, bool ev) {
    const Grid& g = s->fg;
    const int N = s->N;
    pr_status r = PR_OK;
    if (ev) HIPCHK(hipEventRecord(s->ev[1], s->stream));
    unsigned long long* red = s->red();
    HIPCHK(launch_zero_red(red, s->stream));
    if (k > 0)
        HIPCHK(hipMemcpyAsync(Unext + (long long)k * g.stride, Ucur + (long long)k * g.stride,
                              (size_t)g.stride * 8, hipMemcpyDeviceToDevice, s->stream));
    if (s->fineg) {
        double* tg = s->at<double>(s->L.tg);
        double* Gf = s->at<double>(s->L.Gf);
        for (int n = k; n < N; ++n) {
            r = fine_g(s, Unext, n, tg);
            if (r != PR_OK) return r;
            HIPCHK(launch_correct(Ucur, Fold, nullptr, tg, Gf, Unext, red, g, n, n + 1, N, 0, 1,
                                  s->fp32, 1, s->stream));
        }
        if (ev) HIPCHK(hipEventRecord(s->ev[2], s->stream));
    } else {
        ChainArgs ca = chain_args(s, k, N, 0);
        HIPCHK(launch_gather_coincident(Ucur, Fold, s->at<double>(s->L.foldc), g, s->nc, s->q, k,
                                        N, s->fp32 ? 1 : 0, s->stream));
        HIPCHK(launch_chain(Ucur, s->at<double>(s->L.Gold), s->at<double>(s->L.dcor),
                            s->at<double>(s->L.cst), s->at<float>(s->L.lbc), ca, s->stream));
        if (ev) HIPCHK(hipEventRecord(s->ev[2], s->stream));
        HIPCHK(launch_correct(Ucur, Fold, s->at<double>(s->L.dcor), nullptr, nullptr, Unext, red,
                              g, k, N, N, s->nc, s->q, s->fp32, 0, s->stream));
    }
    if (ev) HIPCHK(hipEventRecord(s->ev[3], s->stream));
    return PR_OK;
}

// Run a phase eagerly, or (PR_FLAG_GRAPH) capture it once on the private
// capture stream and replay the cached graph on the solver's stream.
template <class Fn>
pr_status run_phase(pr_solver* s, int key, Fn&& fn) {
    if (!s->graph) return fn();
    auto it = s->graphs.find(key);
    if (it == s->graphs.end()) {
        hipStream_t user = s->stream;
        s->stream = s->cap_stream;
        s->sweep_launches = 0;
        s->sweep_bytes = 0;
        hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            s->stream = user;
            s->err = std::string("hipStreamBeginCapture: ") + hipGetErrorString(e);
            return PR_EDEVICE;
        }
        pr_status r = fn();
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(s->cap_stream, &gr);
        s->stream = user;
        if (r != PR_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return r;
        }
        if (e != hipSuccess) {
            s->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
            return PR_EDEVICE;
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(gr);
            s->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
            return PR_EDEVICE;
        }
        s->graph_defs[key] = gr;
        s->graph_launches[key] = s->sweep_launches;
        s->graph_bytes[key] = s->sweep_bytes;
        it = s->graphs.emplace(key, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, s->stream));
    return PR_OK;
}

// PR_G_FNO fallback: the same-grid LOD propagator with the given (or 4)
// coarse steps per slice; cached graphs of the neural G are dropped.
pr_status switch_to_lod(pr_solver* s) {
    s->fnog = false;
    s->lod = true;
    s->mG = s->opt.coarse_steps > 0 ? s->opt.coarse_steps : 4;
    s->dtG = s->dT / s->mG;
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : s->graph_defs) (void)hipGraphDestroy(kv.second);
    s->graphs.clear();
    s->graph_defs.clear();
    HIPCHK(lod_set_lds(s->fg.nin));
    return PR_OK;
}

pr_status do_solve(pr_solver* s, double* v_out, pr_stats* st) {
    const Grid& g = s->fg;
    const int N = s->N;
    if (s->fnog && !s->fno) {
        s->err = "PR_G_FNO solver without an attached operator (parareal_attach_fno)";
        return PR_EMODEL;
    }
    bool diverging = false;   // PR_G_FNO: non-finite, or two increments in a row growing
    reset_krylov_stats(s);
    s->pipe_B = -1;   // the phased overlap starts a new phase at k = 0
    s->early_k = -1;
    s->timed_launches = 0;
    s->timed_bytes = 0;
    double* Ucur = s->U(0);
    double* Unext = s->U(1);
    double t_fine = 0, t_chain = 0, t_corr = 0, t_steps = 0, step_bytes = 0;
    int64_t launches = 0, psteps = 0;
    // algorithmic bytes of one explicit step per interior node (counted by
    // fine_sweep): FP32 increment form reads d and Lb and writes d (12 B);
    // FP64 reads and writes u (16 B)

    // ---- initialisation: U^0_0 = payoff, U^0_{n+1} = G(U^0_n)
    {
        pr_status r = run_phase(s, -1, [&]() { return init_phase(s, Ucur, Unext); });
        if (r != PR_OK) return r;
    }
    int K = 0;
    pr_status status = PR_OK;
    double inc = 0, scale = 0;
    double st_prev[2] = {0.0, 0.0};
    for (int k = 0; k < s->maxit && k < N; ++k) {
        // ---- F sweep over active slices k..N-1, chain, correction + norm
        s->sweep_launches = 0;
        s->sweep_bytes = 0;
        if (s->events) HIPCHK(hipEventRecord(s->ev[0], s->stream));
        pr_status r = run_phase(s, k, [&]() {
            return iteration_phase(s, k, Ucur, Unext, s->graph ? nullptr : &t_steps);
        });
        if (r != PR_OK) return r;
        if (s->graph && s->events) HIPCHK(hipEventRecord(s->ev[3], s->stream));
        launches += s->graph ? s->graph_launches[k] : s->sweep_launches;
        step_bytes += s->graph ? s->graph_bytes[k] : s->sweep_bytes;
        psteps += (int64_t)(N - k) * s->mF * g.nin * g.nin;
        unsigned long long* red = s->red();
        unsigned long long hred[3];
        HIPCHK(hipMemcpyAsync(hred, red, sizeof(hred), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (s->events && s->graph) {
            t_fine += elapsed(s, 0, 3);
        } else if (s->events) {
            t_fine += elapsed(s, 0, 1);
            t_chain += elapsed(s, 1, 2);
            t_corr += elapsed(s, 2, 3);
            if (s->step_ev.empty()) t_steps += elapsed(s, 4, 5);
        }
        for (int e = 0; e + 1 < s->step_ev_used; e += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->step_ev[e], s->step_ev[e + 1]) == hipSuccess) t_steps += ms;
        }
        s->step_ev_used = 0;
        std::swap(Ucur, Unext);
        std::memcpy(&inc, &hred[0], 8);
        double scint;
        std::memcpy(&scint, &hred[1], 8);
        scale = std::max(scint, s->ring_max_T);
        K = k + 1;
        if (st && k <= PR_MAX_SLICES) st->increments[k] = inc;
        if (s->fnog && !(s->opt.flags & PR_FLAG_NO_FALLBACK) &&
            (hred[2] || (k >= 2 && inc > st_prev[1] && st_prev[1] > st_prev[0]))) {
            diverging = true;
            break;
        }
        st_prev[0] = st_prev[1];
        st_prev[1] = inc;
        if (hred[2]) {
            status = PR_ENONFINITE;
            s->err = "non-finite value in the Parareal iteration";
            break;
        }
        const double thr = s->opt.tol_relative ? s->opt.tol * scale : s->opt.tol;
        if (inc < thr || K == N) break;
        if (K == s->maxit) {
            status = PR_ENOTCONV;
            s->err = "max_iters reached above tolerance";
        }
    }
    if (diverging) {
        pr_status r = switch_to_lod(s);
        if (r != PR_OK) return r;
        r = do_solve(s, v_out, st);
        if (st) st->coarse_fallback = 1;
        return r;
    }
    if (v_out) HIPCHK(launch_unpack(Ucur + (long long)N * g.stride, v_out, g, s->bcf, N * s->dT, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (st) {
        st->iters = K;
        st->last_increment = inc;
        st->scale = scale;
        st->t_fine_ms = t_fine;
        st->t_chain_ms = t_chain;
        st->t_correct_ms = t_corr;
        st->t_step_kernels_ms = t_steps;
        st->timed_step_launches = s->timed_launches;
        st->timed_step_bytes = s->timed_bytes;
        st->fine_point_steps = psteps;
        st->fine_step_launches = launches;
        st->fine_step_bytes = step_bytes;
        write_krylov_stats(s, st);
    }
    return status;
}

}  // namespace

extern "C" {

int32_t parareal_abi_version(void) { return PR_ABI_VERSION; }

const char* parareal_strerror(pr_status st) {
    switch (st) {
        case PR_OK: return "ok";
        case PR_EINVAL: return "invalid argument";
        case PR_EUNSTABLE: return "explicit step above the stability bound";
        case PR_ENOMEM: return "workspace too small";
        case PR_EDEVICE: return "HIP runtime error";
        case PR_ENOTCONV: return "not converged within max_iters";
        case PR_ENONFINITE: return "non-finite value";
        case PR_EMODEL: return "coarse model unavailable";
        case PR_EBUSY: return "request queue full";
    }
    return "unknown status";
}

const char* parareal_last_error(const pr_solver* s) { return s ? s->err.c_str() : "null solver"; }

pr_status parareal_plan(const pr_grid* grid, const pr_model* model, const pr_options* opt,
                        int32_t* fine_steps, int32_t* coarse_steps, double* dt_stable_fine,
                        double* dt_stable_coarse) {
    if (!grid || !model || !opt) return PR_EINVAL;
    if (!valid_basic(grid, opt, nullptr)) return PR_EINVAL;
    if (!(model->sigma1 > 0) || !(model->sigma2 > 0) || !(std::fabs(model->rho) < 1) ||
        !(model->r >= 0) || !(model->T > 0))
        return PR_EINVAL;
    const double dT = model->T / opt->n_slices;
    const double dsf = gershgorin_dt(grid->n, *model);
    int mf = opt->fine_steps;
    if (mf == 0) mf = (int)std::ceil(dT / (opt->cfl * dsf));
    int mg = 0;
    double dsc = 0;
    if (opt->coarse_kind == PR_G_LOD) mg = opt->coarse_steps > 0 ? opt->coarse_steps : 2;
    if (opt->coarse_kind == PR_G_IMPLICIT) mg = opt->coarse_steps > 0 ? opt->coarse_steps : 1;
    if (opt->coarse_kind == PR_G_NUMERICAL) {
        dsc = gershgorin_dt(opt->coarse_n, *model);
        mg = opt->coarse_steps;
        if (mg == 0) mg = (int)std::ceil(dT / (opt->cfl * dsc));
    }
    if (fine_steps) *fine_steps = mf;
    if (coarse_steps) *coarse_steps = mg;
    if (dt_stable_fine) *dt_stable_fine = dsf;
    if (dt_stable_coarse) *dt_stable_coarse = dsc;
    if (opt->fine_scheme != PR_FINE_IMPLICIT && dT / mf > dsf) return PR_EUNSTABLE;
    if (opt->coarse_kind == PR_G_NUMERICAL && dT / mg > dsc) return PR_EUNSTABLE;
    return PR_OK;
}

uint64_t parareal_workspace_bytes(const pr_grid* grid, const pr_options* opt) {
    if (!valid_basic(grid, opt, nullptr)) return 0;
    return layout(grid, opt).total;
}

}  // extern "C"

namespace {

// Validates the arguments and fills a solver bound to device_workspace (no GPU
// call before validation has passed).  with_runtime_objects: create the
// timing events, the capture stream and the step-event pairs (parareal_create);
// without them (the static-scratch entry point) the solver creates no runtime
// object and PR_FLAG_TIME_STEPS / PR_FLAG_GRAPH are ignored.
pr_status setup_solver(pr_solver* s, const pr_grid* grid, const pr_model* model,
                       const pr_payoff* payoff, const pr_options* opt, void* device_workspace,
                       uint64_t workspace_bytes, void* hip_stream, bool with_runtime_objects) {
    if (!grid || !model || !payoff || !opt) return PR_EINVAL;
    std::string why;
    if (!valid_basic(grid, opt, &why)) return PR_EINVAL;
    if (payoff->kind != PR_PAYOFF_BASKET_CALL && payoff->kind != PR_PAYOFF_EXCHANGE &&
        payoff->kind != PR_PAYOFF_CASH_OR_NOTHING)
        return PR_EINVAL;
    if (payoff->bc_kind < 0 || payoff->bc_kind > 2) return PR_EINVAL;
    if (payoff->kind == PR_PAYOFF_CASH_OR_NOTHING) {
        if (payoff->bc_kind == PR_BC_FORWARD_INTRINSIC) return PR_EINVAL;
        if (!(payoff->strike > 0.0) || !(payoff->strike2 > 0.0) || !std::isfinite(payoff->cash))
            return PR_EINVAL;
        if (payoff->bc_kind == PR_BC_EXACT && !(std::fabs(model->rho) <= 0.925)) return PR_EINVAL;
    }
    if (payoff->bc_kind == PR_BC_EXACT && payoff->kind == PR_PAYOFF_BASKET_CALL &&
        !(payoff->w2 == 0.0 && payoff->w1 > 0.0 && payoff->strike > 0.0))
        return PR_EINVAL;
    if (!std::isfinite(payoff->w1) || !std::isfinite(payoff->w2) || !std::isfinite(payoff->strike))
        return PR_EINVAL;
    int32_t mf = 0, mg = 0;
    double dsf = 0, dsc = 0;
    pr_status pst = parareal_plan(grid, model, opt, &mf, &mg, &dsf, &dsc);
    if (pst != PR_OK) return pst;
    const Layout L = layout(grid, opt);
    if (!device_workspace || workspace_bytes < L.total) return PR_ENOMEM;
    if (reinterpret_cast<uintptr_t>(device_workspace) % kAlign) return PR_EINVAL;

    s->grid = *grid;
    s->model = *model;
    s->pay = *payoff;
    s->opt = *opt;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->fg = make_grid(grid->n);
    s->N = opt->n_slices;
    s->maxit = opt->max_iters > 0 ? std::min(opt->max_iters, s->N) : s->N;
    s->fp32 = opt->precision == PR_FP32;
    s->implicit = opt->fine_scheme == PR_FINE_IMPLICIT;
    s->lod = opt->coarse_kind == PR_G_LOD;
    s->fnog = opt->coarse_kind == PR_G_FNO;
    s->implicit_g = opt->coarse_kind == PR_G_IMPLICIT;
    s->fineg = opt->coarse_kind == PR_G_FINE || s->lod || s->fnog || s->implicit_g;
    s->nc = s->fineg ? 0 : opt->coarse_n;
    s->q = s->fineg ? 1 : (grid->n - 1) / (opt->coarse_n - 1);
    s->mF = mf;
    s->mG = mg;
    s->dT = model->T / s->N;
    s->dtF = s->dT / mf;
    s->dtG = mg ? s->dT / mg : 0.0;
    s->coef = Coef{0.5 * model->sigma1 * model->sigma1, 0.5 * model->sigma2 * model->sigma2,
                   0.25 * model->rho * model->sigma1 * model->sigma2, 0.5 * model->r, model->r};
    Bc b{};
    b.payoff = payoff->kind;
    b.kind = payoff->bc_kind;
    b.w1 = payoff->w1;
    b.w2 = payoff->w2;
    b.K = payoff->strike;
    b.K2 = payoff->strike2;
    b.cash = payoff->cash;
    b.s1 = model->sigma1;
    b.s2 = model->sigma2;
    b.rho = model->rho;
    b.r = model->r;
    b.h = grid->s_max / (grid->n - 1);
    s->bcf = b;
    b.h = s->fineg ? b.h : grid->s_max / (opt->coarse_n - 1);
    s->bcc = b;
    s->ws = reinterpret_cast<char*>(device_workspace);
    s->ws_bytes = workspace_bytes;
    s->L = L;
    s->ring_max_T = host_ring_max(s, model->T);
    if (const char* e = std::getenv("PR_STEP_ROWS")) s->rows_override = std::atoi(e);
    if (const char* e = std::getenv("PR_STEP_FUSE")) s->fuse = std::max(1, std::min(8, std::atoi(e)));
    if (const char* e = std::getenv("PR_STEP_FUSE_SMALL"))
        s->fuse_small = std::max(1, std::min(8, std::atoi(e)));
    if (const char* e = std::getenv("PR_STEP_SMALL_COUNT")) s->small_count = std::atoi(e);
    if (const char* e = std::getenv("PR_STEP_WAVES")) s->wave_target = std::max(256, std::atoi(e));
    if (const char* e = std::getenv("PR_STEP_TIME_EVERY")) s->ev_every = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("PR_STEP_MINROWS")) s->min_rows = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("PR_STEP_FIT")) s->step_fit = std::atoi(e);
    if (const char* e = std::getenv("PR_PIPE_GROUPS"))
        s->pipe_groups = std::max(1, std::min(pr_solver::kPipeMaxGroups, std::atoi(e)));
    if (const char* e = std::getenv("PR_PIPE_MIN")) s->pipe_min = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("PR_PIPE_MODE")) s->pipe_mode = std::atoi(e);
    if (const char* e = std::getenv("PR_PIPE_SPLIT"))
        s->pipe_split = std::max(1, std::min(99, std::atoi(e)));
    if (const char* e = std::getenv("PR_PIPE_MINROWS")) s->pipe_min_rows = std::max(1, std::atoi(e));
    if (!s->fineg && chain_set_lds(chain_lds_bytes(s->nc, s->fp32 ? 1 : 0)) != hipSuccess)
        return PR_EDEVICE;
    if ((s->lod || s->fnog) && lod_set_lds(s->fg.nin) != hipSuccess) return PR_EDEVICE;
    if (s->fnog) {
        std::vector<double> R, P;
        sine_transfer_matrices(s->fg.nin, R, P);
        hipError_t e = hipMemcpyAsync(s->at<double>(L.Sr), R.data(), R.size() * 8,
                                      hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->at<double>(L.Sp), P.data(), P.size() * 8, hipMemcpyHostToDevice,
                               s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return PR_EDEVICE;
    }
    if (!with_runtime_objects) return PR_OK;
    bool ok = true;
    for (auto& e : s->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    s->events = ok;
    s->graph = (opt->flags & PR_FLAG_GRAPH) != 0;
    if (s->graph && hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return PR_EDEVICE;
    if (!s->graph && !(opt->flags & PR_FLAG_SERIAL_CHAIN) && !s->implicit && s->pipe_groups > 1 &&
        hipStreamCreateWithFlags(&s->chain_stream, hipStreamNonBlocking) == hipSuccess) {
        bool eok = true;
        for (int i = 0; i <= std::max(s->pipe_groups, 3); ++i)
            eok = eok && hipEventCreateWithFlags(&s->pipe_ev[i], hipEventDisableTiming) == hipSuccess;
        s->pipe = eok;   // otherwise the chain stays serial (the objects are released later)
    }
    if (s->implicit || s->implicit_g) {
        // pinned slots and events for the pipelined convergence polls of BiCGStab;
        // without them the polls wait for the stream (same results)
        bool kok = hipHostMalloc(reinterpret_cast<void**>(&s->kry_pin), 2 * sizeof(int)) ==
                   hipSuccess;
        if (!kok) s->kry_pin = nullptr;
        for (auto& e : s->kry_ev)
            kok = kok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (!kok && s->kry_pin) {
            (void)hipHostFree(s->kry_pin);
            s->kry_pin = nullptr;
        }
    }
    if ((opt->flags & PR_FLAG_TIME_STEPS) && !s->graph) {
        s->step_ev.resize(2 * (size_t)mf, nullptr);
        for (auto& e : s->step_ev)
            if (hipEventCreate(&e) != hipSuccess) {
                e = nullptr;
                ok = false;
            }
        if (!ok) {
            for (auto& e : s->step_ev)
                if (e) (void)hipEventDestroy(e);
            s->step_ev.clear();
        }
    }
    return PR_OK;
}

void release_runtime_objects(pr_solver* s) {
    for (auto& e : s->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : s->step_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : s->graph_defs) (void)hipGraphDestroy(kv.second);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    for (auto& e : s->pipe_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->chain_stream) (void)hipStreamDestroy(s->chain_stream);
    for (auto& e : s->kry_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->kry_pin) (void)hipHostFree(s->kry_pin);
}

// ---------------------------------------------------------------------------
// Static scratch of parareal_solve_static: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel or a
// copy (on the host the name is a stand-in, not a device address); it uses
// the per-device address hipGetSymbolAddress returns.
// ---------------------------------------------------------------------------
constexpr uint64_t kStaticScratchBytes = PR_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current).
pr_status static_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return PR_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PR_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PR_OK;
}

}  // namespace

extern "C" {

pr_status parareal_create(const pr_grid* grid, const pr_model* model, const pr_payoff* payoff,
                          const pr_options* opt, void* device_workspace, uint64_t workspace_bytes,
                          void* hip_stream, pr_solver** out) {
    if (!out) return PR_EINVAL;
    *out = nullptr;
    pr_solver* s = new (std::nothrow) pr_solver();
    if (!s) return PR_ENOMEM;
    const pr_status st = setup_solver(s, grid, model, payoff, opt, device_workspace,
                                      workspace_bytes, hip_stream, true);
    if (st != PR_OK) {
        release_runtime_objects(s);
        delete s;
        return st;
    }
    *out = s;
    return PR_OK;
}

pr_status parareal_solve_static(const pr_grid* grid, const pr_model* model,
                                const pr_payoff* payoff, const pr_options* opt, void* hip_stream,
                                double* v_out, pr_stats* st) {
    if (st) std::memset(st, 0, sizeof(*st));
    if (!grid || !model || !payoff || !opt || !v_out) return PR_EINVAL;
    if (opt->coarse_kind == PR_G_FNO) return PR_EINVAL;   // needs an attached operator
    if (!valid_basic(grid, opt, nullptr)) return PR_EINVAL;
    if (layout(grid, opt).total > kStaticScratchBytes) return PR_ENOMEM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PR_EDEVICE;
    void* ws = nullptr;
    pr_status r = static_scratch(dev, &ws);
    if (r != PR_OK) return r;
    auto t0 = std::chrono::steady_clock::now();
    pr_solver s;   // on the stack: no runtime objects, no device memory
    pr_options o = *opt;
    o.flags &= ~(PR_FLAG_TIME_STEPS | PR_FLAG_GRAPH);
    r = setup_solver(&s, grid, model, payoff, &o, ws, kStaticScratchBytes, hip_stream, false);
    if (r == PR_OK) {
        try {
            r = do_solve(&s, v_out, st);
        } catch (...) {
            r = PR_EDEVICE;
        }
    }
    if (st) {
        st->status = r;
        st->fine_steps = s.mF;
        st->coarse_steps = s.mG;
        st->workspace_bytes = s.L.total;
        st->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return r;
}

pr_status parareal_solve(pr_solver* s, double* v_out, pr_stats* st) {
    if (!s || !v_out) return PR_EINVAL;
    if (st) std::memset(st, 0, sizeof(*st));
    auto t0 = std::chrono::steady_clock::now();
    pr_status r;
    try {
        r = do_solve(s, v_out, st);
    } catch (...) {
        s->err = "internal error";
        r = PR_EDEVICE;
    }
    if (st) {
        st->status = r;
        st->fine_steps = s->mF;
        st->coarse_steps = s->mG;
        st->workspace_bytes = s->L.total;
        st->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return r;
}

pr_status parareal_serial_fine(pr_solver* s, double* v_out, pr_stats* st) {
    if (!s || !v_out) return PR_EINVAL;
    if (st) std::memset(st, 0, sizeof(*st));
    auto t0 = std::chrono::steady_clock::now();
    pr_status r;
    try {
        r = do_serial_fine(s, v_out, st);
    } catch (...) {
        s->err = "internal error";
        r = PR_EDEVICE;
    }
    if (st) {
        st->status = r;
        st->fine_steps = s->mF;
        st->coarse_steps = s->mG;
        st->iters = 0;
        st->workspace_bytes = s->L.total;
        st->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return r;
}

pr_status parareal_apply(pr_solver* s, int32_t op, int32_t slice, const double* in, double* out) {
    if (!s || !in || !out || in == out) return PR_EINVAL;
    if (slice < 0 || slice >= s->N || (op != PR_OP_FINE && op != PR_OP_COARSE)) return PR_EINVAL;
    const Grid& g = s->fg;
    double* U = s->U(0);
    double* Us = U + (long long)slice * g.stride;
    double* Us1 = U + (long long)(slice + 1) * g.stride;
    HIPCHK(launch_pack(in, Us, g, s->stream));
    if (op == PR_OP_FINE) {
        const float* d = nullptr;
        const double* w = nullptr;
        pr_status r = fine_sweep(s, U, slice, 1, false, &d, &w, nullptr);
        if (r != PR_OK) return r;
        r = fine_result_to_state(s, Us, d ? d + (long long)slice * g.stride : nullptr,
                                 w ? w + (long long)slice * g.stride : nullptr, Us1);
        if (r != PR_OK) return r;
    } else if (s->fineg) {
        if (s->fnog && !s->fno) {
            s->err = "PR_G_FNO solver without an attached operator (parareal_attach_fno)";
            return PR_EMODEL;
        }
        pr_status r = fine_g(s, U, slice, Us1);
        if (r != PR_OK) return r;
    } else {
        ChainArgs ca = chain_args(s, slice, slice + 1, 1);
        HIPCHK(launch_chain(U, s->at<double>(s->L.Gold), s->at<double>(s->L.dcor),
                            s->at<double>(s->L.cst), s->at<float>(s->L.lbc), ca, s->stream));
        HIPCHK(launch_prolong(s->at<double>(s->L.Gold), U, g, s->nc, s->q, slice, slice + 1,
                              s->stream));
    }
    HIPCHK(launch_unpack(Us1, out, g, s->bcf, (slice + 1) * s->dT, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return PR_OK;
}

pr_status parareal_attach_fno(pr_solver* s, pr_fno* f) {
    if (!s || !f) return PR_EINVAL;
    if (s->opt.coarse_kind != PR_G_FNO) {
        s->err = "the solver was not created with PR_G_FNO";
        return PR_EINVAL;
    }
    s->fno = f;
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : s->graph_defs) (void)hipGraphDestroy(kv.second);
    s->graphs.clear();
    s->graph_defs.clear();
    return PR_OK;
}

pr_status parareal_fno_pair(pr_solver* s, int32_t slice, const double* v0, const double* v1,
                            int32_t base, float* pair_out) {
    if (!s || !v0 || !v1 || !pair_out) return PR_EINVAL;
    if (base < PR_FNO_BASE_ZERO || base > PR_FNO_BASE_FINE_LOD) return PR_EINVAL;
    if (s->opt.coarse_kind != PR_G_FNO) {
        s->err = "the solver was not created with PR_G_FNO";
        return PR_EINVAL;
    }
    if (slice < 0 || slice >= s->N) return PR_EINVAL;
    const Grid& g = s->fg;
    double* u = s->at<double>(s->L.tg);
    double* w0 = s->at<double>(s->L.fwc);
    double* w1 = s->at<double>(s->L.fwc1);
    HIPCHK(launch_pack(v0, u, g, s->stream));
    pr_status r = fno_restrict(s, u, slice * s->dT, w0);
    if (r != PR_OK) return r;
    double* wb = nullptr;
    if (base == PR_FNO_BASE_FINE_LOD) {
        double* lo = s->at<double>(s->L.Gf);   // one-slice temporary outside a solve
        r = fno_fine_lod(s, u, slice, lo);
        if (r != PR_OK) return r;
        wb = s->at<double>(s->L.fwb);
        r = fno_restrict(s, lo, (slice + 1) * s->dT, wb);
        if (r != PR_OK) return r;
    }
    HIPCHK(launch_pack(v1, u, g, s->stream));
    r = fno_restrict(s, u, (slice + 1) * s->dT, w1);
    if (r != PR_OK) return r;
    if (base == PR_FNO_BASE_LOD) {
        wb = s->at<double>(s->L.fwb);
        r = fno_lod_base(s, w0, slice, wb);
        if (r != PR_OK) return r;
    }
    HIPCHK(launch_pair(w0, w1, wb, pair_out, s->bcf, s->grid.s_max, slice * s->dT,
                       (slice + 1) * s->dT, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return PR_OK;
}

pr_status parareal_fno_pairs(pr_solver* s, int32_t base, float* pairs_out) {
    if (!s || !pairs_out) return PR_EINVAL;
    if (base < PR_FNO_BASE_ZERO || base > PR_FNO_BASE_FINE_LOD) return PR_EINVAL;
    if (s->opt.coarse_kind != PR_G_FNO) {
        s->err = "the solver was not created with PR_G_FNO";
        return PR_EINVAL;
    }
    const Grid& g = s->fg;
    double* U = s->U(0);
    s->sweep_launches = 0;
    s->sweep_bytes = 0;
    HIPCHK(launch_payoff(U, g, s->bcf, s->stream));
    for (int n = 0; n < s->N; ++n) {   // serial F, every slice state kept
        const float* d = nullptr;
        const double* w = nullptr;
        pr_status r = fine_sweep(s, U, n, 1, false, &d, &w, nullptr);
        if (r != PR_OK) return r;
        r = fine_result_to_state(s, U + (long long)n * g.stride,
                                 d ? d + (long long)n * g.stride : nullptr,
                                 w ? w + (long long)n * g.stride : nullptr,
                                 U + (long long)(n + 1) * g.stride);
        if (r != PR_OK) return r;
    }
    double* w0 = s->at<double>(s->L.fwc);
    double* w1 = s->at<double>(s->L.fwc1);
    pr_status r = fno_restrict(s, U, 0.0, w0);
    if (r != PR_OK) return r;
    for (int n = 0; n < s->N; ++n) {
        r = fno_restrict(s, U + (long long)(n + 1) * g.stride, (n + 1) * s->dT, w1);
        if (r != PR_OK) return r;
        double* wb = nullptr;
        if (base == PR_FNO_BASE_LOD) {
            wb = s->at<double>(s->L.fwb);
            r = fno_lod_base(s, w0, n, wb);
            if (r != PR_OK) return r;
        }
        if (base == PR_FNO_BASE_FINE_LOD) {
            double* lo = s->at<double>(s->L.tg);
            r = fno_fine_lod(s, U + (long long)n * g.stride, n, lo);
            if (r != PR_OK) return r;
            wb = s->at<double>(s->L.fwb);
            r = fno_restrict(s, lo, (n + 1) * s->dT, wb);
            if (r != PR_OK) return r;
        }
        HIPCHK(launch_pair(w0, w1, wb, pairs_out + (long long)n * 4 * 64 * 64, s->bcf,
                           s->grid.s_max, n * s->dT, (n + 1) * s->dT, s->stream));
        std::swap(w0, w1);
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return PR_OK;
}

pr_status parareal_destroy(pr_solver* s) {
    if (!s) return PR_EINVAL;
    release_runtime_objects(s);
    delete s;
    return PR_OK;
}

}  // extern "C"

// ===========================================================================
// Serving: continuous batching over a caller-provided device arena.
// ===========================================================================
#include <deque>

namespace {

struct Req {
    int64_t id = 0;
    pr_grid g{};
    pr_model m{};
    pr_payoff p{};
    pr_options o{};
    double* v_out = nullptr;
    uint64_t bytes = 0, off = 0;
    pr_solver* s = nullptr;
    int state = 0;   // 0 queued, 1 iteration in flight, 2 result write in flight, 3 done
    int k = 0;       // iterations completed
    int slot = -1;   // pinned read-back slot
    hipEvent_t ev = nullptr;
    pr_status status = PR_OK;
    double inc = 0;
    double inc_prev[2] = {0.0, 0.0};   // PR_G_FNO: the two increments before the last
    bool fnog = false;                 // submitted with PR_G_FNO
    int fallback = 0;                  // the neural G diverged; restarted on LOD
    std::chrono::steady_clock::time_point t_submit, t_admit, t_done;
};

}  // namespace

struct pr_server {
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> size of free blocks
    std::vector<hipStream_t> streams;
    unsigned long long* pinned = nullptr;  // 4 words per slot
    std::vector<int> free_slots;
    std::deque<int64_t> queue;
    std::map<int64_t, Req> reqs;
    std::vector<int64_t> resident;
    int64_t next_id = 1;
    int max_resident = 1, rr = 0, peak_resident = 0, n_done = 0;
    int max_queued = 0;                   // 0: no bound on waiting requests
    int64_t n_rejected = 0;               // submissions refused with PR_EBUSY
    pr_fno* fno = nullptr;                // operator of PR_G_FNO requests
    int n_fno = 0;                        // PR_G_FNO requests queued or resident
    uint64_t used = 0, peak_bytes = 0;
    // PR_SERVER_RAGGED_F: the requests that are ready for an iteration gather
    // here during a progress pass; their fine sweeps then share launches on
    // one of fstreams (in turn, so that consecutive passes overlap)
    bool ragged = false;
    std::vector<hipStream_t> fstreams;
    std::vector<int64_t> ready;
    int64_t ragged_ticks = 0, ragged_launches = 0, ragged_entries = 0;
};

namespace {

// PR_SERVER_RAGGED_F: streams the shared fine launches of successive progress
// passes take in turn (at most n_streams)
constexpr int kRaggedStreams = 4;

bool arena_alloc(pr_server* sv, uint64_t bytes, uint64_t* off) {
    bytes = al(bytes);
    for (auto it = sv->free_.begin(); it != sv->free_.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const uint64_t rest = it->second - bytes, at = it->first + bytes;
            sv->free_.erase(it);
            if (rest) sv->free_[at] = rest;
            sv->used += bytes;
            sv->peak_bytes = std::max(sv->peak_bytes, sv->used);
            return true;
        }
    }
    return false;
}

void arena_free(pr_server* sv, uint64_t off, uint64_t bytes) {
    bytes = al(bytes);
    sv->used -= bytes;
    auto it = sv->free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != sv->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        sv->free_.erase(nx);
    }
    if (it != sv->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            sv->free_.erase(it);
        }
    }
}

// The read-back of r's norms after its iteration, and the event progress polls.
pr_status req_readback(pr_server* sv, Req& r) {
    pr_solver* s = r.s;
    HIPCHK(hipMemcpyAsync(sv->pinned + 4 * r.slot, s->red(), 3 * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipEventRecord(r.ev, s->stream));
    return PR_OK;
}

// Enqueue iteration k of request r and the read-back of its norms (ragged
// mode: mark r ready; flush_ready enqueues it at the end of the pass).
pr_status req_enqueue_iteration(pr_server* sv, Req& r) {
    if (sv->ragged) {
        sv->ready.push_back(r.id);
        return PR_OK;
    }
    pr_solver* s = r.s;
    double* Ucur = s->U(r.k & 1);
    double* Unext = s->U((r.k + 1) & 1);
    pr_status st = iteration_phase(s, r.k, Ucur, Unext, nullptr);
    if (st != PR_OK) return st;
    return req_readback(sv, r);
}

// The ragged tick: the fine sweeps of every ready request in shared launches,
// then each request's coarse chain, correction and norm read-back on its own
// stream, from the end of its own sweep.  Sweeps are bucketed by their work
// per step (point-steps per step in powers of 4): a bucket shares launches on
// one of the ragged streams, and different buckets take different streams, so
// that a small request's rounds do not wait behind a large request's share of
// the same launch.  On an error every request of the tick is listed in
// *failed (its work may be partly enqueued).
pr_status flush_ready(pr_server* sv, std::vector<int64_t>* failed) {
    const size_t nr = sv->ready.size();
    std::vector<RaggedSweep> jobs(nr);
    std::map<int, std::vector<size_t>> buckets;   // log4(points per step) -> jobs
    pr_status st = PR_OK;
    for (size_t i = 0; i < nr && st == PR_OK; ++i) {
        Req& r = sv->reqs[sv->ready[i]];
        pr_solver* s = r.s;
        st = ragged_begin(s, s->U(r.k & 1), r.k, s->N - r.k, &jobs[i]);
        if (st == PR_OK && hipEventRecord(r.ev, s->stream) != hipSuccess) st = PR_EDEVICE;
        jobs[i].done = r.ev;   // re-recorded on the bucket's stream after the last launch
        const double pts = (double)(s->N - r.k) * s->fg.nin * s->fg.nin;
        buckets[(int)std::floor(std::log(std::max(pts, 1.0)) / std::log(4.0))].push_back(i);
    }
    int b = 0;
    for (auto it = buckets.begin(); it != buckets.end() && st == PR_OK; ++it, ++b) {
        hipStream_t fs = sv->fstreams[(size_t)(sv->ragged_ticks + b) % sv->fstreams.size()];
        std::vector<RaggedSweep> bj;
        for (size_t i : it->second) {
            if (hipStreamWaitEvent(fs, jobs[i].done, 0) != hipSuccess) st = PR_EDEVICE;
            bj.push_back(jobs[i]);
        }
        if (st == PR_OK) st = ragged_run(bj, fs, &sv->ragged_launches, &sv->ragged_entries);
        for (size_t k = 0; k < it->second.size(); ++k) jobs[it->second[k]] = bj[k];
    }
    for (size_t i = 0; i < nr && st == PR_OK; ++i) {
        Req& r = sv->reqs[sv->ready[i]];
        pr_solver* s = r.s;
        if (hipStreamWaitEvent(s->stream, r.ev, 0) != hipSuccess) {
            st = PR_EDEVICE;
            break;
        }
        const float* d = nullptr;
        const double* w = nullptr;
        ragged_end(jobs[i], &d, &w);
        st = iteration_after_sweep(s, r.k, s->U(r.k & 1), s->U((r.k + 1) & 1),
                                   s->fp32 ? (const void*)d : (const void*)w, false);
        if (st == PR_OK) st = req_readback(sv, r);
    }
    if (st != PR_OK) {
        failed->assign(sv->ready.begin(), sv->ready.end());
        for (hipStream_t fs : sv->fstreams) (void)hipStreamSynchronize(fs);
    } else {
        sv->ragged_ticks += 1;
    }
    sv->ready.clear();
    return st;
}

pr_status req_admit(pr_server* sv, Req& r) {
    // PR_G_FNO requests share the first stream: one request at a time uses the
    // operator's activation workspace
    const int si = r.fnog ? 0 : sv->rr++ % (int)sv->streams.size();
    pr_options o = r.o;
    o.flags &= ~(PR_FLAG_GRAPH | PR_FLAG_TIME_STEPS);
    // requests already overlap across the server's streams: no per-request
    // chain stream (it would be created and destroyed at every admission)
    o.flags |= PR_FLAG_SERIAL_CHAIN;
    pr_status st = parareal_create(&r.g, &r.m, &r.p, &o, sv->arena + r.off, r.bytes,
                                   sv->streams[si], &r.s);
    if (st != PR_OK) return st;
    pr_solver* s = r.s;
    if (r.fnog) {
        st = parareal_attach_fno(s, sv->fno);
        if (st != PR_OK) return st;
    }
    if (hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) != hipSuccess) return PR_EDEVICE;
    r.slot = sv->free_slots.back();
    sv->free_slots.pop_back();
    st = init_phase(s, s->U(0), s->U(1));
    if (st != PR_OK) return st;
    r.k = 0;
    r.state = 1;
    return req_enqueue_iteration(sv, r);
}

void req_retire(pr_server* sv, Req& r) {
    if (r.fnog) sv->n_fno -= 1;
    if (r.ev) (void)hipEventDestroy(r.ev);
    r.ev = nullptr;
    if (r.s) parareal_destroy(r.s);
    r.s = nullptr;
    if (r.slot >= 0) sv->free_slots.push_back(r.slot);
    r.slot = -1;
    arena_free(sv, r.off, r.bytes);
    r.state = 3;
    r.t_done = std::chrono::steady_clock::now();
    sv->n_done++;
}

// The iteration of r has finished: stop or continue.
pr_status req_advance(pr_server* sv, Req& r) {
    pr_solver* s = r.s;
    const unsigned long long* h = sv->pinned + 4 * r.slot;
    double inc, scint;
    std::memcpy(&inc, &h[0], 8);
    std::memcpy(&scint, &h[1], 8);
    r.k += 1;
    r.inc = inc;
    // PR_G_FNO: a diverging neural G (non-finite, or two increments in a row
    // growing) restarts the solve on the LOD propagator, as parareal_solve does
    if (s->fnog && !(s->opt.flags & PR_FLAG_NO_FALLBACK) &&
        (h[2] || (r.k >= 3 && inc > r.inc_prev[1] && r.inc_prev[1] > r.inc_prev[0]))) {
        pr_status st = switch_to_lod(s);
        if (st != PR_OK) return st;
        r.fallback = 1;
        r.k = 0;
        r.inc_prev[0] = r.inc_prev[1] = 0.0;
        st = init_phase(s, s->U(0), s->U(1));
        if (st != PR_OK) return st;
        return req_enqueue_iteration(sv, r);
    }
    r.inc_prev[0] = r.inc_prev[1];
    r.inc_prev[1] = inc;
    const double scale = std::max(scint, s->ring_max_T);
    const double thr = s->opt.tol_relative ? s->opt.tol * scale : s->opt.tol;
    bool stop = false;
    if (h[2]) { r.status = PR_ENONFINITE; stop = true; }
    else if (inc < thr || r.k == s->N) stop = true;
    else if (r.k == s->maxit) { r.status = PR_ENOTCONV; stop = true; }
    if (!stop) return req_enqueue_iteration(sv, r);
    HIPCHK(launch_unpack(s->U(r.k & 1) + (long long)s->N * s->fg.stride, r.v_out, s->fg, s->bcf,
                         s->N * s->dT, s->stream));
    HIPCHK(hipEventRecord(r.ev, s->stream));
    r.state = 2;
    return PR_OK;
}

}  // namespace

extern "C" {

uint64_t pr_server_footprint(const pr_grid* grid, const pr_options* opt) {
    const uint64_t b = parareal_workspace_bytes(grid, opt);
    return b ? al(b) : 0;
}

pr_status pr_server_create(void* arena, uint64_t arena_bytes, const pr_server_options* opt,
                           pr_server** out) {
    if (!out || !arena || !opt) return PR_EINVAL;
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(arena) % kAlign) return PR_EINVAL;
    if (opt->max_resident < 1 || opt->n_streams < 1 || opt->n_streams > 32 || opt->max_queued < 0 ||
        (opt->flags & ~PR_SERVER_RAGGED_F) != 0)
        return PR_EINVAL;
    pr_server* sv = new (std::nothrow) pr_server();
    if (!sv) return PR_ENOMEM;
    sv->arena = reinterpret_cast<char*>(arena);
    sv->arena_bytes = arena_bytes / kAlign * kAlign;
    sv->free_[0] = sv->arena_bytes;
    sv->max_resident = opt->max_resident;
    sv->max_queued = opt->max_queued;
    for (int i = 0; i < opt->n_streams; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            pr_server_destroy(sv);
            return PR_EDEVICE;
        }
        sv->streams.push_back(st);
    }
    if (opt->flags & PR_SERVER_RAGGED_F) {
        sv->ragged = true;
        const int nf = std::min(opt->n_streams, kRaggedStreams);
        for (int i = 0; i < nf; ++i) {
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                pr_server_destroy(sv);
                return PR_EDEVICE;
            }
            sv->fstreams.push_back(st);
        }
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&sv->pinned),
                      sizeof(unsigned long long) * 4 * (size_t)sv->max_resident) != hipSuccess) {
        sv->pinned = nullptr;
        pr_server_destroy(sv);
        return PR_EDEVICE;
    }
    for (int i = sv->max_resident - 1; i >= 0; --i) sv->free_slots.push_back(i);
    *out = sv;
    return PR_OK;
}

pr_status pr_server_submit(pr_server* sv, const pr_grid* grid, const pr_model* model,
                           const pr_payoff* payoff, const pr_options* opt, double* v_out,
                           int64_t* id_out) {
    if (!sv || !grid || !model || !payoff || !opt || !v_out || !id_out) return PR_EINVAL;
    int32_t mf = 0, mg = 0;
    pr_status st = parareal_plan(grid, model, opt, &mf, &mg, nullptr, nullptr);
    if (st != PR_OK) return st;
    if (opt->coarse_kind == PR_G_FNO && !sv->fno) return PR_EMODEL;   // pr_server_attach_fno
    // the BiCGStab steps poll their convergence on the host; the server never blocks
    if (opt->fine_scheme != PR_FINE_EXPLICIT || opt->coarse_kind == PR_G_IMPLICIT) return PR_EINVAL;
    Req r;
    r.id = sv->next_id++;
    r.g = *grid;
    r.m = *model;
    r.p = *payoff;
    r.o = *opt;
    r.v_out = v_out;
    r.bytes = pr_server_footprint(grid, opt);
    if (r.bytes == 0) return PR_EINVAL;
    if (r.bytes > sv->arena_bytes) return PR_ENOMEM;
    if (sv->max_queued > 0 && (int)sv->queue.size() >= sv->max_queued) {
        sv->n_rejected += 1;
        return PR_EBUSY;
    }
    r.t_submit = std::chrono::steady_clock::now();
    r.fnog = opt->coarse_kind == PR_G_FNO;
    if (r.fnog) sv->n_fno += 1;
    *id_out = r.id;
    sv->queue.push_back(r.id);
    sv->reqs.emplace(r.id, r);
    return PR_OK;
}

pr_status pr_server_progress(pr_server* sv, int32_t* n_resident, int32_t* n_queued,
                             int32_t* n_done) {
    if (!sv) return PR_EINVAL;
    pr_status first_err = PR_OK;
    // 1. advance requests whose in-flight work has finished
    for (size_t i = 0; i < sv->resident.size();) {
        Req& r = sv->reqs[sv->resident[i]];
        const hipError_t q = hipEventQuery(r.ev);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        bool retire = false;
        if (q != hipSuccess) {
            r.status = PR_EDEVICE;
            retire = true;
        } else if (r.state == 1) {
            // iteration done: enqueue the next one or the write of the result (state 2)
            const pr_status st = req_advance(sv, r);
            if (st != PR_OK) {
                r.status = st;
                retire = true;
            }
        } else {
            retire = true;   // state 2: the result has been written
        }
        if (retire) {
            // a solve's own outcome (not converged, a non-finite iterate) is the
            // request's status, reported by pr_server_poll only
            if (r.status != PR_OK && r.status != PR_ENOTCONV && r.status != PR_ENONFINITE &&
                first_err == PR_OK)
                first_err = r.status;
            if (r.status != PR_OK && r.s) (void)hipStreamSynchronize(r.s->stream);
            req_retire(sv, r);
            sv->resident.erase(sv->resident.begin() + i);
            continue;
        }
        ++i;
    }
    // 2. admit queued requests in order while they fit
    while (!sv->queue.empty() && (int)sv->resident.size() < sv->max_resident) {
        Req& r = sv->reqs[sv->queue.front()];
        if (!arena_alloc(sv, r.bytes, &r.off)) break;
        sv->queue.pop_front();
        r.t_admit = std::chrono::steady_clock::now();
        pr_status st = req_admit(sv, r);
        sv->resident.push_back(r.id);
        sv->peak_resident = std::max(sv->peak_resident, (int)sv->resident.size());
        if (st != PR_OK) {
            r.status = st;
            if (first_err == PR_OK) first_err = st;
            if (r.s) (void)hipStreamSynchronize(r.s->stream);
            req_retire(sv, r);
            sv->resident.pop_back();
        }
    }
    // 3. ragged mode: the fine sweeps of every request made ready above
    if (sv->ragged && !sv->ready.empty()) {
        std::vector<int64_t> failed;
        const pr_status st = flush_ready(sv, &failed);
        if (st != PR_OK) {
            if (first_err == PR_OK) first_err = st;
            for (int64_t id : failed) {
                Req& r = sv->reqs[id];
                r.status = st;
                if (r.s) (void)hipStreamSynchronize(r.s->stream);
                req_retire(sv, r);
                sv->resident.erase(std::find(sv->resident.begin(), sv->resident.end(), id));
            }
        }
    }
    if (n_resident) *n_resident = (int32_t)sv->resident.size();
    if (n_queued) *n_queued = (int32_t)sv->queue.size();
    if (n_done) *n_done = sv->n_done;
    return first_err;
}

pr_status pr_server_poll(pr_server* sv, int64_t id, int32_t* done, pr_request_info* info) {
    if (!sv || !done) return PR_EINVAL;
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return PR_EINVAL;
    const Req& r = it->second;
    *done = r.state == 3;
    if (*done && info) {
        info->status = r.status;
        info->iters = r.k;
        info->last_increment = r.inc;
        info->latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
        info->queue_ms = std::chrono::duration<double, std::milli>(r.t_admit - r.t_submit).count();
        info->workspace_bytes = r.bytes;
        info->coarse_fallback = r.fallback;
        info->reserved_ = 0;
    }
    return PR_OK;
}

pr_status pr_server_attach_fno(pr_server* sv, pr_fno* f) {
    if (!sv) return PR_EINVAL;
    if (sv->n_fno > 0 && f != sv->fno) return PR_EINVAL;   // in use by queued or resident requests
    sv->fno = f;
    return PR_OK;
}

pr_status pr_server_peaks(const pr_server* sv, int32_t* peak_resident, uint64_t* peak_bytes) {
    if (!sv) return PR_EINVAL;
    if (peak_resident) *peak_resident = sv->peak_resident;
    if (peak_bytes) *peak_bytes = sv->peak_bytes;
    return PR_OK;
}

pr_status pr_server_rejected(const pr_server* sv, int64_t* n_rejected) {
    if (!sv || !n_rejected) return PR_EINVAL;
    *n_rejected = sv->n_rejected;
    return PR_OK;
}

pr_status pr_server_ragged_stats(const pr_server* sv, int64_t* ticks, int64_t* launches,
                                 int64_t* entries) {
    if (!sv) return PR_EINVAL;
    if (ticks) *ticks = sv->ragged_ticks;
    if (launches) *launches = sv->ragged_launches;
    if (entries) *entries = sv->ragged_entries;
    return PR_OK;
}

pr_status pr_server_destroy(pr_server* sv) {
    if (!sv) return PR_EINVAL;
    for (hipStream_t st : sv->fstreams) (void)hipStreamSynchronize(st);
    for (hipStream_t st : sv->streams) (void)hipStreamSynchronize(st);
    for (int64_t id : sv->resident) {
        Req& r = sv->reqs[id];
        if (r.ev) (void)hipEventDestroy(r.ev);
        if (r.s) parareal_destroy(r.s);
    }
    for (hipStream_t st : sv->streams) (void)hipStreamDestroy(st);
    for (hipStream_t st : sv->fstreams) (void)hipStreamDestroy(st);
    if (sv->pinned) (void)hipHostFree(sv->pinned);
    delete sv;
    return PR_OK;
}

}  // extern "C"
