// internal.hpp -- structures shared by the host driver and the gfx950 kernels.
//
// Storage layout of every fine-grid state in the workspace ("interior layout"):
// only the (n-2) x (n-2) interior nodes are stored, row i-1 (S1 index i) at
// offset (i-1)*pitch, column j-1 (S2 index j) contiguous, pitch a multiple of
// 64 elements so that each 64-lane wavefront row load is aligned.  The
// Dirichlet ring is never stored: every kernel evaluates it from its closed
// form g(S1, S2, tau) when a stencil reaches it.  Slices follow each other at
// slice_stride = (n-2)*pitch elements.
#pragma once
#include <cstdint>

namespace pr {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 wavefronts per workgroup
constexpr int kChainThreads = 1024;  // one workgroup runs the whole coarse chain
constexpr int kChainMaxN = 257;      // coarse nodes per side: 4 (n - 1) ring nodes <= 1024 threads

// Dirichlet data and payoff; everything in index form needs only h.
struct Bc {
    int payoff;   // PR_PAYOFF_*
    int kind;     // PR_BC_*
    double w1, w2, K;
    double s1, s2, rho, r;
    double h;     // grid spacing of the grid this struct describes
    double K2;    // cash-or-nothing: second strike (K is the first)
    double cash;  // cash-or-nothing: cash amount
};

// Model coefficients in index form (h cancels): at node (i, j)
//   alpha = a1 i^2, beta = a2 j^2, gamma = g12 i j, mu = hr i, nu = hr j.
struct Coef {
    double a1, a2, g12, hr, r;
};

struct Grid {
    int n;            // nodes per side including the ring
    int nin;          // n - 2
    int pitch;        // stored row pitch in elements
    long long stride; // elements per slice
};

// One explicit step (or the FP32 preparation step) over `count` slices
// starting at `first`: slice s uses base time first_tau + s*dT.
struct StepArgs {
    Grid g;
    Coef c;
    Bc bc;
    double dt;
    double dT;        // slice length
    int first;        // first slice index (absolute, for time)
    int count;        // slices in this launch
    int step;         // index q of the step: input at tau = T_n + q dt
    int rows;         // rows per wavefront chunk
    int nchunks;
    int nstrips;
    long long in_off, out_off;   // element offsets of slice `first` in in/out
};

// One solver's share of a ragged multi-request step launch: its operands, its
// launch arguments (geometry as for its own launch) and its first workgroup.
struct TbEntry {
    const void* in;    // float (increments) or double (states), as the launch's type
    const float* lb;   // FP32 increment form: dt L b; nullptr for FP64 states
    void* out;
    const void* wt;    // the solver's row-weight table
    StepArgs a;
    int block0;        // workgroups [block0, next entry's block0) are this entry's
};
constexpr int kTbBatchMax = 8;   // entries per launch (about 2 KB of kernel arguments)
struct TbBatch {
    int n;         // entries in use
    int nblocks;   // workgroups of the launch
    TbEntry e[kTbBatchMax];
};

// Coarse chain over slices [k0, k1) on a coarse grid of nc nodes per side.
struct ChainArgs {
    Grid fg;          // fine grid (interior layout)
    int nc;           // coarse nodes per side
    int q;            // (n - 1) / (nc - 1)
    int k0, k1;
    int steps;        // coarse steps per slice
    int init;         // 1: c_{n+1} = Gc(c_n) (initial sweep); 0: correction chain
    int fp32;         // 1: increment form with FP32 increments
    Coef c;
    Bc bc;            // coarse h
    double dt, dT;
    void* gstate;     // 2 nc^2 elements in global memory holding the stepped coarse
                      // state when it does not fit in LDS; nullptr: LDS
    const double* foldc;   // [slice][nc][nc]: F(U^k_n) at the coincident nodes
};

// Implicit-Euler fine steps by BiCGStab (krylov.hip).
struct KrylovArgs {
    Grid g;
    Coef c;
    Bc bc;
    double dt;      // implicit step
    double dT;      // slice length
    int first;      // first slice index (absolute, for time)
    int count;      // slices in the sweep
    int step;       // step q of the slice: the new time is T_n + (q + 1) dt
    int rows;       // interior rows per workgroup
    int nblk;       // workgroups per slice (= partials per slice)
    int it;         // BiCGStab iteration (selects the scalar slot and the p / v buffers)
    double tol2;    // squared relative residual tolerance
};

// Per-slice scalars: two slots alternating by iteration parity, then flags.
struct KScal {
    double rho[2], alpha[2], omega[2];
    double bb;         // (b, b)
    double rr;         // (r, r) when the slice finished (or at the iteration cap)
    int done;          // 1 once converged (or broke down)
    int iters;         // iterations performed
    int breakdown;     // 1 if the slice stopped without meeting the tolerance
    int verified;      // 1 once the true residual b - A x has been checked
    int restarts;      // restarts from the true residual so far
    int pad_;
};

struct KrylovBufs {
    double *B, *R, *RH, *P[2], *V[2], *S, *T;   // count slices each (interior layout)
    double *partA, *partB, *partC;           // count * nblk (* 2) partial sums
    KScal* sc;                               // count scalar records
    int* ndone;                              // finished-slice counter (device)
    int* hpoll;                              // 2 pinned host slots for ndone, or nullptr:
    void* pev[2];                            // with their events (hipEvent_t), the host
                                             // reads a poll one round of iterations late
};

}  // namespace pr
