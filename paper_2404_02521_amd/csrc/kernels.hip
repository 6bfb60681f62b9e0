// kernels.hip -- gfx950 kernels of the Parareal hot path.
//
//  k_fine_prep   : the first explicit Euler step of the FP32 increment form
//                  over a batch of time slices: evaluates L b of the centred
//                  9-point operator of Eq. (fd) (Sec. 3.2) in FP64 for the FP64
//                  slice base b and writes dt*L b (the stored term of every
//                  later step, and the first increment).
//  k_fine_tb     : S explicit steps of the same operator per launch
//                  (temporal blocking in registers), the hot kernel of F;
//                  k_row_weights fills its per-row weight table.
//  k_coarse_chain: the serial sweep of Eq. (parareal) (Sec. 3.1) restricted
//                  to the coarse grid, one workgroup, coarse state in LDS (in
//                  global memory when it does not fit).
//  k_gather_coincident: F(U^k_n) at the coarse nodes for all active slices,
//                  ahead of the chain.
//  k_correct     : U^{k+1}_{n+1} = F(U^k_n) + P(Gc_new - Gc_old) in FP64 over
//                  all active slices, fused with the max-increment reduction.
//  small kernels : payoff, prolongation of the initial sweep, pack / unpack
//                  between full grids and the interior layout, finalise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"
#include "step_tb.hpp"

namespace pr {


// ---------------------------------------------------------------------------
// Preparation step of the FP32 increment form.  Each wavefront owns a strip
// of 64 consecutive interior columns and a chunk of `rows` consecutive rows of
// one slice.  It walks down the rows keeping rows i-1, i, i+1 of the FP64 base
// in registers: every value is loaded once (plus two halo columns), the j +- 1
// neighbours come from DPP wavefront shifts, and the Dirichlet ring is
// evaluated in place at the slice's start time.  Writes dt*L b, rounded once
// to FP32, to both outputs.
// ---------------------------------------------------------------------------
template <bool CHEAP>
__global__ __launch_bounds__(kBlock) void k_fine_prep(const double* __restrict__ in,
                                                      float* __restrict__ out,
                                                      float* __restrict__ out2, StepArgs a) {
#pragma clang fp contract(on)
    const int lane = threadIdx.x & 63;
    const int wid = xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) + (threadIdx.x >> 6);
    const int strip = wid % a.nstrips;
    const int t = wid / a.nstrips;
    const int chunk = t % a.nchunks;
    const int s = t / a.nchunks;
    if (s >= a.count) return;

    const int M = a.g.n;
    const int P = a.g.pitch;
    const int n = a.first + s;
    const double tau = n * a.dT;
    const double disc_tau = exp(-a.bc.r * tau);
    const int j0 = 1 + strip * kWave;
    const int j = j0 + lane;
    const int ia = 1 + chunk * a.rows;
    const int ib = min(ia + a.rows, M - 1);
    const double* src = in + (long long)s * a.g.stride;

    // ring value of the base at node (i, jj)
    auto ring = [&](int i, int jj) -> double {
        return ring_value<CHEAP>(a.bc, i * a.bc.h, jj * a.bc.h, tau, disc_tau);
    };
    // row i of the base as (left, centre, right) for this lane's column j
    auto load_row = [&](int i, double& l, double& c, double& r) {
        const bool ringrow = (i == 0) || (i == M - 1);
        const double* row = src + (long long)(i - 1) * P;
        if (ringrow) {
            c = (j <= M - 1) ? ring(i, j) : 0.0;
        } else {
            c = (j <= M - 2) ? row[j - 1] : (j == M - 1 ? ring(i, j) : 0.0);
        }
        double h = 0.0;
        const int jh = (lane == 0) ? j0 - 1 : j0 + kWave;
        if (lane < 2) {
            if (!ringrow && jh >= 1 && jh <= M - 2)
                h = row[jh - 1];
            else if (jh <= M - 1)
                h = ring(i, jh);
        }
        const double hl = bcast(h, 0), hr = bcast(h, 1);
        l = shr1(c);
        r = shl1(c);
        if (lane == 0) l = hl;
        if (lane == kWave - 1) r = hr;
    };

    const double fj = (double)j;
    const double bj = a.c.a2 * fj * fj;
    const double nj = a.c.hr * fj;
    const double gj = a.c.g12 * fj;
    const double rr = a.c.r;
    const bool active = (j <= M - 2);

    double lm, cm, rm, l0, c0, r0, lp, cp, rp;
    load_row(ia - 1, lm, cm, rm);
    load_row(ia, l0, c0, r0);
    for (int i = ia; i < ib; ++i) {
        load_row(i + 1, lp, cp, rp);
        const long long o = (long long)(i - 1) * P + (j - 1);
        const double fi = (double)i;
        const double A = a.c.a1 * fi * fi;
        const double Mu = a.c.hr * fi;
        const double G = gj * fi;
        const double uxx = cp - 2.0 * c0 + cm;
        const double uyy = r0 - 2.0 * c0 + l0;
        const double uxy = rp + lm - lp - rm;
        const double ux = cp - cm;
        const double uy = r0 - l0;
        const double L = A * uxx + bj * uyy + G * uxy + Mu * ux + nj * uy - rr * c0;
        if (active) {
            const float v = (float)(a.dt * L);
            out[(long long)s * a.g.stride + o] = v;
            out2[(long long)s * a.g.stride + o] = v;
        }
        lm = l0; cm = c0; rm = r0;
        l0 = lp; c0 = cp; r0 = rp;
    }
}

// ---------------------------------------------------------------------------
// Temporally blocked fine steps of one solver (the body is tb_body, step_tb.hpp).
// ---------------------------------------------------------------------------
template <int MODE, bool CHEAP, typename T, int S, int PF>
__global__ __launch_bounds__(kBlock) void k_fine_tb(const T* __restrict__ in,
                                                    const float* __restrict__ lb,
                                                    T* __restrict__ out,
                                                    const T* __restrict__ wt, StepArgs a) {
    // the wavefront index is uniform: taken through readfirstlane so that the
    // row / strip / slice logic of the body lives in scalar registers and branches
    const int wid = xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    tb_body<MODE, CHEAP, T, S, PF>(in, lb, out, wt, a, wid);
}

// ---------------------------------------------------------------------------
// Coarse chain (numerical G restricted to the coarse grid).  One workgroup of
// kChainThreads threads walks slices k0..k1-1 in order:
//   g_n   = Gc(c_n)                    (`steps` explicit steps in LDS)
//   d_n   = g_n - Gold_n,  Gold_n = g_n
//   c_n+1 = R F(U^k_n) + d_n           (init: c_n+1 = g_n)
// This is Eq. (parareal) at the coincident nodes: injection after bilinear
// prolongation returns the coarse values unchanged, so the chain never needs
// the fine grid except F at coincident nodes, which k_gather_coincident has
// collected into a.foldc before the chain starts.
// The stepped quantity (FP64 state, or FP32 increments over the FP64 base
// c_n) is double-buffered in LDS; c_n and the FP32 Lb = L c_n live in global
// memory (L2-resident).  Each thread owns one coarse column J and a segment of
// consecutive rows, walked with a 3-row register window; row coefficients
// come from an LDS table.  NC > 0 compiles the coarse side in (NC = a.nc),
// so that every neighbour and row offset becomes an immediate.  GB: the two
// state buffers live in global memory (a.gstate, L2-resident) for coarse grids
// whose state does not fit in LDS; the waves of the one workgroup share the
// CU's L1, so the per-step barrier orders them as it does LDS.
// ---------------------------------------------------------------------------
template <bool CHEAP, bool FP32, int NC, bool GB>
__global__ __launch_bounds__(kChainThreads) void k_coarse_chain(
    const double* __restrict__ Ucur, double* __restrict__ Gold, double* __restrict__ dcor,
    double* __restrict__ cst, float* __restrict__ lbc, ChainArgs a) {
    using T = typename std::conditional<FP32, float, double>::type;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int nc = NC > 0 ? NC : a.nc, nin = nc - 2, nn = nc * nc;
    const int q = a.q;
    const long long FS = a.fg.stride;
    const int FP = a.fg.pitch;
    const double hc = a.bc.h;
    // One explicit step u+ = u + dt (Lb + L u) with the operator in the form
    //   L = (A+Mu) u_{I+1} + (A-Mu) u_{I-1} + (B+Nu) u_{J+1} + (B-Nu) u_{J-1}
    //       + G (mixed difference) - (2A + 2B + r) u,
    // A = a1 I^2, Mu = hr I, B = a2 J^2, Nu = hr J, G = g12 I J, and dt folded
    // into the weights: per row [dt(A+Mu), dt(A-Mu), 1 - dt(2A+r), dt g12 I]
    // in LDS (read as a broadcast), per column dt(B+Nu), dt(B-Nu), 2 dt B in
    // registers; the FP32 path keeps dt Lb per node.
    T* tab = reinterpret_cast<T*>(lds);                 // 4*nc row weights
    T* buf0 = GB ? reinterpret_cast<T*>(a.gstate) : tab + 4 * nc;   // nc*nc
    T* buf1 = buf0 + nn;                                            // nc*nc
    for (int I = tid; I < nc; I += kChainThreads) {
        const double A = a.c.a1 * I * I, Mu = a.c.hr * I;
        tab[4 * I] = (T)(a.dt * (A + Mu));
        tab[4 * I + 1] = (T)(a.dt * (A - Mu));
        tab[4 * I + 2] = (T)(1.0 - a.dt * (2.0 * A + a.c.r));
        tab[4 * I + 3] = (T)(a.dt * a.c.g12 * I);
    }
    // Ring nodes: thread tid < 4*(nc-1) owns ring node number tid.
    const bool ring_thread = tid < 4 * (nc - 1);
    int rI = 0, rJ = 0;
    if (ring_thread) {
        const int e = nc - 1, r = tid;
        if (r < e) { rI = 0; rJ = r; }
        else if (r < 2 * e) { rI = r - e; rJ = e; }
        else if (r < 3 * e) { rI = e; rJ = e - (r - 2 * e); }
        else { rI = e - (r - 3 * e); rJ = 0; }
    }
    auto gring = [&](double t) {
        return ring_value<CHEAP>(a.bc, rI * hc, rJ * hc, t, exp(-a.bc.r * t));
    };
    // Column and row segment of this thread.
    const int ncolt = (nin + kWave - 1) / kWave * kWave;
    const int segs = kChainThreads / ncolt;
    const int rows = (nin + segs - 1) / segs;
    const int J = 1 + tid % ncolt;
    const int I0 = 1 + (tid / ncolt) * rows;
    const int nr = (J <= nin) ? max(0, min(rows, nc - 1 - I0)) : 0;
    const double bJd = a.c.a2 * J * J, nJd = a.c.hr * J;
    const T cpJ = (T)(a.dt * (bJd + nJd)), cmJ = (T)(a.dt * (bJd - nJd)),
            b2J = (T)(a.dt * 2.0 * bJd), fJ = (T)J;

    // c_{k0} = R U_{k0}
#pragma unroll 4
    for (int r = 0; r < nr; ++r)
        cst[(I0 + r) * nc + J] =
            Ucur[(long long)a.k0 * FS + (long long)((I0 + r) * q - 1) * FP + (J * q - 1)];
    __syncthreads();

    for (int n = a.k0; n < a.k1; ++n) {
        const double Tn = n * a.dT;
        const double gT = ring_thread ? gring(Tn) : 0.0;
        int first = 0;
        if (!FP32) {
            for (int r = 0; r < nr; ++r) buf0[(I0 + r) * nc + J] = (T)cst[(I0 + r) * nc + J];
            if (ring_thread) buf0[rI * nc + rJ] = (T)gT;
        } else {
            // Lb = L c_n in FP64 from the global c_n (ring g(T_n)); first
            // increment dt*Lb, ring increment 0 at T_n.
            if (ring_thread) cst[rI * nc + rJ] = gT;
            __syncthreads();
#pragma unroll 2
            for (int r = 0; r < nr; ++r) {
                const int I = I0 + r;
                const double* c = cst + I * nc + J;
                const double L = a.c.a1 * I * I * (c[nc] - 2.0 * c[0] + c[-nc]) +
                                 a.c.a2 * J * J * (c[1] - 2.0 * c[0] + c[-1]) +
                                 a.c.g12 * I * J * (c[nc + 1] + c[-nc - 1] - c[nc - 1] - c[-nc + 1]) +
                                 a.c.hr * I * (c[nc] - c[-nc]) + a.c.hr * J * (c[1] - c[-1]) -
                                 a.c.r * c[0];
                lbc[I * nc + J] = (float)(a.dt * L);
                buf0[I * nc + J] = (T)(a.dt * L);
            }
            if (ring_thread) buf0[rI * nc + rJ] = (T)(gring(Tn + a.dt) - gT);
            first = 1;
        }
        __syncthreads();
        T* cur = buf0;
        T* nxt = buf1;
        const double dq = exp(-a.bc.r * a.dt);
        double disc = ring_thread ? exp(-a.bc.r * (Tn + first * a.dt)) : 1.0;
        for (int st = first; st < a.steps; ++st) {
            if (nr > 0) {
                // three-row window in slots 0..2 (row I in slot (I - I0 + 2) % 3 after
                // it is loaded); the loop is unrolled by 3 so rotating it costs no moves.
                // dx = u_{J+1} - u_{J-1} of each window row gives the mixed
                // difference as dx_{I+1} - dx_{I-1}.
                T wl[3], wc[3], wr[3], dx[3];
                wl[0] = cur[(I0 - 1) * nc + J - 1]; wc[0] = cur[(I0 - 1) * nc + J];
                wr[0] = cur[(I0 - 1) * nc + J + 1];
                wl[1] = cur[I0 * nc + J - 1]; wc[1] = cur[I0 * nc + J]; wr[1] = cur[I0 * nc + J + 1];
                dx[0] = wr[0] - wl[0];
                dx[1] = wr[1] - wl[1];
                auto row = [&](int r, auto Uc, auto Cc, auto Dc) __attribute__((always_inline)) {
                    constexpr int U = decltype(Uc)::value, Cs = decltype(Cc)::value,
                                  D = decltype(Dc)::value;
                    const int I = I0 + r;
                    wl[D] = cur[(I + 1) * nc + J - 1];
                    wc[D] = cur[(I + 1) * nc + J];
                    wr[D] = cur[(I + 1) * nc + J + 1];
                    dx[D] = wr[D] - wl[D];
                    const T* w = tab + 4 * I;
                    const T wd = w[2] - b2J, G = w[3] * fJ;
                    const T c = wc[Cs];
                    T acc = FP32 ? wd * c + (T)lbc[I * nc + J] : wd * c;
                    acc += w[0] * wc[D];
                    acc += w[1] * wc[U];
                    acc += cpJ * wr[Cs];
                    acc += cmJ * wl[Cs];
                    acc += G * (dx[D] - dx[U]);
                    nxt[I * nc + J] = acc;
                };
                using K0 = std::integral_constant<int, 0>;
                using K1 = std::integral_constant<int, 1>;
                using K2 = std::integral_constant<int, 2>;
                int r = 0;
                for (; r + 2 < nr; r += 3) {
                    row(r, K0{}, K1{}, K2{});
                    row(r + 1, K1{}, K2{}, K0{});
                    row(r + 2, K2{}, K0{}, K1{});
                }
                if (r < nr) row(r, K0{}, K1{}, K2{});
                if (r + 1 < nr) row(r + 1, K1{}, K2{}, K0{});
            }
            if (ring_thread) {
                // e^{-r t1} carried as a running product (one multiply per step)
                disc *= dq;
                const double t1 = Tn + (st + 1) * a.dt;
                nxt[rI * nc + rJ] =
                    (T)(ring_value<CHEAP>(a.bc, rI * hc, rJ * hc, t1, disc) - (FP32 ? gT : 0.0));
            }
            __syncthreads();
            T* t = cur; cur = nxt; nxt = t;
        }
        // g_n = Gc(c_n) -> d_n, Gold_n and the next coarse state c_{n+1}
        double* Go = Gold + (long long)n * nn;
        double* dc = dcor + (long long)n * nn;
        if (ring_thread) {
            Go[rI * nc + rJ] = gring(Tn + a.steps * a.dt);
            dc[rI * nc + rJ] = 0.0;
        }
        // Rows are taken EB at a time, every load of a batch issued before the
        // first use (rows clamped into the segment), so that a batch waits for
        // memory once instead of once per row.
        constexpr int EB = 4;
        for (int r0 = 0; r0 < nr; r0 += EB) {
            double cs[EB], go[EB], fu[EB];
#pragma unroll
            for (int e = 0; e < EB; ++e) {
                const int I = I0 + min(r0 + e, nr - 1), off = I * nc + J;
                cs[e] = FP32 ? cst[off] : 0.0;
                go[e] = 0.0;
                fu[e] = 0.0;
                if (!a.init) {
                    go[e] = Go[off];
                    fu[e] = a.foldc[(long long)n * nn + off];
                }
            }
#pragma unroll
            for (int e = 0; e < EB; ++e) {
                if (r0 + e < nr) {
                    const int off = (I0 + r0 + e) * nc + J;
                    const double g = FP32 ? cs[e] + (double)cur[off] : (double)cur[off];
                    if (a.init) {
                        Go[off] = g;
                        dc[off] = 0.0;
                        cst[off] = g;
                    } else {
                        const double d = g - go[e];
                        Go[off] = g;
                        dc[off] = d;
                        cst[off] = fu[e] + d;   // R F(U^k_n) + d_n
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Correction + norm over slices n in [k0, k1):
//   U^{k+1}_{n+1} = F_n + P(d_n)   (numerical G, d_n coarse)   or
//   U^{k+1}_{n+1} = F_n + (g - Gf_n), Gf_n = g   (G on the fine grid, one slice)
// with F_n = U^k_n + delta_n (FP32) or w_n (FP64), and the fused reductions
// red[0] = max |U^{k+1} - U^k| (bit pattern), red[1] = max |U^{k+1}_N|,
// red[2] = non-finite flag.  P is bilinear prolongation.
// ---------------------------------------------------------------------------
struct CorrArgs {
    Grid g;
    int k0, k1, N, nc, q, fp32, fineg;
    int rows;   // interior rows per workgroup
};

__device__ inline void wave_max2(double& a, double& b) {
    for (int o = 32; o > 0; o >>= 1) {
        a = fmax(a, __shfl_xor(a, o));
        b = fmax(b, __shfl_xor(b, o));
    }
}

__global__ __launch_bounds__(kBlock) void k_correct(const double* __restrict__ Ucur,
                                                    const void* __restrict__ Fold,
                                                    const double* __restrict__ dcor,
                                                    const double* __restrict__ gfine,
                                                    double* __restrict__ Gf,
                                                    double* __restrict__ Unext,
                                                    unsigned long long* __restrict__ red,
                                                    CorrArgs a) {
    __shared__ double sm[2][kBlock / kWave];
    __shared__ int sflag;
    if (threadIdx.x == 0) sflag = 0;
    const int nin = a.g.nin;
    const int n = a.k0 + blockIdx.y;
    // a workgroup takes a.rows rows of one slice, so that the per-workgroup
    // reduction (and its global atomics) is paid once per a.rows * nin nodes
    const int r0 = blockIdx.x * a.rows, r1 = min(r0 + a.rows, nin);
    double inc = 0.0, sc = 0.0;
    int bad = 0;
    __syncthreads();
    for (int row = r0; row < r1; ++row) {
        for (int jj = threadIdx.x; jj < nin; jj += kBlock) {   // 0-based interior column
            const int i = row + 1, j = jj + 1;
            const long long o = (long long)row * a.g.pitch + jj;
            const long long on = (long long)n * a.g.stride + o;
            const long long on1 = (long long)(n + 1) * a.g.stride + o;
            const double fo = a.fp32 ? Ucur[on] + (double)((const float*)Fold)[on]
                                     : ((const double*)Fold)[on];
            double corr;
            if (a.fineg) {
                const long long ol = o;   // gfine holds one slice
                const double g = gfine[ol];
                corr = g - Gf[on];
                Gf[on] = g;
            } else {
                const int q = a.q, nc = a.nc;
                const int I = i / q, J = j / q;
                const double al = (double)(i - I * q) / (double)q;
                const double be = (double)(j - J * q) / (double)q;
                const double* d = dcor + (long long)n * nc * nc + I * nc + J;
                corr = (1.0 - al) * (1.0 - be) * d[0] + (1.0 - al) * be * d[1] +
                       al * (1.0 - be) * d[nc] + al * be * d[nc + 1];
            }
            const double v = fo + corr;
            const double old = Ucur[on1];
            Unext[on1] = v;
            const double dv = fabs(v - old);
            if (!(dv <= DBL_MAX)) bad = 1;
            inc = fmax(inc, dv);
            if (n + 1 == a.N) sc = fmax(sc, fabs(v));
        }
    }
    if (bad) sflag = 1;   // benign race: every writer stores 1
    wave_max2(inc, sc);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sm[0][w] = inc; sm[1][w] = sc; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m0 = sm[0][0], m1 = sm[1][0];
        for (int k = 1; k < kBlock / kWave; ++k) { m0 = fmax(m0, sm[0][k]); m1 = fmax(m1, sm[1][k]); }
        if (m0 > 0.0) atomicMax(&red[0], (unsigned long long)__double_as_longlong(m0));
        if (m1 > 0.0) atomicMax(&red[1], (unsigned long long)__double_as_longlong(m1));
        if (sflag) atomicMax(&red[2], 1ull);
    }
}

__global__ void k_zero_red(unsigned long long* red) {
    if (threadIdx.x < 4) red[threadIdx.x] = 0ull;
}

// Interior of slice 0 <- payoff.
__global__ void k_payoff(double* __restrict__ U, Grid g, Bc bc) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (jj >= g.nin) return;
    U[(long long)row * g.pitch + jj] = payoff_at(bc, (row + 1) * bc.h, (jj + 1) * bc.h);
}

// U_{n+1} (interior) <- P(Gold_n) for n in [k0, k1) (initial sweep).
__global__ void k_prolong(const double* __restrict__ Gold, double* __restrict__ U, Grid g, int nc,
                          int q, int k0) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    const int n = k0 + blockIdx.z;
    if (jj >= g.nin) return;
    const int i = row + 1, j = jj + 1;
    const int I = i / q, J = j / q;
    const double al = (double)(i - I * q) / (double)q;
    const double be = (double)(j - J * q) / (double)q;
    const double* c = Gold + (long long)n * nc * nc + I * nc + J;
    U[(long long)(n + 1) * g.stride + (long long)row * g.pitch + jj] =
        (1.0 - al) * (1.0 - be) * c[0] + (1.0 - al) * be * c[1] + al * (1.0 - be) * c[nc] +
        al * be * c[nc + 1];
}

// F(U^k_n) at the coincident nodes of the coarse interior for slices k0..k1-1,
// gathered into a dense nc x nc array per slice (the coarse chain then reads it
// contiguously instead of one strided fine value per node):
//   foldc[n][I][J] = U^k_n + delta_n (FP32 increments) or w_n (FP64) at fine (I q, J q).
__global__ void k_gather_coincident(const double* __restrict__ Ucur, const void* __restrict__ Fold,
                                    double* __restrict__ foldc, Grid g, int nc, int q, int k0,
                                    int fp32) {
    const int J = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int I = 1 + blockIdx.y;
    const int n = k0 + blockIdx.z;
    if (J > nc - 2) return;
    const long long fo = (long long)n * g.stride + (long long)(I * q - 1) * g.pitch + (J * q - 1);
    foldc[(long long)n * nc * nc + I * nc + J] =
        fp32 ? Ucur[fo] + (double)((const float*)Fold)[fo] : ((const double*)Fold)[fo];
}

// Interior layout <- full n x n grid (ring ignored).
__global__ void k_pack(const double* __restrict__ full, double* __restrict__ U, Grid g) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (jj >= g.nin) return;
    U[(long long)row * g.pitch + jj] = full[(long long)(row + 1) * g.n + jj + 1];
}

// Full n x n grid <- interior layout, ring = g(tau).
__global__ void k_unpack(const double* __restrict__ U, double* __restrict__ full, Grid g, Bc bc,
                         double tau) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= g.n) return;
    double v;
    if (i == 0 || i == g.n - 1 || j == 0 || j == g.n - 1)
        v = ring_value(bc, i * bc.h, j * bc.h, tau, exp(-bc.r * tau));
    else
        v = U[(long long)(i - 1) * g.pitch + (j - 1)];
    full[(long long)i * g.n + j] = v;
}

// U_out = U_in + delta (FP32 increments), interior, one slice.
__global__ void k_finalize(const double* __restrict__ Uin, const float* __restrict__ d,
                           double* __restrict__ Uout, Grid g) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (jj >= g.nin) return;
    const long long o = (long long)row * g.pitch + jj;
    Uout[o] = Uin[o] + (double)d[o];
}

// ---------------------------------------------------------------------------
// Host-side launchers (C++ linkage, used by the driver).
// ---------------------------------------------------------------------------
static int step_waves(const StepArgs& a) { return a.count * a.nchunks * a.nstrips; }

static int prep_blocks(const StepArgs& a) { return (step_waves(a) + 3) / 4; }

// Rows in flight per wavefront: 3 measured faster than 6 on the 513^2 x 64
// slice workload (deeper queues cost occupancy).
constexpr int kTbPrefetch = 3;

// Launch geometry of k_fine_tb for S fused steps over a.count slices: strips of
// 64 - 2S output columns; row chunks sized so that a launch has about
// wave_target wavefronts, between min_rows and kTbMaxRows rows (rows_override
// > 0 replaces the rule; every chunk is capped at kTbMaxRows, the rows the
// kernel's LDS weight table holds).  With fit, chunks are then lengthened until
// the launch has at most wave_target wavefronts: at 4 wavefronts per SIMD the
// chip holds 4096 of them, and a launch just above that ends with a short
// second round on a mostly idle chip.
void tb_geometry(StepArgs& a, int S, int wave_target, int min_rows, int rows_override, int fit) {
    const int W = kWave - 2 * S;
    a.nstrips = (a.g.nin + W - 1) / W;
    long long rows = (long long)a.g.nin * a.nstrips * a.count / wave_target;
    rows = std::max<long long>(min_rows, std::min<long long>(kTbMaxRows, rows));
    if (rows_override > 0) rows = std::min(rows_override, kTbMaxRows);
    a.rows = (int)std::min<long long>(rows, a.g.nin);
    a.nchunks = (a.g.nin + a.rows - 1) / a.rows;
    // fit: lengthen the chunks until the launch has at most wave_target wavefronts
    while (fit && rows_override <= 0 && a.rows < std::min(kTbMaxRows, a.g.nin) &&
           (long long)a.count * a.nchunks * a.nstrips > wave_target) {
        a.rows += 1;
        a.nchunks = (a.g.nin + a.rows - 1) / a.rows;
    }
}

template <int MODE, typename T, int S>
static void launch_tb_s(const T* in, const float* lb, T* out, const T* wt, const StepArgs& a,
                        hipStream_t st) {
    const int blocks = (step_waves(a) + 3) / 4;
    if (a.bc.kind == 2)
        hipLaunchKernelGGL((k_fine_tb<MODE, false, T, S, kTbPrefetch>), dim3(blocks), dim3(kBlock),
                           0, st, in, lb, out, wt, a);
    else
        hipLaunchKernelGGL((k_fine_tb<MODE, true, T, S, kTbPrefetch>), dim3(blocks), dim3(kBlock),
                           0, st, in, lb, out, wt, a);
}

template <int MODE, typename T>
static hipError_t launch_tb(const T* in, const float* lb, T* out, const T* wt, const StepArgs& a,
                            int S, hipStream_t st) {
    if (a.rows > kTbMaxRows) return hipErrorInvalidValue;   // beyond the LDS weight table
    switch (S) {
        case 1: launch_tb_s<MODE, T, 1>(in, lb, out, wt, a, st); break;
        case 2: launch_tb_s<MODE, T, 2>(in, lb, out, wt, a, st); break;
        case 3: launch_tb_s<MODE, T, 3>(in, lb, out, wt, a, st); break;
        case 4: launch_tb_s<MODE, T, 4>(in, lb, out, wt, a, st); break;
        case 5: launch_tb_s<MODE, T, 5>(in, lb, out, wt, a, st); break;
        case 6: launch_tb_s<MODE, T, 6>(in, lb, out, wt, a, st); break;
        case 7: launch_tb_s<MODE, T, 7>(in, lb, out, wt, a, st); break;
        case 8: launch_tb_s<MODE, T, 8>(in, lb, out, wt, a, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fine_tb_f32(const float* in, const float* lb, float* out, const float* wt,
                              const StepArgs& a, int S, hipStream_t st) {
    return launch_tb<MODE_INCR, float>(in, lb, out, wt, a, S, st);
}

hipError_t launch_fine_tb_f64(const double* in, double* out, const double* wt, const StepArgs& a,
                              int S, hipStream_t st) {
    return launch_tb<MODE_DIRECT, double>(in, nullptr, out, wt, a, S, st);
}

// Row weights of the temporally blocked step for rows 0..n-1 (see k_fine_tb):
// [wP, wM, cR, gI] = [dt (alpha + mu), dt (alpha - mu), 1 - dt (2 alpha + r),
// dt rho s1 s2 i / 4], evaluated in FP64 and rounded once to T.
template <typename T>
__global__ void k_row_weights(T* __restrict__ wt, int n, Coef c, double dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double A = c.a1 * (double)i * (double)i, Mu = c.hr * (double)i;
    wt[4 * i] = (T)(dt * (A + Mu));
    wt[4 * i + 1] = (T)(dt * (A - Mu));
    wt[4 * i + 2] = (T)(1.0 - dt * (2.0 * A + c.r));
    wt[4 * i + 3] = (T)(dt * c.g12 * (double)i);
}

hipError_t launch_row_weights(void* wt, int n, const Coef& c, double dt, int fp32, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL(k_row_weights<float>, dim3((n + 255) / 256), dim3(256), 0, st,
                           (float*)wt, n, c, dt);
    else
        hipLaunchKernelGGL(k_row_weights<double>, dim3((n + 255) / 256), dim3(256), 0, st,
                           (double*)wt, n, c, dt);
    return hipGetLastError();
}

hipError_t launch_fine_prep(const double* base, float* lb, float* d1, const StepArgs& a,
                            hipStream_t st) {
    if (a.bc.kind == 2)
        hipLaunchKernelGGL(k_fine_prep<false>, dim3(prep_blocks(a)), dim3(kBlock), 0, st, base, lb,
                           d1, a);
    else
        hipLaunchKernelGGL(k_fine_prep<true>, dim3(prep_blocks(a)), dim3(kBlock), 0, st, base, lb,
                           d1, a);
    return hipGetLastError();
}

// the coarse side compiled into the chain kernel (the at-scale coarse grid)
constexpr int kChainNC = 129;
// dynamic LDS one workgroup may take on gfx950
constexpr int kChainLdsMax = 160 * 1024;

hipError_t chain_set_lds(int bytes) {
    const void* fns[10] = {(const void*)k_coarse_chain<true, true, 0, false>,
                           (const void*)k_coarse_chain<true, false, 0, false>,
                           (const void*)k_coarse_chain<false, true, 0, false>,
                           (const void*)k_coarse_chain<false, false, 0, false>,
                           (const void*)k_coarse_chain<true, true, kChainNC, false>,
                           (const void*)k_coarse_chain<true, false, kChainNC, false>,
                           (const void*)k_coarse_chain<true, true, 0, true>,
                           (const void*)k_coarse_chain<true, false, 0, true>,
                           (const void*)k_coarse_chain<false, true, 0, true>,
                           (const void*)k_coarse_chain<false, false, 0, true>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// LDS of the chain kernel: the row table, and the two state buffers when they fit
int chain_lds_bytes(int nc, int fp32) {
    const int es = fp32 ? 4 : 8;
    const int all = (4 * nc + 2 * nc * nc) * es;
    return all <= kChainLdsMax ? all : 4 * nc * es;
}

bool chain_state_in_lds(int nc, int fp32) {
    return (4 * nc + 2 * nc * nc) * (fp32 ? 4 : 8) <= kChainLdsMax;
}

hipError_t launch_chain(const double* Ucur, double* Gold, double* dcor, double* cst, float* lbc,
                        const ChainArgs& a, hipStream_t st) {
    const int lds = chain_lds_bytes(a.nc, a.fp32);
#define PR_CHAIN(C, F, N, G)                                                                \
    hipLaunchKernelGGL((k_coarse_chain<C, F, N, G>), dim3(1), dim3(kChainThreads), lds, st, Ucur, \
                       Gold, dcor, cst, lbc, a)
    if (a.gstate) {
        if (a.bc.kind == 2) {
            if (a.fp32) PR_CHAIN(false, true, 0, true); else PR_CHAIN(false, false, 0, true);
        } else {
            if (a.fp32) PR_CHAIN(true, true, 0, true); else PR_CHAIN(true, false, 0, true);
        }
    } else if (a.bc.kind == 2) {
        if (a.fp32) PR_CHAIN(false, true, 0, false); else PR_CHAIN(false, false, 0, false);
    } else if (a.nc == kChainNC) {
        if (a.fp32) PR_CHAIN(true, true, kChainNC, false); else PR_CHAIN(true, false, kChainNC, false);
    } else {
        if (a.fp32) PR_CHAIN(true, true, 0, false); else PR_CHAIN(true, false, 0, false);
    }
#undef PR_CHAIN
    return hipGetLastError();
}

hipError_t launch_correct(const double* Ucur, const void* Fold, const double* dcor,
                          const double* gfine, double* Gf, double* Unext,
                          unsigned long long* red, const Grid& g, int k0, int k1, int N, int nc,
                          int q, int fp32, int fineg, hipStream_t st) {
    // rows per workgroup: about 2048 workgroups per launch, at least one row
    const long long nodes = (long long)g.nin * g.nin * (k1 - k0);
    const int rows = (int)std::max<long long>(1, std::min<long long>(g.nin, nodes / (2048LL * kBlock * 4)));
    CorrArgs a{g, k0, k1, N, nc, q, fp32, fineg, rows};
    hipLaunchKernelGGL(k_correct, dim3((g.nin + rows - 1) / rows, k1 - k0), dim3(kBlock), 0, st,
                       Ucur, Fold, dcor, gfine, Gf, Unext, red, a);
    return hipGetLastError();
}

hipError_t launch_zero_red(unsigned long long* red, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_red, dim3(1), dim3(64), 0, st, red);
    return hipGetLastError();
}

hipError_t launch_payoff(double* U, const Grid& g, const Bc& bc, hipStream_t st) {
    hipLaunchKernelGGL(k_payoff, dim3((g.nin + 255) / 256, g.nin), dim3(256), 0, st, U, g, bc);
    return hipGetLastError();
}

hipError_t launch_gather_coincident(const double* Ucur, const void* Fold, double* foldc,
                                    const Grid& g, int nc, int q, int k0, int k1, int fp32,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_gather_coincident, dim3((nc - 2 + 255) / 256, nc - 2, k1 - k0), dim3(256),
                       0, st, Ucur, Fold, foldc, g, nc, q, k0, fp32);
    return hipGetLastError();
}

hipError_t launch_prolong(const double* Gold, double* U, const Grid& g, int nc, int q, int k0,
                          int k1, hipStream_t st) {
    hipLaunchKernelGGL(k_prolong, dim3((g.nin + 255) / 256, g.nin, k1 - k0), dim3(256), 0, st,
                       Gold, U, g, nc, q, k0);
    return hipGetLastError();
}

hipError_t launch_pack(const double* full, double* U, const Grid& g, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3((g.nin + 255) / 256, g.nin), dim3(256), 0, st, full, U, g);
    return hipGetLastError();
}

hipError_t launch_unpack(const double* U, double* full, const Grid& g, const Bc& bc, double tau,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_unpack, dim3((g.n + 255) / 256, g.n), dim3(256), 0, st, U, full, g, bc,
                       tau);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* Uin, const float* d, double* Uout, const Grid& g,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3((g.nin + 255) / 256, g.nin), dim3(256), 0, st, Uin, d,
                       Uout, g);
    return hipGetLastError();
}

}  // namespace pr
