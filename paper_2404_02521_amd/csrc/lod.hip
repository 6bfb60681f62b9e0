// lod.hip -- same-grid coarse propagator on gfx950: locally one-dimensional
// implicit Euler.  Sec. 3.2's coarse propagator is implicit Euler on the fine
// grid with a coarser time step; here each implicit step is split by
// direction:
//   (I - dt Ly)(I - dt Lx) u+ = u + dt Lxy u,   u+ = g(tau1) on the ring,
//   Lx = alpha D_xx + mu D_x - r/2,  Ly = beta D_yy + nu D_y - r/2,  Lxy = gamma D_xy,
// with the x-stage end rows (I - dt Ly) g(tau1).
//
// The coarse chain runs one slice at a time, so a step must use the whole
// chip on a single grid: every tridiagonal line system is solved by one
// workgroup with parallel cyclic reduction in LDS (log2 of the line length
// steps), all lines of a direction at once.
//   k_lod_x : one workgroup per interior column; builds u + dt Lxy u and the
//             column-line system, solves it (reads of a column hit L2);
//   k_lod_x2: the same for two adjacent columns per workgroup (lines of 256 to
//             512 unknowns), the columns both read staged in LDS row by row;
//   k_lod_y : one workgroup per interior row; row loads and stores are
//             contiguous.
// The stages run in FP64: in FP32 the rounding of G(U^{k+1}) - G(U^k) sets a
// floor near 1.5e-6 relative under the Parareal increments.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "device.hpp"
#include "internal.hpp"

namespace pr {

constexpr int kPcrThreads = 1024;
constexpr int kPcrMaxPerThread = 2;   // lines up to 2048 unknowns
constexpr int kPcrTail = 8;           // unknowns per system left to elimination
constexpr int kPcrStop = 64;          // stop reduction only when >= 64 systems remain

struct LodArgs {
    Grid g;
    Coef c;
    Bc bc;
    double dt;
    double tau0;   // time of the step's input (its ring)
    double tau1;   // time of the step's output
    int npad;      // power of two >= nin
};

// Parallel cyclic reduction of a_k x_{k-1} + x_k + c_k x_{k+1} = d_k on
// k < npad, every row normalised to a unit diagonal (rows >= n are identity
// rows; a_0 = c_{n-1} = 0 after folding the end values into d).  A reduction
// step with stride s eliminates x_{k-s} and x_{k+s} from row k with rows
// k - s and k + s and divides the result by its new diagonal, so that each
// row costs one division per step.  The arrays ping-pong between the two LDS
// sets (one barrier per step).  The reduction stops at stride kPcrStop: the
// rows then form kPcrStop independent systems k0, k0 + kPcrStop, ... of
// npad / kPcrStop unknowns each, which threads k0 < kPcrStop solve by
// elimination and back substitution.  Returns the set that holds x_k = d_k.
// Threads tid = 0 .. nt-1 work on the system (several groups of a workgroup may
// each solve their own system of the same npad); every thread of the workgroup
// takes the same number of barriers.
struct PcrSet {
    double* a;
    double* c;
    double* d;
};
__device__ inline PcrSet pcr_solve(PcrSet in, PcrSet out, int npad, int tid, int nt) {
    const int stop = npad >= kPcrStop * kPcrTail ? npad / kPcrTail : npad;
    for (int s = 1; s < stop; s <<= 1) {
#pragma unroll
        for (int e = 0; e < kPcrMaxPerThread; ++e) {
            const int k = tid + e * nt;
            if (k < npad) {
                const int km = k - s, kp = k + s;
                const double ak = in.a[k], ck = in.c[k];
                const double am = km >= 0 ? in.a[km] : 0.0, cm = km >= 0 ? in.c[km] : 0.0;
                const double dm = km >= 0 ? in.d[km] : 0.0;
                const double ap = kp < npad ? in.a[kp] : 0.0, cp = kp < npad ? in.c[kp] : 0.0;
                const double dp = kp < npad ? in.d[kp] : 0.0;
                const double inv = 1.0 / (1.0 - ak * cm - ck * ap);
                out.a[k] = -ak * am * inv;
                out.c[k] = -ck * cp * inv;
                out.d[k] = (in.d[k] - ak * dm - ck * dp) * inv;
            }
        }
        __syncthreads();
        const PcrSet t = in;
        in = out;
        out = t;
    }
    if (stop < npad && tid < stop) {
        // rows tid + q * stop, q = 0 .. m-1: a couples to q - 1, c to q + 1
        const int m = npad / stop;
        double cprime[kPcrTail], dprime[kPcrTail];
        double cp = 0.0, dp = 0.0;
#pragma unroll
        for (int q = 0; q < kPcrTail; ++q) {
            const int k = tid + q * stop;
            if (q < m) {
                const double ak = in.a[k];
                const double inv = 1.0 / (1.0 - ak * cp);
                cp = in.c[k] * inv;
                dp = (in.d[k] - ak * dp) * inv;
                cprime[q] = cp;
                dprime[q] = dp;
            }
        }
        double x = 0.0;
#pragma unroll
        for (int q = kPcrTail - 1; q >= 0; --q) {
            if (q < m) {
                x = dprime[q] - cprime[q] * x;
                in.d[tid + q * stop] = x;
            }
        }
    }
    __syncthreads();
    return in;
}

// (I - dt Lx) w = u + dt Lxy u along interior column j = blockIdx.x + 1.
// in / w: interior layout, FP64; the ring of u is g(tau0).
template <bool CHEAP>
__global__ __launch_bounds__(kPcrThreads) void k_lod_x(const double* __restrict__ in,
                                                       double* __restrict__ w, LodArgs a) {
    extern __shared__ double sm[];
    const int npad = a.npad;
    const PcrSet s0{sm, sm + npad, sm + 2 * npad}, s1{sm + 3 * npad, sm + 4 * npad, sm + 5 * npad};
    const int M = a.g.n, n = a.g.nin, P = a.g.pitch;
    const int j = blockIdx.x + 1;
    const double h = a.bc.h, dt = a.dt;
    const double disc0 = exp(-a.bc.r * a.tau0), disc1 = exp(-a.bc.r * a.tau1);
    auto u_at = [&](int i, int jq) -> double {
        if (i == 0 || i == M - 1 || jq == 0 || jq == M - 1)
            return ring_value<CHEAP>(a.bc, i * h, jq * h, a.tau0, disc0);
        return in[(long long)(i - 1) * P + (jq - 1)];
    };
    auto endrow = [&](int i) {   // (I - dt Ly) g(tau1) at ring row i, column j
        const double gm = ring_value<CHEAP>(a.bc, i * h, (j - 1) * h, a.tau1, disc1);
        const double g0 = ring_value<CHEAP>(a.bc, i * h, j * h, a.tau1, disc1);
        const double gp = ring_value<CHEAP>(a.bc, i * h, (j + 1) * h, a.tau1, disc1);
        const double be = a.c.a2 * j * j, nu = a.c.hr * j;
        return g0 - dt * (be * (gp - 2.0 * g0 + gm) + nu * (gp - gm) - 0.5 * a.c.r * g0);
    };
    for (int k = threadIdx.x; k < npad; k += blockDim.x) {
        if (k < n) {
            const int i = k + 1;
            const double al = a.c.a1 * i * i, mu = a.c.hr * i;
            double ak = -dt * (al - mu), ck = -dt * (al + mu);
            double dk = u_at(i, j) + dt * a.c.g12 * i * j *
                                         (u_at(i + 1, j + 1) + u_at(i - 1, j - 1) -
                                          u_at(i + 1, j - 1) - u_at(i - 1, j + 1));
            if (k == 0) { dk -= ak * endrow(0); ak = 0.0; }
            if (k == n - 1) { dk -= ck * endrow(M - 1); ck = 0.0; }
            const double ib = 1.0 / (1.0 + dt * (2.0 * al + 0.5 * a.c.r));
            s0.a[k] = ak * ib; s0.c[k] = ck * ib; s0.d[k] = dk * ib;
        } else {
            s0.a[k] = 0.0; s0.c[k] = 0.0; s0.d[k] = 0.0;
        }
    }
    __syncthreads();
    const PcrSet x = pcr_solve(s0, s1, npad, threadIdx.x, blockDim.x);
    for (int k = threadIdx.x; k < n; k += blockDim.x) w[(long long)k * P + (j - 1)] = x.d[k];
}

// The x stage for lines of at most kLodX2MaxPad unknowns: two adjacent interior
// columns j0 = 2 blockIdx.x + 1 and j0 + 1 per workgroup of 2 npad threads.
// Columns j0 - 1 .. j0 + 2 of every row (what both line systems read, with the
// mixed term) are staged in LDS by consecutive threads, four values of a row at
// a time, instead of one column value per thread; each half of the workgroup
// then builds and solves its column's system exactly as k_lod_x does (same
// values, same operations), and the two results leave through LDS as row pairs.
constexpr int kLodX2MaxPad = 512;
template <bool CHEAP>
__global__ __launch_bounds__(kPcrThreads) void k_lod_x2(const double* __restrict__ in,
                                                        double* __restrict__ w, LodArgs a) {
    extern __shared__ double sm[];
    const int npad = a.npad;
    const int half = threadIdx.x / npad;          // which of the two columns
    const int tl = threadIdx.x - half * npad;     // thread index within its half
    double* const sb = sm + half * 6 * npad;
    const PcrSet s0{sb, sb + npad, sb + 2 * npad}, s1{sb + 3 * npad, sb + 4 * npad, sb + 5 * npad};
    double* const tile = sm + 12 * npad;          // [row][4]: columns j0 - 1 .. j0 + 2
    const int M = a.g.n, n = a.g.nin, P = a.g.pitch;
    const int j0 = 2 * blockIdx.x + 1;
    const int j = j0 + half;
    const double h = a.bc.h, dt = a.dt;
    const double disc0 = exp(-a.bc.r * a.tau0), disc1 = exp(-a.bc.r * a.tau1);
    for (int e = threadIdx.x; e < M * 4; e += blockDim.x) {
        const int i = e >> 2, jq = j0 - 1 + (e & 3);
        double v = 0.0;   // a column past the grid: never read
        if (jq <= M - 1) {
            if (i == 0 || i == M - 1 || jq == 0 || jq == M - 1)
                v = ring_value<CHEAP>(a.bc, i * h, jq * h, a.tau0, disc0);
            else
                v = in[(long long)(i - 1) * P + (jq - 1)];
        }
        tile[e] = v;
    }
    __syncthreads();
    auto u_at = [&](int i, int jq) -> double { return tile[i * 4 + (jq - j0 + 1)]; };
    auto endrow = [&](int i) {   // (I - dt Ly) g(tau1) at ring row i, column j
        const double gm = ring_value<CHEAP>(a.bc, i * h, (j - 1) * h, a.tau1, disc1);
        const double g0 = ring_value<CHEAP>(a.bc, i * h, j * h, a.tau1, disc1);
        const double gp = ring_value<CHEAP>(a.bc, i * h, (j + 1) * h, a.tau1, disc1);
        const double be = a.c.a2 * j * j, nu = a.c.hr * j;
        return g0 - dt * (be * (gp - 2.0 * g0 + gm) + nu * (gp - gm) - 0.5 * a.c.r * g0);
    };
    {
        const int k = tl;
        if (k < n && j <= n) {
            const int i = k + 1;
            const double al = a.c.a1 * i * i, mu = a.c.hr * i;
            double ak = -dt * (al - mu), ck = -dt * (al + mu);
            double dk = u_at(i, j) + dt * a.c.g12 * i * j *
                                         (u_at(i + 1, j + 1) + u_at(i - 1, j - 1) -
                                          u_at(i + 1, j - 1) - u_at(i - 1, j + 1));
            if (k == 0) { dk -= ak * endrow(0); ak = 0.0; }
            if (k == n - 1) { dk -= ck * endrow(M - 1); ck = 0.0; }
            const double ib = 1.0 / (1.0 + dt * (2.0 * al + 0.5 * a.c.r));
            s0.a[k] = ak * ib; s0.c[k] = ck * ib; s0.d[k] = dk * ib;
        } else {
            s0.a[k] = 0.0; s0.c[k] = 0.0; s0.d[k] = 0.0;
        }
    }
    __syncthreads();
    const PcrSet x = pcr_solve(s0, s1, npad, tl, npad);
    // the tile is free again (pcr_solve ends with a barrier): results as row pairs
    if (tl < n) tile[2 * tl + half] = x.d[tl];
    __syncthreads();
    const int ncol = min(2, n - j0 + 1);
    for (int e = threadIdx.x; e < 2 * n; e += blockDim.x) {
        const int k = e >> 1, c = e & 1;
        if (c < ncol) w[(long long)k * P + (j0 - 1 + c)] = tile[e];
    }
}

// (I - dt Ly) u+ = w along interior row i = blockIdx.x + 1; ends g(i, 0, tau1)
// and g(i, M-1, tau1).
template <bool CHEAP>
__global__ __launch_bounds__(kPcrThreads) void k_lod_y(const double* __restrict__ w,
                                                       double* __restrict__ out, LodArgs a) {
    extern __shared__ double sm[];
    const int npad = a.npad;
    const PcrSet s0{sm, sm + npad, sm + 2 * npad}, s1{sm + 3 * npad, sm + 4 * npad, sm + 5 * npad};
    const int M = a.g.n, n = a.g.nin, P = a.g.pitch;
    const int i = blockIdx.x + 1;
    const double h = a.bc.h, dt = a.dt;
    const double disc1 = exp(-a.bc.r * a.tau1);
    const double* row = w + (long long)(i - 1) * P;
    for (int k = threadIdx.x; k < npad; k += blockDim.x) {
        if (k < n) {
            const int j = k + 1;
            const double be = a.c.a2 * j * j, nu = a.c.hr * j;
            double ak = -dt * (be - nu), ck = -dt * (be + nu);
            double dk = row[k];
            if (k == 0) {
                dk -= ak * ring_value<CHEAP>(a.bc, i * h, 0.0, a.tau1, disc1);
                ak = 0.0;
            }
            if (k == n - 1) {
                dk -= ck * ring_value<CHEAP>(a.bc, i * h, (M - 1) * h, a.tau1, disc1);
                ck = 0.0;
            }
            const double ib = 1.0 / (1.0 + dt * (2.0 * be + 0.5 * a.c.r));
            s0.a[k] = ak * ib; s0.c[k] = ck * ib; s0.d[k] = dk * ib;
        } else {
            s0.a[k] = 0.0; s0.c[k] = 0.0; s0.d[k] = 0.0;
        }
    }
    __syncthreads();
    const PcrSet x = pcr_solve(s0, s1, npad, threadIdx.x, blockDim.x);
    double* orow = out + (long long)(i - 1) * P;
    for (int k = threadIdx.x; k < n; k += blockDim.x) orow[k] = x.d[k];
}

int lod_npad(int nin) {
    int p = 1;
    while (p < nin) p <<= 1;
    return p;
}

// two sets of three npad-long FP64 arrays (a, c, d)
int lod_lds_bytes(int nin) { return 6 * lod_npad(nin) * (int)sizeof(double); }

// k_lod_x2: those sets for both columns, and the four staged columns of every row
int lod_x2_lds_bytes(int nin) {
    return (12 * lod_npad(nin) + 4 * (nin + 2)) * (int)sizeof(double);
}

// k_lod_x2 takes the x stage of lines of 256 (PR_LOD_X2_MIN) to kLodX2MaxPad
// (padded) unknowns
bool lod_use_x2(int nin) {
    static const int lo = std::getenv("PR_LOD_X2_MIN") ? std::atoi(std::getenv("PR_LOD_X2_MIN")) : 256;
    const int npad = lod_npad(nin);
    return npad >= lo && npad <= kLodX2MaxPad;
}

// The kernels' dynamic-LDS limit, set to what the longest supported line needs
// (2048 unknowns; kLodX2MaxPad for k_lod_x2), so that solvers of different grid
// sizes in one process never lower each other's limit.  The argument is the
// line length of the solver at hand, checked against that bound.
hipError_t lod_set_lds(int nin) {
    if (lod_npad(nin) > kPcrThreads * kPcrMaxPerThread) return hipErrorInvalidValue;
    const int bytes = lod_lds_bytes(kPcrThreads * kPcrMaxPerThread);
    const void* fns[4] = {(const void*)k_lod_x<true>, (const void*)k_lod_x<false>,
                          (const void*)k_lod_y<true>, (const void*)k_lod_y<false>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    const int b2 = lod_x2_lds_bytes(kLodX2MaxPad);
    for (const void* f : {(const void*)k_lod_x2<true>, (const void*)k_lod_x2<false>}) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b2);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// G over slice n: m LOD steps of dt from tau0 on the FP64 state `in`
// (interior layout), result in `out`; work0 / work1 / wbuf are slice-sized
// FP64 scratch arrays.
hipError_t launch_lod_slice(const double* in, double* out, double* work0, double* work1,
                            double* wbuf, const Grid& g, const Coef& c, const Bc& bc, double dt,
                            double tau0, int m, hipStream_t st) {
    const int npad = lod_npad(g.nin);
    const int threads = npad < kPcrThreads ? npad : kPcrThreads;
    const int lds = lod_lds_bytes(g.nin);
    const bool x2 = lod_use_x2(g.nin);
    const int lds2 = lod_x2_lds_bytes(g.nin);
    const dim3 gx2((g.nin + 1) / 2), bx2(2 * npad);
    const double* cur = in;
    for (int q = 0; q < m; ++q) {
        LodArgs a{g, c, bc, dt, tau0 + q * dt, tau0 + (q + 1) * dt, npad};
        double* dst = (q == m - 1) ? out : ((q & 1) ? work1 : work0);
        if (bc.kind == 2) {
            if (x2)
                hipLaunchKernelGGL(k_lod_x2<false>, gx2, bx2, lds2, st, cur, wbuf, a);
            else
                hipLaunchKernelGGL(k_lod_x<false>, dim3(g.nin), dim3(threads), lds, st, cur, wbuf, a);
            hipLaunchKernelGGL(k_lod_y<false>, dim3(g.nin), dim3(threads), lds, st, wbuf, dst, a);
        } else {
            if (x2)
                hipLaunchKernelGGL(k_lod_x2<true>, gx2, bx2, lds2, st, cur, wbuf, a);
            else
                hipLaunchKernelGGL(k_lod_x<true>, dim3(g.nin), dim3(threads), lds, st, cur, wbuf, a);
            hipLaunchKernelGGL(k_lod_y<true>, dim3(g.nin), dim3(threads), lds, st, wbuf, dst, a);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur = dst;
    }
    return hipSuccess;
}

}  // namespace pr
