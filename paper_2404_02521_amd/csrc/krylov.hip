// krylov.hip -- the implicit-Euler fine propagator of Eq. (fd) (Sec. 3.2) on
// gfx950.  Every step solves
//     (I - dt L_h) u+ = u        at the interior nodes, ring of u+ = g(tau+),
// by BiCGStab with Jacobi preconditioning (the operator is not symmetric, so
// the conjugate-gradient method of Sec. 3.3 does not apply to it), matrix-free:
// the nine-point stencil is the matrix-vector product and its coefficients come
// from the node indices.  All slices of a sweep iterate together: one launch
// covers every active slice, each slice keeps its own scalars and stops on its
// own residual.
//
// One BiCGStab iteration is three kernels; each starts by summing the previous
// kernel's per-workgroup partial dot products of its slice in a fixed order
// (every workgroup of a slice gets bitwise the same scalar, and the result does
// not depend on timing), then does its vector work and writes new partials:
//   KA: rho = (rh, r); beta = (rho / rho_prev) (alpha / omega);
//       p = r + beta (p - omega v); v = A M^-1 p;            partials (rh, v)
//   KB: alpha = rho / (rh, v); s = r - alpha v; t = A M^-1 s; partials (t, s), (t, t)
//   KC: omega = (t, s) / (t, t); x += M^-1 (alpha p + omega s);
//       r = s - omega t;                                       partials (rh, r), (r, r)
// p and v are read at the neighbours while their new values are written, so
// each has two buffers.  A slice is done when the recursively updated (r, r)
// is <= tol^2 (b, b); the host polls the count of finished slices every few
// iterations.  The recursive residual can drift from b - A x after the large
// intermediate residuals BiCGStab sometimes passes through, so every finished
// slice is then checked with its true residual (KCHK, KVER): one that misses
// the tolerance restarts from its current x with r = rh = b - A x (at most
// kMaxRestarts times; it is then reported as not converged).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "device.hpp"
#include "internal.hpp"

namespace pr {

constexpr int kKBlock = 256;
constexpr int kMaxRestarts = 4;

static_assert(kKBlock == 4 * 64, "the workgroup sums below combine four wavefronts");

// Sum of a per-lane value over the wavefront in a fixed pairing (lane l takes
// lane l + o for o = 32, 16, ..., 1): the total is in lane 0.
__device__ inline double wave_sum_fixed(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Workgroup sum of a per-thread value in a fixed order (each wavefront, then
// the four wavefront sums), the same bits in every thread.
__device__ double block_sum_tree(double v, double* sm) {
    v = wave_sum_fixed(v);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sm[0] + sm[1]) + (sm[2] + sm[3]);
    __syncthreads();   // sm is reused by the next sum
    return r;
}

// Sum of `n` partial values (stride `st`) in a fixed order, broadcast to the
// whole workgroup: thread t adds t, t + 256, ...; then block_sum_tree.
__device__ double block_sum_fixed(const double* part, int n, int st, double* sm) {
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += kKBlock) v += part[(long long)k * st];
    return block_sum_tree(v, sm);
}

// Row (i, j) of (I - dt L_h) in index form.
struct KRow {
    double d, xp, xm, yp, ym, gm;   // gm = dt gamma
};
__device__ inline KRow krow(const KrylovArgs& a, int i, int j) {
    const double A = a.c.a1 * (double)i * (double)i, B = a.c.a2 * (double)j * (double)j;
    const double mu = a.c.hr * (double)i, nu = a.c.hr * (double)j;
    KRow w;
    w.d = 1.0 + a.dt * (2.0 * A + 2.0 * B + a.c.r);
    w.xp = -a.dt * (A + mu);
    w.xm = -a.dt * (A - mu);
    w.yp = -a.dt * (B + nu);
    w.ym = -a.dt * (B - nu);
    w.gm = a.dt * a.c.g12 * (double)i * (double)j;
    return w;
}
__device__ inline double kdiag(const KrylovArgs& a, int i, int j) {
    const double A = a.c.a1 * (double)i * (double)i, B = a.c.a2 * (double)j * (double)j;
    return 1.0 + a.dt * (2.0 * A + 2.0 * B + a.c.r);
}

// (A z)_ij for a node function z(i, j) (callers make z zero or g on the ring).
template <class Z>
__device__ inline double apply_row(const KRow& w, int i, int j, Z&& z) {
    double v = w.d * z(i, j);
    v = v + w.xp * z(i + 1, j);
    v = v + w.xm * z(i - 1, j);
    v = v + w.yp * z(i, j + 1);
    v = v + w.ym * z(i, j - 1);
    v = v - w.gm * (z(i + 1, j + 1) + z(i - 1, j - 1) - z(i + 1, j - 1) - z(i - 1, j + 1));
    return v;
}

__device__ inline bool interior(const Grid& g, int i, int j) {
    return i >= 1 && i <= g.n - 2 && j >= 1 && j <= g.n - 2;
}
__device__ inline long long koff(const Grid& g, int i, int j) {
    return (long long)(i - 1) * g.pitch + (j - 1);
}

// Start of a step: b = u - (ring terms of g(tau+)), x0 = u, r = rh = b - A x0,
// p = v = 0, scalar slots 1, partials (rh, r) = (r, r) and (b, b).
__global__ __launch_bounds__(kKBlock) void k_kry_init(const double* __restrict__ X, double* __restrict__ Bv,
                                                     double* __restrict__ R,
                                                     double* __restrict__ RH, double* __restrict__ P0,
                                                     double* __restrict__ V0, double* __restrict__ part,
                                                     KScal* __restrict__ sc, KrylovArgs a) {
#pragma clang fp contract(on)
    __shared__ double sm[kKBlock];
    const int s = blockIdx.y;
    const int n = a.first + s;
    const long long base = (long long)s * a.g.stride;
    const double tau1 = n * a.dT + (a.step + 1) * a.dt;
    const double disc = exp(-a.bc.r * tau1);
    const Grid& g = a.g;
    const int r0 = blockIdx.x * a.rows, r1 = min(r0 + a.rows, g.nin);
    double rr = 0.0, bb = 0.0;
    for (int row = r0; row < r1; ++row) {
        const int i = row + 1;
        for (int j = 1 + threadIdx.x; j <= g.n - 2; j += kKBlock) {
            const KRow w = krow(a, i, j);
            // the state with the new ring (x0 = u inside, g(tau+) on the ring)
            auto xg = [&](int ii, int jj) -> double {
                if (interior(g, ii, jj)) return X[base + koff(g, ii, jj)];
                return ring_value<false>(a.bc, ii * a.bc.h, jj * a.bc.h, tau1, disc);
            };
            auto ring_only = [&](int ii, int jj) -> double {
                if (interior(g, ii, jj)) return 0.0;
                return ring_value<false>(a.bc, ii * a.bc.h, jj * a.bc.h, tau1, disc);
            };
            const long long o = base + koff(g, i, j);
            const double u = X[o];
            const double b = u - apply_row(w, i, j, ring_only);
            const double r = u - apply_row(w, i, j, xg);
            Bv[o] = b;
            R[o] = r;
            RH[o] = r;
            P0[o] = 0.0;
            V0[o] = 0.0;
            rr += r * r;
            bb += b * b;
        }
    }
    const double prr = block_sum_tree(rr, sm);
    const double pbb = block_sum_tree(bb, sm);
    if (threadIdx.x == 0) {
        double* pp = part + ((long long)s * a.nblk + blockIdx.x) * 2;
        pp[0] = prr;
        pp[1] = pbb;
        if (blockIdx.x == 0) {
            KScal& k = sc[s];
            for (int q = 0; q < 2; ++q) { k.rho[q] = 1.0; k.alpha[q] = 1.0; k.omega[q] = 1.0; }
            k.done = 0;
            k.iters = 0;
            k.breakdown = 0;
            k.verified = 0;
            k.restarts = 0;
            k.rr = 0.0;
            k.bb = 0.0;
        }
    }
}

// (b, b) of each slice from the init partials (second value), and slices whose
// initial residual already meets the tolerance.
__global__ void k_kry_start(const double* __restrict__ part, KScal* __restrict__ sc, int* __restrict__ ndone,
                            KrylovArgs a) {
    __shared__ double sm[kKBlock];
    const int s = blockIdx.x;
    const double rr = block_sum_fixed(part + (long long)s * a.nblk * 2, a.nblk, 2, sm);
    const double bb = block_sum_fixed(part + (long long)s * a.nblk * 2 + 1, a.nblk, 2, sm);
    if (threadIdx.x == 0) {
        sc[s].bb = bb;
        if (!(rr > a.tol2 * bb)) {   // also catches b = 0
            sc[s].done = 1;
            sc[s].rr = rr;
            atomicAdd(ndone, 1);
        }
    }
}

// KA: p = r + beta (p - omega v); v = A M^-1 p; partials (rh, v).
__global__ __launch_bounds__(kKBlock) void k_kry_a(const double* __restrict__ R, const double* __restrict__ RH,
                                                  const double* __restrict__ Pin, double* __restrict__ Pout,
                                                  const double* __restrict__ Vin, double* __restrict__ Vout,
                                                  const double* __restrict__ partC, double* __restrict__ partA,
                                                  KScal* __restrict__ sc, int* __restrict__ ndone,
                                                  KrylovArgs a) {
#pragma clang fp contract(on)
    __shared__ double sm[kKBlock];
    const int s = blockIdx.y;
    KScal& k = sc[s];
    if (k.done) return;
    const double* pc = partC + (long long)s * a.nblk * 2;
    const double rho = block_sum_fixed(pc, a.nblk, 2, sm);
    const double rr = block_sum_fixed(pc + 1, a.nblk, 2, sm);
    const int cur = a.it & 1, prev = cur ^ 1;
    if (!(rr > a.tol2 * k.bb) || rho == 0.0) {   // converged (or rh orthogonal to r)
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            k.done = 1;
            k.rr = rr;
            k.iters = a.it;
            k.breakdown = (rr > a.tol2 * k.bb) ? 1 : 0;
            atomicAdd(ndone, 1);
        }
        return;
    }
    const double beta = (rho / k.rho[prev]) * (k.alpha[prev] / k.omega[prev]);
    const double om = k.omega[prev];
    const Grid& g = a.g;
    const long long base = (long long)s * g.stride;
    const int r0 = blockIdx.x * a.rows, r1 = min(r0 + a.rows, g.nin);
    double acc = 0.0;
    for (int row = r0; row < r1; ++row) {
        const int i = row + 1;
        for (int j = 1 + threadIdx.x; j <= g.n - 2; j += kKBlock) {
            // new p at a node, preconditioned (zero on the ring)
            auto zp = [&](int ii, int jj) -> double {
                if (!interior(g, ii, jj)) return 0.0;
                const long long o = base + koff(g, ii, jj);
                const double p = R[o] + beta * (Pin[o] - om * Vin[o]);
                return p / kdiag(a, ii, jj);
            };
            const long long o = base + koff(g, i, j);
            const KRow w = krow(a, i, j);
            const double v = apply_row(w, i, j, zp);
            Pout[o] = R[o] + beta * (Pin[o] - om * Vin[o]);
            Vout[o] = v;
            acc += RH[o] * v;
        }
    }
    const double p = block_sum_tree(acc, sm);
    if (threadIdx.x == 0) {
        partA[(long long)s * a.nblk + blockIdx.x] = p;
        if (blockIdx.x == 0) k.rho[cur] = rho;
    }
}

// KB: alpha = rho / (rh, v); s = r - alpha v; t = A M^-1 s; partials (t, s), (t, t).
__global__ __launch_bounds__(kKBlock) void k_kry_b(const double* __restrict__ R, const double* __restrict__ V,
                                                  double* __restrict__ S, double* __restrict__ T,
                                                  const double* __restrict__ partA, double* __restrict__ partB,
                                                  KScal* __restrict__ sc, int* __restrict__ ndone,
                                                  KrylovArgs a) {
#pragma clang fp contract(on)
    __shared__ double sm[kKBlock];
    const int s = blockIdx.y;
    KScal& k = sc[s];
    if (k.done) return;
    const double sig = block_sum_fixed(partA + (long long)s * a.nblk, a.nblk, 1, sm);
    const int cur = a.it & 1;
    if (sig == 0.0) {   // breakdown: (rh, A M^-1 p) vanished
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            k.done = 1;
            k.iters = a.it;
            k.breakdown = 1;
            atomicAdd(ndone, 1);
        }
        return;
    }
    const double alpha = k.rho[cur] / sig;
    const Grid& g = a.g;
    const long long base = (long long)s * g.stride;
    const int r0 = blockIdx.x * a.rows, r1 = min(r0 + a.rows, g.nin);
    double ts = 0.0, tt = 0.0;
    for (int row = r0; row < r1; ++row) {
        const int i = row + 1;
        for (int j = 1 + threadIdx.x; j <= g.n - 2; j += kKBlock) {
            auto zs = [&](int ii, int jj) -> double {
                if (!interior(g, ii, jj)) return 0.0;
                const long long o = base + koff(g, ii, jj);
                return (R[o] - alpha * V[o]) / kdiag(a, ii, jj);
            };
            const long long o = base + koff(g, i, j);
            const KRow w = krow(a, i, j);
            const double t = apply_row(w, i, j, zs);
            const double sv = R[o] - alpha * V[o];
            S[o] = sv;
            T[o] = t;
            ts += t * sv;
            tt += t * t;
        }
    }
    const double pts = block_sum_tree(ts, sm);
    const double ptt = block_sum_tree(tt, sm);
    if (threadIdx.x == 0) {
        double* pp = partB + ((long long)s * a.nblk + blockIdx.x) * 2;
        pp[0] = pts;
        pp[1] = ptt;
        if (blockIdx.x == 0) k.alpha[cur] = alpha;
    }
}

// KC: omega = (t, s) / (t, t); x += M^-1 (alpha p + omega s); r = s - omega t;
// partials (rh, r), (r, r).
__global__ __launch_bounds__(kKBlock) void k_kry_c(double* __restrict__ X, double* __restrict__ R,
                                                  const double* __restrict__ RH, const double* __restrict__ P,
                                                  const double* __restrict__ S, const double* __restrict__ T,
                                                  const double* __restrict__ partB, double* __restrict__ partC,
                                                  KScal* __restrict__ sc, int* __restrict__ ndone,
                                                  KrylovArgs a) {
#pragma clang fp contract(on)
    __shared__ double sm[kKBlock];
    const int s = blockIdx.y;
    KScal& k = sc[s];
    if (k.done) return;
    const double* pb = partB + (long long)s * a.nblk * 2;
    const double ts = block_sum_fixed(pb, a.nblk, 2, sm);
    const double tt = block_sum_fixed(pb + 1, a.nblk, 2, sm);
    const int cur = a.it & 1;
    const double alpha = k.alpha[cur];
    // t = 0 means s = 0 (A M^-1 is nonsingular): the step ends with x += alpha p
    // and r = 0; omega = 0 with t != 0 is a breakdown (the slice stops after
    // this update)
    const double omega = tt > 0.0 ? ts / tt : 0.0;
    const bool stall = tt > 0.0 && ts == 0.0;
    const Grid& g = a.g;
    const long long base = (long long)s * g.stride;
    const int r0 = blockIdx.x * a.rows, r1 = min(r0 + a.rows, g.nin);
    double rhr = 0.0, rr = 0.0;
    for (int row = r0; row < r1; ++row) {
        const int i = row + 1;
        for (int j = 1 + threadIdx.x; j <= g.n - 2; j += kKBlock) {
            const long long o = base + koff(g, i, j);
            const double sv = S[o];
            const double x = X[o] + (alpha * P[o] + omega * sv) / kdiag(a, i, j);
            const double r = sv - omega * T[o];
            X[o] = x;
            R[o] = r;
            rhr += RH[o] * r;
            rr += r * r;
        }
    }
    const double p1 = block_sum_tree(rhr, sm);
    const double p2 = block_sum_tree(rr, sm);
    if (threadIdx.x == 0) {
        double* pp = partC + ((long long)s * a.nblk + blockIdx.x) * 2;
        pp[0] = p1;
        pp[1] = p2;
        if (blockIdx.x == 0) {
            k.omega[cur] = omega == 0.0 ? 1.0 : omega;   // keeps the next beta finite
            k.iters = a.it + 1;
            if (stall) {
                k.done = 1;
                k.breakdown = 1;
                atomicAdd(ndone, 1);
            }
        }
    }
}

// KCHK: for every slice that finished and has not been checked, the true
// residual r = b - A x (x zero on the ring: b already holds the ring terms)
// into R and RH, p and v of the next iteration cleared (a restart begins with
// p = r), partials (r, r) twice (the (rh, r) and (r, r) slots KA reads).
__global__ __launch_bounds__(kKBlock) void k_kry_check(const double* __restrict__ X,
                                                      const double* __restrict__ Bv,
                                                      double* __restrict__ R, double* __restrict__ RH,
                                                      double* __restrict__ Pz, double* __restrict__ Vz,
                                                      double* __restrict__ partC,
                                                      const KScal* __restrict__ sc, KrylovArgs a) {
#pragma clang fp contract(on)
    __shared__ double sm[kKBlock];
    const int s = blockIdx.y;
    const KScal& k = sc[s];
    if (!k.done || k.verified) return;
    const Grid& g = a.g;
    const long long base = (long long)s * g.stride;
    const int r0 = blockIdx.x * a.rows, r1 = min(r0 + a.rows, g.nin);
    double rr = 0.0;
    for (int row = r0; row < r1; ++row) {
        const int i = row + 1;
        for (int j = 1 + threadIdx.x; j <= g.n - 2; j += kKBlock) {
            auto xz = [&](int ii, int jj) -> double {
                return interior(g, ii, jj) ? X[base + koff(g, ii, jj)] : 0.0;
            };
            const long long o = base + koff(g, i, j);
            const double r = Bv[o] - apply_row(krow(a, i, j), i, j, xz);
            R[o] = r;
            RH[o] = r;
            Pz[o] = 0.0;
            Vz[o] = 0.0;
            rr += r * r;
        }
    }
    const double p = block_sum_tree(rr, sm);
    if (threadIdx.x == 0) {
        double* pp = partC + ((long long)s * a.nblk + blockIdx.x) * 2;
        pp[0] = p;
        pp[1] = p;
    }
}

// KVER: accept a checked slice whose true residual meets the tolerance, else
// restart it (scalars reset, done cleared) or, past kMaxRestarts, keep it
// stopped and flag it as not converged.
__global__ void k_kry_verify(const double* __restrict__ partC, KScal* __restrict__ sc,
                             int* __restrict__ ndone, KrylovArgs a) {
    __shared__ double sm[kKBlock];
    const int s = blockIdx.x;
    KScal& k = sc[s];
    if (!k.done || k.verified) return;
    const double rr = block_sum_fixed(partC + (long long)s * a.nblk * 2 + 1, a.nblk, 2, sm);
    if (threadIdx.x == 0) {
        k.rr = rr;
        if (!(rr > a.tol2 * k.bb)) {
            k.verified = 1;
            k.breakdown = 0;
        } else if (k.restarts < kMaxRestarts) {
            k.restarts += 1;
            k.done = 0;
            k.breakdown = 0;
            for (int q = 0; q < 2; ++q) { k.rho[q] = 1.0; k.alpha[q] = 1.0; k.omega[q] = 1.0; }
            atomicSub(ndone, 1);
        } else {
            k.verified = 1;
            k.breakdown = 1;
        }
    }
}

__global__ void k_kry_zero(int* p) {
    if (threadIdx.x == 0) *p = 0;
}

// End of a step: (r, r) of every slice from the last partials, whether or not
// it met the tolerance.
__global__ void k_kry_final(const double* __restrict__ partC, KScal* __restrict__ sc, KrylovArgs a) {
    __shared__ double sm[kKBlock];
    const int s = blockIdx.x;
    const double rr = block_sum_fixed(partC + (long long)s * a.nblk * 2 + 1, a.nblk, 2, sm);
    if (threadIdx.x == 0) sc[s].rr = rr;
}

// ---------------------------------------------------------------------------
// Host side: one implicit step of every slice of the sweep.
// ---------------------------------------------------------------------------
int krylov_blocks_per_slice(const Grid& g, int count) {
    // about 2048 workgroups per launch, at most one per row
    const int want = std::max(1, 2048 / std::max(1, count));
    return std::min(g.nin, std::max(4, want));
}

hipError_t krylov_step(double* X, const KrylovBufs& b, const KrylovArgs& a0, int max_iters,
                       int poll_every, int* host_done, int* iters_out, hipStream_t st) {
    KrylovArgs a = a0;
    const dim3 grid(a.nblk, a.count), blk(kKBlock);
    hipLaunchKernelGGL(k_kry_zero, dim3(1), dim3(64), 0, st, b.ndone);
    hipLaunchKernelGGL(k_kry_init, grid, blk, 0, st, X, b.B, b.R, b.RH, b.P[0], b.V[0], b.partC,
                       b.sc, a);
    hipLaunchKernelGGL(k_kry_start, dim3(a.count), blk, 0, st, b.partC, b.sc, b.ndone, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // Pipelined polls (b.hpoll set): the finished-slice count is copied to a
    // pinned slot every poll_every iterations and read one round later, while
    // the next round is already queued, so the device never waits for the
    // host.  The iterations queued after the round that finished every slice
    // return at once (finished slices skip their work); they are not counted.
    const bool piped = b.hpoll != nullptr && b.pev[0] != nullptr && b.pev[1] != nullptr;
    int it = 0, nd = 0, idle = 0;
    int pending = -1, pending_it = 0, polls = 0;
    for (;;) {
        for (; it < max_iters; ++it) {
            a.it = it;
            const int cur = it & 1, nxt = cur ^ 1;
            hipLaunchKernelGGL(k_kry_a, grid, blk, 0, st, b.R, b.RH, b.P[cur], b.P[nxt], b.V[cur],
                               b.V[nxt], b.partC, b.partA, b.sc, b.ndone, a);
            hipLaunchKernelGGL(k_kry_b, grid, blk, 0, st, b.R, b.V[nxt], b.S, b.T, b.partA,
                               b.partB, b.sc, b.ndone, a);
            hipLaunchKernelGGL(k_kry_c, grid, blk, 0, st, X, b.R, b.RH, b.P[nxt], b.S, b.T,
                               b.partB, b.partC, b.sc, b.ndone, a);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((it + 1) % poll_every != 0) continue;
            if (!piped) {
                if ((e = hipMemcpyAsync(&nd, b.ndone, sizeof(int), hipMemcpyDeviceToHost, st)) !=
                    hipSuccess)
                    return e;
                if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
                if (nd >= a.count) { ++it; break; }
                continue;
            }
            const int slot = polls & 1;
            hipEvent_t ev = static_cast<hipEvent_t>(b.pev[slot]);
            if ((e = hipMemcpyAsync(b.hpoll + slot, b.ndone, sizeof(int), hipMemcpyDeviceToHost,
                                    st)) != hipSuccess)
                return e;
            if ((e = hipEventRecord(ev, st)) != hipSuccess) return e;
            ++polls;
            if (pending >= 0) {
                if ((e = hipEventSynchronize(static_cast<hipEvent_t>(b.pev[pending]))) != hipSuccess)
                    return e;
                if (b.hpoll[pending] >= a.count) {
                    idle += it + 1 - pending_it;   // the round queued after that poll
                    ++it;
                    break;
                }
            }
            pending = slot;
            pending_it = it + 1;
        }
        pending = -1;
        // true residuals of the finished slices; restarted ones continue
        hipLaunchKernelGGL(k_kry_check, grid, blk, 0, st, X, b.B, b.R, b.RH, b.P[it & 1],
                           b.V[it & 1], b.partC, b.sc, a);
        hipLaunchKernelGGL(k_kry_verify, dim3(a.count), blk, 0, st, b.partC, b.sc, b.ndone, a);
        if ((e = hipMemcpyAsync(&nd, b.ndone, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if (nd >= a.count || it >= max_iters) break;
    }
    hipLaunchKernelGGL(k_kry_final, dim3(a.count), blk, 0, st, b.partC, b.sc, a);
    if ((e = hipMemcpyAsync(&nd, b.ndone, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *host_done = nd;
    *iters_out = it - idle;
    return hipGetLastError();
}

}  // namespace pr
