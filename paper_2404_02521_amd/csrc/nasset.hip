// nasset.hip -- Parareal for the three-asset Black-Scholes equation on gfx950:
// Eq. (bse_general) of Sec. 3.2 with n = 3, the centred differences of Eq. (fd)
// along every axis and every pair of axes (19 points), explicit Euler, FP64.
// The C ABI is include/parareal3.h.
//
// Storage ("interior layout"): a state holds the (n-2)^3 interior nodes, k (the
// S3 index) contiguous with a row pitch of a multiple of 64 elements, rows of j
// one pitch apart, planes of i one (n-2) * pitch apart; slices follow each
// other.  The faces are never stored: a kernel that reaches one evaluates the
// forward intrinsic value there.
//
// Kernels:
//   k3_step    : one explicit step of every active slice.  A workgroup owns a
//                tile of 16 j-rows x 64 k-columns (256 threads, four rows each) and
//                marches along i over a chunk of planes through a ring of four
//                LDS planes (the tile and its one-node halo): each plane is
//                read from HBM once per tile and serves three output planes;
//                one barrier per plane, the next plane's loads in flight while
//                a plane is computed.
//   k3_restrict: injection of a fine state to the coarse interior.
//   k3_correct : U_{n+1} = F_n + P(g_new - g_old) (trilinear P), or P(g) in
//                the initial sweep, fused with the max-increment reduction.
//   k3_payoff, k3_unpack: the payoff; interior layout -> full n^3 grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "device.hpp"

#include "parareal3.h"

namespace pr3 {

constexpr int kTK = 64;                  // k columns per tile: one wavefront
constexpr int kThreads = 512;            // workgroup of the 512-thread tile shapes: kTK x (TJ / RJ)
constexpr int kSlots = 4;                // LDS ring of planes
constexpr int kCorrBlock = 256;

struct G3 {
    int n, nin, pitch;
    long long plane, stride;   // elements per i-plane and per slice
};

// Index-form coefficients: a_d = s_d^2 / 2 (times k_d^2), g_p = rho_p s_d s_e / 4
// (times k_d k_e) for the pairs (0,1), (0,2), (1,2), hr = r / 2 (times k_d).
struct C3 {
    double a[3], g[3], hr, r;
};

// Forward intrinsic value max(w . S - K e^{-r tau}, 0) on the grid of spacing h.
struct B3 {
    double w[3], K, r, h;
};

__device__ __host__ inline double face_value(const B3& b, int i, int j, int k, double disc) {
    const double v = b.w[0] * ((double)i * b.h) + b.w[1] * ((double)j * b.h) +
                     b.w[2] * ((double)k * b.h) - b.K * disc;
    return v > 0.0 ? v : 0.0;
}

struct Step3 {
    G3 g;
    C3 c;
    B3 b;
    double dt, dT, tq;   // input of slice s at tau = (first + s) dT + tq
    int first;           // absolute index of the launch's slice 0
    int rows;            // i-planes per workgroup
    int ntk;             // k tiles
    int ntiles;          // (j, k) tiles per plane chunk
    int nchunks;         // plane chunks per slice
    int xcd;             // 1: XCD-aware workgroup order
};

// TJ j-rows per tile, RJ rows per thread (rows tj, tj + TJ / RJ, ...).
template <int TJ, int RJ>
__global__ __launch_bounds__(kTK * TJ / RJ) void k3_step(const double* __restrict__ in,
                                                    double* __restrict__ out, Step3 a) {
#pragma clang fp contract(on)
    constexpr int kNT = kTK * TJ / RJ;   // threads of the workgroup
    static_assert(TJ % RJ == 0 && kNT <= 1024, "tile shape and workgroup size disagree");
    constexpr int kTJ = TJ, kRJ = RJ;
    // A tile and its one-node halo: (kTJ + 2) x (kTK + 2) values per plane, at
    // most kPer per thread (element e = threadIdx.x + t * kNT).
    constexpr int kTile = (kTJ + 2) * (kTK + 2);
    constexpr int kPer = (kTile + kNT - 1) / kNT;
    __shared__ double pl[kSlots][kTJ + 2][kTK + 2];
    const G3& g = a.g;
    const int tk = threadIdx.x % kTK, tj = threadIdx.x / kTK;
    // one-dimensional grid, renumbered so that each XCD takes a contiguous run
    // of (tile, plane chunk, slice): neighbouring tiles and chunks then share
    // that XCD's L2, where their halo planes and rows are read again
    const int bid = a.xcd ? pr::xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int tile = bid % a.ntiles, chunk = (bid / a.ntiles) % a.nchunks;
    const int kt = tile % a.ntk, jt = tile / a.ntk;
    const int jb = jt * kTJ, kb = kt * kTK;   // node indices of the tile's halo row / column
    const int s = bid / (a.ntiles * a.nchunks);
    const long long base = (long long)s * g.stride;
    const double tau = (a.first + s) * a.dT + a.tq;
    const double disc = exp(-a.b.r * tau);
    const int i0 = 1 + chunk * a.rows, i1 = min(i0 + a.rows - 1, g.nin);
    // the halo elements this thread loads, mapped once: node (j, k), whether it
    // lies on the grid and whether it is interior in j and k
    int ej[kPer], ek[kPer];
    long long eo[kPer];
    bool eon[kPer], ein[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int e = threadIdx.x + t * kNT;
        ej[t] = jb + e / (kTK + 2);
        ek[t] = kb + e % (kTK + 2);
        eon[t] = e < kTile && ej[t] < g.n && ek[t] < g.n;   // past the grid: never read
        ein[t] = ej[t] >= 1 && ej[t] <= g.nin && ek[t] >= 1 && ek[t] <= g.nin;
        eo[t] = (long long)(ej[t] - 1) * g.pitch + (ek[t] - 1);
    }
    auto fetch = [&](int i, double* r) {   // plane i of the input, node values
        const bool iin = i >= 1 && i <= g.nin;
        const long long po = base + (long long)(i - 1) * g.plane;
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            r[t] = 0.0;
            if (eon[t]) r[t] = (iin && ein[t]) ? in[po + eo[t]] : face_value(a.b, i, ej[t], ek[t], disc);
        }
    };
    auto store = [&](int i, const double* r) {
        double* slot = &pl[i & (kSlots - 1)][0][0];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int e = threadIdx.x + t * kNT;
            if (e < kTile) slot[e] = r[t];
        }
    };
    const int k = kb + 1 + tk;   // this thread's output column and rows
    int j[kRJ];
    bool act[kRJ];
    double kj[kRJ], ay[kRJ], my[kRJ], gyz[kRJ];
    const double kk = k, az = a.c.a[2] * kk * kk, mz = a.c.hr * kk;
#pragma unroll
    for (int q = 0; q < kRJ; ++q) {
        j[q] = jb + 1 + tj + q * (kTJ / kRJ);
        act[q] = j[q] <= g.nin && k <= g.nin;
        kj[q] = j[q];
        ay[q] = a.c.a[1] * kj[q] * kj[q];
        my[q] = a.c.hr * kj[q];
        gyz[q] = a.c.g[2] * kj[q] * kk;
    }
    // Ring of four planes, one barrier per plane: while plane i is computed
    // from planes i-1, i, i+1, plane i+2 goes into the fourth slot (its last
    // reader, plane i-1's computation, ended before this plane's barrier) and
    // the loads of plane i+3 are in flight.
    double nxt[kPer];
    fetch(i0 - 1, nxt);
    store(i0 - 1, nxt);
    fetch(i0, nxt);
    store(i0, nxt);
    fetch(i0 + 1, nxt);
    store(i0 + 1, nxt);
    if (i0 + 1 <= i1) fetch(i0 + 2, nxt);
    for (int i = i0; i <= i1; ++i) {
        __syncthreads();
        const double (*pm)[kTK + 2] = pl[(i - 1) & (kSlots - 1)];
        const double (*pc)[kTK + 2] = pl[i & (kSlots - 1)];
        const double (*pp)[kTK + 2] = pl[(i + 1) & (kSlots - 1)];
        const double ki = i;
        const double ax = a.c.a[0] * ki * ki, mx = a.c.hr * ki;
        const double gxz = a.c.g[1] * ki * kk;
        const int z = tk + 1;
#pragma unroll
        for (int q = 0; q < kRJ; ++q) {
            if (!act[q]) continue;
            const double gxy = a.c.g[0] * ki * kj[q];
            const int y = tj + 1 + q * (kTJ / kRJ);
            const double u = pc[y][z];
            const double xp = pp[y][z], xm = pm[y][z];
            const double yp = pc[y + 1][z], ym = pc[y - 1][z];
            const double zp = pc[y][z + 1], zm = pc[y][z - 1];
            double L = -a.c.r * u;
            L += ax * (xp - 2.0 * u + xm) + mx * (xp - xm);
            L += ay[q] * (yp - 2.0 * u + ym) + my[q] * (yp - ym);
            L += az * (zp - 2.0 * u + zm) + mz * (zp - zm);
            L += gxy * (pp[y + 1][z] + pm[y - 1][z] - pp[y - 1][z] - pm[y + 1][z]);
            L += gxz * (pp[y][z + 1] + pm[y][z - 1] - pp[y][z - 1] - pm[y][z + 1]);
            L += gyz[q] * (pc[y + 1][z + 1] + pc[y - 1][z - 1] - pc[y + 1][z - 1] - pc[y - 1][z + 1]);
            out[base + (long long)(i - 1) * g.plane + (long long)(j[q] - 1) * g.pitch + (k - 1)] =
                u + a.dt * L;
        }
        if (i + 1 <= i1) {   // plane i + 2 is read by plane i + 1's computation
            store(i + 2, nxt);
            if (i + 2 <= i1) fetch(i + 3, nxt);
        }
    }
}

// c(I, J, K) = u(I q, J q, K q) at the coarse interior nodes.
__global__ void k3_restrict(const double* __restrict__ fine, double* __restrict__ coarse, G3 fg,
                            G3 cg, int q) {
    const int K = 1 + blockIdx.x * blockDim.x + threadIdx.x, J = 1 + blockIdx.y,
              I = 1 + blockIdx.z;
    if (K > cg.nin) return;
    coarse[(long long)(I - 1) * cg.plane + (long long)(J - 1) * cg.pitch + (K - 1)] =
        fine[(long long)(I * q - 1) * fg.plane + (long long)(J * q - 1) * fg.pitch + (K * q - 1)];
}

struct Corr3 {
    G3 fg, cg;
    int q;
    int init;     // 1: P(g) with the coarse faces at tau1; 0: F + P(g_new - g_old)
    B3 bc;        // coarse-grid boundary data (init)
    double tau1;  // end of the slice
};

// One thread per fine interior node of one slice.
__global__ __launch_bounds__(kCorrBlock) void k3_correct(const double* __restrict__ F,
                                                         const double* __restrict__ gnew,
                                                         const double* __restrict__ gold,
                                                         const double* __restrict__ Uold,
                                                         double* __restrict__ Unext,
                                                         unsigned long long* __restrict__ red,
                                                         Corr3 a) {
#pragma clang fp contract(on)
    __shared__ double sm[kCorrBlock / 64];
    __shared__ int sflag;
    if (threadIdx.x == 0) sflag = 0;
    __syncthreads();
    const G3& fg = a.fg;
    const G3& cg = a.cg;
    const int k = 1 + blockIdx.x * blockDim.x + threadIdx.x, j = 1 + blockIdx.y, i = 1 + blockIdx.z;
    double inc = 0.0;
    if (k <= fg.nin) {
        const double disc = exp(-a.bc.r * a.tau1);
        auto cval = [&](int I, int J, int K) -> double {
            const bool in = I >= 1 && I <= cg.nin && J >= 1 && J <= cg.nin && K >= 1 && K <= cg.nin;
            if (!in) return a.init ? face_value(a.bc, I, J, K, disc) : 0.0;
            const long long o = (long long)(I - 1) * cg.plane + (long long)(J - 1) * cg.pitch + (K - 1);
            return a.init ? gnew[o] : gnew[o] - gold[o];
        };
        const int q = a.q;
        const int I = i / q, J = j / q, K = k / q;
        const double fi = (double)(i - I * q) / q, fj = (double)(j - J * q) / q,
                     fk = (double)(k - K * q) / q;
        double p = 0.0;
        for (int di = 0; di < 2; ++di) {
            const double wi = di ? fi : 1.0 - fi;
            for (int dj = 0; dj < 2; ++dj) {
                const double wj = dj ? fj : 1.0 - fj;
                for (int dk = 0; dk < 2; ++dk) {
                    const double wk = dk ? fk : 1.0 - fk;
                    const double w = wi * wj * wk;
                    if (w != 0.0) p += w * cval(I + di, J + dj, K + dk);
                }
            }
        }
        const long long o = (long long)(i - 1) * fg.plane + (long long)(j - 1) * fg.pitch + (k - 1);
        const double v = (F ? F[o] : 0.0) + p;
        Unext[o] = v;
        if (Uold) {
            inc = fabs(v - Uold[o]);
            if (!(inc <= DBL_MAX)) sflag = 1;   // benign race: every writer stores 1
        }
    }
    if (!Uold) return;
    for (int off = 32; off > 0; off >>= 1) inc = fmax(inc, __shfl_xor(inc, off));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sm[0];
        for (int w = 1; w < kCorrBlock / 64; ++w) m = fmax(m, sm[w]);
        if (m > 0.0) atomicMax(&red[0], (unsigned long long)__double_as_longlong(m));
        if (sflag) atomicMax(&red[2], 1ull);
    }
}

__global__ void k3_zero_red(unsigned long long* red) {
    if (threadIdx.x < 4) red[threadIdx.x] = 0ull;
}

__global__ void k3_payoff(double* __restrict__ U, G3 g, B3 b) {
    const int k = 1 + blockIdx.x * blockDim.x + threadIdx.x, j = 1 + blockIdx.y, i = 1 + blockIdx.z;
    if (k > g.nin) return;
    U[(long long)(i - 1) * g.plane + (long long)(j - 1) * g.pitch + (k - 1)] =
        face_value(b, i, j, k, 1.0);   // max(w . S - K, 0) is the face formula at tau = 0
}

__global__ void k3_unpack(const double* __restrict__ U, double* __restrict__ out, G3 g, B3 b,
                          double tau) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, i = blockIdx.z;
    if (k >= g.n) return;
    double v;
    if (i == 0 || i == g.n - 1 || j == 0 || j == g.n - 1 || k == 0 || k == g.n - 1)
        v = face_value(b, i, j, k, exp(-b.r * tau));
    else
        v = U[(long long)(i - 1) * g.plane + (long long)(j - 1) * g.pitch + (k - 1)];
    out[((long long)i * g.n + j) * g.n + k] = v;
}

G3 make_g3(int n) {
    G3 g;
    g.n = n;
    g.nin = n - 2;
    g.pitch = (g.nin + 63) / 64 * 64;
    g.plane = (long long)g.nin * g.pitch;
    g.stride = (long long)g.nin * g.plane;
    return g;
}

// Gershgorin bound of explicit Euler: 2 / max over interior rows of
// |diag| + sum |off|, with diag = -(2 sum a_d k_d^2 + r), off-diagonals
// a_d k_d^2 +- hr k_d (two per axis) and +-g_p k_d k_e (four per pair).  Every
// per-axis term 2 a k^2 + |a k^2 + hr k| + |a k^2 - hr k| and every pair term
// grows with its indices, so the maximum is at k_d = n - 2 on every axis.
double stable_dt(const C3& c, int nin) {
    const double k = nin;
    double row = c.r;
    for (int d = 0; d < 3; ++d) {
        const double A = c.a[d] * k * k, M = c.hr * k;
        row += 2.0 * A + std::fabs(A + M) + std::fabs(A - M);
    }
    for (int p = 0; p < 3; ++p) row += 4.0 * std::fabs(c.g[p] * k * k);
    return 2.0 / row;
}

C3 make_c3(const pr3_problem* p) {
    C3 c;
    for (int d = 0; d < 3; ++d) c.a[d] = 0.5 * p->sigma[d] * p->sigma[d];
    const int pd[3] = {0, 0, 1}, pe[3] = {1, 2, 2};
    for (int q = 0; q < 3; ++q) c.g[q] = 0.25 * p->rho[q] * p->sigma[pd[q]] * p->sigma[pe[q]];
    c.hr = 0.5 * p->r;
    c.r = p->r;
    return c;
}

B3 make_b3(const pr3_problem* p, int n) {
    B3 b;
    for (int d = 0; d < 3; ++d) b.w[d] = p->w[d];
    b.K = p->strike;
    b.r = p->r;
    b.h = p->s_max / (n - 1);
    return b;
}

const char* validate(const pr3_problem* p) {
    if (!p) return "null problem";
    if (p->n < 5 || p->n > 513) return "n must be in [5, 513]";
    if (p->coarse_n < 3 || p->coarse_n > p->n) return "coarse_n must be in [3, n]";
    if ((p->n - 1) % (p->coarse_n - 1)) return "(n - 1) must be divisible by (coarse_n - 1)";
    if (p->n_slices < 1 || p->n_slices > PR_MAX_SLICES) return "n_slices out of range";
    if (p->max_iters < 0 || p->fine_steps < 0 || p->coarse_steps < 0) return "negative count";
    if (!(p->s_max > 0) || !(p->T > 0) || !(p->tol >= 0) || !(p->r >= 0)) return "s_max, T, tol, r";
    if (!(p->cfl >= 0 && p->cfl <= 1)) return "cfl must be in [0, 1]";
    for (int d = 0; d < 3; ++d) {
        if (!(p->sigma[d] > 0) || !std::isfinite(p->sigma[d])) return "sigma must be > 0";
        if (!(std::fabs(p->rho[d]) < 1)) return "|rho| must be < 1";
        if (!std::isfinite(p->w[d])) return "w must be finite";
    }
    if (!std::isfinite(p->strike)) return "strike must be finite";
    const double a = p->rho[0], b = p->rho[1], c = p->rho[2];
    if (1.0 - a * a - b * b - c * c + 2.0 * a * b * c < 0.0)
        return "the correlation matrix is not positive semi-definite";
    return nullptr;
}

int steps_for(double dT, double cfl, double dt_stab) {
    return std::max(1, (int)std::ceil(dT / (cfl * dt_stab) - 1e-12));
}

uint64_t al(uint64_t b) { return (b + 255) / 256 * 256; }

struct Layout {
    uint64_t Ua, Ub, Wa, Wb, ca, cb, cr, gold, red, total;
};

Layout layout(const pr3_problem* p) {
    const G3 fg = make_g3(p->n), cg = make_g3(p->coarse_n);
    const uint64_t N = p->n_slices, fs = (uint64_t)fg.stride * 8, cs = (uint64_t)cg.stride * 8;
    Layout L{};
    uint64_t o = 0;
    auto take = [&](uint64_t b) { const uint64_t r = o; o += al(b); return r; };
    L.Ua = take((N + 1) * fs);
    L.Ub = take((N + 1) * fs);
    L.Wa = take(N * fs);
    L.Wb = take(N * fs);
    L.ca = take(cs);
    L.cb = take(cs);
    L.cr = take(cs);
    L.gold = take(N * cs);
    L.red = take(64);
    L.total = o;
    return L;
}

}  // namespace pr3

using namespace pr3;

struct pr3_solver {
    pr3_problem p{};
    G3 fg{}, cg{};
    C3 c{};
    B3 bf{}, bc{};
    int N = 0, mF = 0, mG = 0, q = 1, maxit = 0;
    double dT = 0, dtF = 0, dtG = 0;
    char* ws = nullptr;
    Layout L{};
    hipStream_t st = nullptr;
    hipEvent_t ev[4]{};
    bool events = false;
    int tile_rows = 16;   // j-rows per step tile: 8, 16 or 32 (PR3_TILE_ROWS)
    int xcd = 1;          // XCD-aware workgroup order of the step kernel (PR3_XCD; 0: off)
    bool half_wg = true;  // 8- and 16-row tiles on 256 threads, twice the rows per thread
                          // (PR3_HALF_WG=0: on 512 threads)
    std::string err;
    template <class T> T* at(uint64_t off) { return reinterpret_cast<T*>(ws + off); }
};

namespace {

#define P3CHK(expr)                                                        \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) {                                            \
            s->err = std::string(#expr) + ": " + hipGetErrorString(e_);    \
            return PR_EDEVICE;                                             \
        }                                                                  \
    } while (0)

int step_rows(const G3& g, int tiles, int count) {
    // about 2048 workgroups per launch, 4 .. 64 planes each
    const long long want = (long long)g.nin * tiles * count / 2048;
    return (int)std::max(4LL, std::min<long long>(64, want));
}

// m explicit steps of dt over `count` slices (absolute first slice `first`)
// from `in` (slice pointers at in + s * stride) into ping-pong buffers A/B;
// returns the buffer holding the result.  in may equal neither A nor B.
pr_status sweep(pr3_solver* s, const G3& g, const C3& c, const B3& b, const double* in, double* A,
                double* B, int first, int count, int m, double dt, const double** res,
                int64_t* psteps) {
    Step3 a{};
    a.g = g;
    a.c = c;
    a.b = b;
    a.dt = dt;
    a.dT = s->dT;
    a.first = first;
    a.ntk = (g.nin + kTK - 1) / kTK;
    const int TJ = s->tile_rows;
    const int ntj = (g.nin + TJ - 1) / TJ;
    a.rows = step_rows(g, a.ntk * ntj, count);
    a.ntiles = a.ntk * ntj;
    a.nchunks = (g.nin + a.rows - 1) / a.rows;
    a.xcd = s->xcd;
    const dim3 grid(a.ntiles * a.nchunks * count);
    const double* src = in;
    double* dst = A;
    for (int q = 0; q < m; ++q) {
        a.tq = q * dt;
        if (TJ == 32)
            hipLaunchKernelGGL((k3_step<32, 4>), grid, dim3(kThreads), 0, s->st, src, dst, a);
        else if (TJ == 8 && s->half_wg)
            hipLaunchKernelGGL((k3_step<8, 2>), grid, dim3(kThreads / 2), 0, s->st, src, dst, a);
        else if (TJ == 8)
            hipLaunchKernelGGL((k3_step<8, 1>), grid, dim3(kThreads), 0, s->st, src, dst, a);
        else if (s->half_wg)
            hipLaunchKernelGGL((k3_step<16, 4>), grid, dim3(kThreads / 2), 0, s->st, src, dst, a);
        else
            hipLaunchKernelGGL((k3_step<16, 2>), grid, dim3(kThreads), 0, s->st, src, dst, a);
        P3CHK(hipGetLastError());
        src = dst;
        dst = (dst == A) ? B : A;
    }
    *res = src;
    if (psteps) *psteps += (int64_t)m * count * g.nin * g.nin * g.nin;
    return PR_OK;
}

// G over slice n from the fine state Us: restrict, m_G coarse steps; returns the
// coarse result (interior layout).
pr_status coarse_g(pr3_solver* s, const double* Us, int n, const double** gres) {
    const G3& fg = s->fg;
    const G3& cg = s->cg;
    double* cr = s->at<double>(s->L.cr);
    hipLaunchKernelGGL(k3_restrict, dim3((cg.nin + 63) / 64, cg.nin, cg.nin), dim3(64), 0, s->st,
                       Us, cr, fg, cg, s->q);
    P3CHK(hipGetLastError());
    return sweep(s, cg, s->c, s->bc, cr, s->at<double>(s->L.ca), s->at<double>(s->L.cb), n, 1, s->mG,
                 s->dtG, gres, nullptr);
}

pr_status correct(pr3_solver* s, int init, const double* F, const double* gnew, const double* gold,
                  const double* Uold, double* Unext, int n) {
    Corr3 a{};
    a.fg = s->fg;
    a.cg = s->cg;
    a.q = s->q;
    a.init = init;
    a.bc = s->bc;
    a.tau1 = (n + 1) * s->dT;
    const G3& g = s->fg;
    hipLaunchKernelGGL(k3_correct, dim3((g.nin + kCorrBlock - 1) / kCorrBlock, g.nin, g.nin),
                       dim3(kCorrBlock), 0, s->st, F, gnew, gold, Uold, Unext,
                       s->at<unsigned long long>(s->L.red), a);
    P3CHK(hipGetLastError());
    return PR_OK;
}

pr_status payoff(pr3_solver* s, double* U) {
    const G3& g = s->fg;
    hipLaunchKernelGGL(k3_payoff, dim3((g.nin + 63) / 64, g.nin, g.nin), dim3(64), 0, s->st, U, g,
                       s->bf);
    P3CHK(hipGetLastError());
    return PR_OK;
}

pr_status unpack(pr3_solver* s, const double* U, double* out, double tau) {
    const G3& g = s->fg;
    hipLaunchKernelGGL(k3_unpack, dim3((g.n + 63) / 64, g.n, g.n), dim3(64), 0, s->st, U, out, g,
                       s->bf, tau);
    P3CHK(hipGetLastError());
    return PR_OK;
}

double ms_between(pr3_solver* s, int a, int b) {
    float ms = 0.f;
    if (!s->events || hipEventElapsedTime(&ms, s->ev[a], s->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0;
    }
    return ms;
}

#define P3RUN(expr)                       \
    do {                                  \
        pr_status r_ = (expr);            \
        if (r_ != PR_OK) return r_;       \
    } while (0)

pr_status do_solve(pr3_solver* s, double* v_out, pr3_stats* st) {
    const G3& g = s->fg;
    const int N = s->N;
    const long long fs = g.stride, cs = s->cg.stride;
    double* Ucur = s->at<double>(s->L.Ua);
    double* Unext = s->at<double>(s->L.Ub);
    double* gold = s->at<double>(s->L.gold);
    double* Wa = s->at<double>(s->L.Wa);
    double* Wb = s->at<double>(s->L.Wb);
    unsigned long long* red = s->at<unsigned long long>(s->L.red);
    double t_fine = 0, t_coarse = 0, inc = 0;
    int64_t psteps = 0;
    // initial coarse sweep: U_0 = payoff, U_{n+1} = G(U_n), g_old_n = G_c(R U_n)
    if (s->events) P3CHK(hipEventRecord(s->ev[2], s->st));
    P3RUN(payoff(s, Ucur));
    for (int n = 0; n < N; ++n) {
        const double* gr = nullptr;
        P3RUN(coarse_g(s, Ucur + n * fs, n, &gr));
        P3RUN(correct(s, 1, nullptr, gr, nullptr, nullptr, Ucur + (n + 1) * fs, n));
        P3CHK(hipMemcpyAsync(gold + n * cs, gr, cs * 8, hipMemcpyDeviceToDevice, s->st));
    }
    P3CHK(hipMemcpyAsync(Unext, Ucur, fs * 8, hipMemcpyDeviceToDevice, s->st));
    if (s->events) P3CHK(hipEventRecord(s->ev[3], s->st));
    P3CHK(hipStreamSynchronize(s->st));
    t_coarse += ms_between(s, 2, 3);
    int K = 0;
    pr_status status = PR_OK;
    for (int k = 0; k < s->maxit && k < N; ++k) {
        // F over the active slices k..N-1, all in each launch
        if (s->events) P3CHK(hipEventRecord(s->ev[0], s->st));
        const double* R = nullptr;
        P3RUN(sweep(s, g, s->c, s->bf, Ucur + k * fs, Wa + k * fs, Wb + k * fs, k, N - k, s->mF,
                    s->dtF, &R, &psteps));
        R -= k * fs;
        if (s->events) P3CHK(hipEventRecord(s->ev[1], s->st));
        // G chain and correction, slice by slice
        hipLaunchKernelGGL(k3_zero_red, dim3(1), dim3(64), 0, s->st, red);
        P3CHK(hipGetLastError());
        P3CHK(hipMemcpyAsync(Unext + k * fs, Ucur + k * fs, fs * 8, hipMemcpyDeviceToDevice, s->st));
        for (int n = k; n < N; ++n) {
            const double* gr = nullptr;
            P3RUN(coarse_g(s, Unext + n * fs, n, &gr));
            P3RUN(correct(s, 0, R + n * fs, gr, gold + n * cs, Ucur + (n + 1) * fs,
                          Unext + (n + 1) * fs, n));
            P3CHK(hipMemcpyAsync(gold + n * cs, gr, cs * 8, hipMemcpyDeviceToDevice, s->st));
        }
        if (s->events) P3CHK(hipEventRecord(s->ev[2], s->st));
        unsigned long long h[3];
        P3CHK(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s->st));
        P3CHK(hipStreamSynchronize(s->st));
        t_fine += ms_between(s, 0, 1);
        t_coarse += ms_between(s, 1, 2);
        std::memcpy(&inc, &h[0], 8);
        std::swap(Ucur, Unext);
        K = k + 1;
        if (st && k <= PR_MAX_SLICES) st->increments[k] = inc;
        if (h[2]) {
            s->err = "non-finite value in the Parareal iteration";
            status = PR_ENONFINITE;
            break;
        }
        if (inc < s->p.tol || K == N) break;
        if (K == s->maxit) {
            s->err = "max_iters reached above tol";
            status = PR_ENOTCONV;
        }
    }
    if (v_out) P3RUN(unpack(s, Ucur + N * fs, v_out, N * s->dT));
    P3CHK(hipStreamSynchronize(s->st));
    if (st) {
        st->iters = K;
        st->last_increment = inc;
        st->t_fine_ms = t_fine;
        st->t_coarse_ms = t_coarse;
        st->fine_point_steps = psteps;
    }
    return status;
}

}  // namespace

extern "C" {

pr_status pr3_plan(const pr3_problem* p, int32_t* fine_steps, int32_t* coarse_steps) {
    if (validate(p)) return PR_EINVAL;
    const double cfl = p->cfl > 0 ? p->cfl : 0.9;
    const double dT = p->T / p->n_slices;
    const C3 c = make_c3(p);
    const double sf = stable_dt(c, p->n - 2), sc = stable_dt(c, p->coarse_n - 2);
    const int mf = p->fine_steps > 0 ? p->fine_steps : steps_for(dT, cfl, sf);
    const int mg = p->coarse_steps > 0 ? p->coarse_steps : steps_for(dT, cfl, sc);
    if (dT / mf > sf * (1 + 1e-12) || dT / mg > sc * (1 + 1e-12)) return PR_EUNSTABLE;
    if (fine_steps) *fine_steps = mf;
    if (coarse_steps) *coarse_steps = mg;
    return PR_OK;
}

uint64_t pr3_workspace_bytes(const pr3_problem* p) {
    if (validate(p)) return 0;
    return layout(p).total;
}

pr_status pr3_create(const pr3_problem* p, void* workspace, uint64_t workspace_bytes,
                     void* hip_stream, pr3_solver** out) {
    if (!out) return PR_EINVAL;
    *out = nullptr;
    int32_t mf = 0, mg = 0;
    const pr_status ps = pr3_plan(p, &mf, &mg);
    if (ps != PR_OK) return ps;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256) return PR_EINVAL;
    const Layout L = layout(p);
    if (workspace_bytes < L.total) return PR_ENOMEM;
    pr3_solver* s = new (std::nothrow) pr3_solver();
    if (!s) return PR_ENOMEM;
    s->p = *p;
    s->fg = make_g3(p->n);
    s->cg = make_g3(p->coarse_n);
    s->c = make_c3(p);
    s->bf = make_b3(p, p->n);
    s->bc = make_b3(p, p->coarse_n);
    s->N = p->n_slices;
    s->mF = mf;
    s->mG = mg;
    s->q = (p->n - 1) / (p->coarse_n - 1);
    s->maxit = p->max_iters > 0 ? std::min(p->max_iters, p->n_slices) : p->n_slices;
    s->dT = p->T / p->n_slices;
    s->dtF = s->dT / mf;
    s->dtG = s->dT / mg;
    s->ws = reinterpret_cast<char*>(workspace);
    s->L = L;
    s->st = reinterpret_cast<hipStream_t>(hip_stream);
    if (const char* e = std::getenv("PR3_TILE_ROWS")) {
        const int t = std::atoi(e);
        s->tile_rows = (t == 8 || t == 32) ? t : 16;
    }
    if (const char* e = std::getenv("PR3_XCD")) s->xcd = std::atoi(e) != 0;
    if (const char* e = std::getenv("PR3_HALF_WG")) s->half_wg = std::atoi(e) != 0;
    bool ok = true;
    for (auto& e : s->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    s->events = ok;
    *out = s;
    return PR_OK;
}

pr_status pr3_solve(pr3_solver* s, double* v_out, pr3_stats* st) {
    if (!s || !v_out) return PR_EINVAL;
    if (st) std::memset(st, 0, sizeof(*st));
    const auto t0 = std::chrono::steady_clock::now();
    const pr_status r = do_solve(s, v_out, st);
    if (st) {
        st->fine_steps = s->mF;
        st->coarse_steps = s->mG;
        st->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return r;
}

pr_status pr3_serial_fine(pr3_solver* s, double* v_out, pr3_stats* st) {
    if (!s || !v_out) return PR_EINVAL;
    if (st) std::memset(st, 0, sizeof(*st));
    const auto t0 = std::chrono::steady_clock::now();
    const G3& g = s->fg;
    const long long fs = g.stride;
    double* U = s->at<double>(s->L.Ua);
    double* Wa = s->at<double>(s->L.Wa);
    double* Wb = s->at<double>(s->L.Wb);
    int64_t psteps = 0;
    P3RUN(payoff(s, U));
    if (s->events) P3CHK(hipEventRecord(s->ev[0], s->st));
    for (int n = 0; n < s->N; ++n) {
        const double* R = nullptr;
        P3RUN(sweep(s, g, s->c, s->bf, U + n * fs, Wa, Wb, n, 1, s->mF, s->dtF, &R, &psteps));
        P3CHK(hipMemcpyAsync(U + (n + 1) * fs, R, fs * 8, hipMemcpyDeviceToDevice, s->st));
    }
    if (s->events) P3CHK(hipEventRecord(s->ev[1], s->st));
    P3RUN(unpack(s, U + s->N * fs, v_out, s->N * s->dT));
    P3CHK(hipStreamSynchronize(s->st));
    if (st) {
        st->iters = 0;
        st->fine_steps = s->mF;
        st->coarse_steps = s->mG;
        st->t_fine_ms = ms_between(s, 0, 1);
        st->fine_point_steps = psteps;
        st->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return PR_OK;
}

pr_status pr3_fine_sweep_probe(pr3_solver* s, double* ms, int64_t* point_steps) {
    if (!s || !ms || !point_steps) return PR_EINVAL;
    const G3& g = s->fg;
    const long long fs = g.stride;
    double* U = s->at<double>(s->L.Ua);
    P3RUN(payoff(s, U));
    for (int n = 1; n < s->N; ++n)
        P3CHK(hipMemcpyAsync(U + n * fs, U, fs * 8, hipMemcpyDeviceToDevice, s->st));
    int64_t psteps = 0;
    const double* R = nullptr;
    if (s->events) P3CHK(hipEventRecord(s->ev[0], s->st));
    P3RUN(sweep(s, g, s->c, s->bf, U, s->at<double>(s->L.Wa), s->at<double>(s->L.Wb), 0, s->N,
                s->mF, s->dtF, &R, &psteps));
    if (s->events) P3CHK(hipEventRecord(s->ev[1], s->st));
    P3CHK(hipStreamSynchronize(s->st));
    *ms = ms_between(s, 0, 1);
    *point_steps = psteps;
    return PR_OK;
}

pr_status pr3_destroy(pr3_solver* s) {
    if (!s) return PR_EINVAL;
    for (auto& e : s->ev)
        if (e) (void)hipEventDestroy(e);
    delete s;
    return PR_OK;
}

const char* pr3_last_error(const pr3_solver* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
