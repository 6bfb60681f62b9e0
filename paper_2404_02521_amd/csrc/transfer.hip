// transfer.hip -- moving states between a fine grid and the 64 x 64 grid of
// the neural coarse propagator.
//
// The option value is not periodic, so the transfers work on the part that
// vanishes on the ring: w = V - B, where B is the transfinite (Coons) patch of
// the ring values g(tau).  w is expanded in the sine series of its interior
// nodes (DST-I); restriction keeps the first 62 modes per direction and
// evaluates them on the 62 x 62 interior of the 64 x 64 grid, prolongation
// zero-pads the 62 modes back to the fine grid.  Both are separable, so each
// is two FP64 matrix products with host-built (62 x nf) / (nf x 62) matrices
// (Sec. 3.4 runs the operator on its own grid; the transfer to and from the
// fine grid is an addition of this library).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace pr {

constexpr int kFG = 64;        // FNO grid nodes per side
constexpr int kFI = kFG - 2;   // its interior nodes per side (sine modes kept)

// Coons patch of the ring values of an n x n grid with spacing h at (i, j).
template <bool CHEAP>
__device__ inline double coons(const Bc& bc, int n, double h, int i, int j, double tau,
                               double disc) {
    const double e = (n - 1) * h;
    const double xi = (double)i / (n - 1), eta = (double)j / (n - 1);
    const double x = i * h, y = j * h;
    const double gl = ring_value<CHEAP>(bc, 0.0, y, tau, disc);
    const double gr = ring_value<CHEAP>(bc, e, y, tau, disc);
    const double gb = ring_value<CHEAP>(bc, x, 0.0, tau, disc);
    const double gt = ring_value<CHEAP>(bc, x, e, tau, disc);
    const double c00 = ring_value<CHEAP>(bc, 0.0, 0.0, tau, disc);
    const double c10 = ring_value<CHEAP>(bc, e, 0.0, tau, disc);
    const double c01 = ring_value<CHEAP>(bc, 0.0, e, tau, disc);
    const double c11 = ring_value<CHEAP>(bc, e, e, tau, disc);
    return (1 - xi) * gl + xi * gr + (1 - eta) * gb + eta * gt -
           ((1 - xi) * (1 - eta) * c00 + xi * (1 - eta) * c10 + (1 - xi) * eta * c01 +
            xi * eta * c11);
}

// out = in + sign * B(tau) on the fine interior (interior layout; in may equal out).
template <bool CHEAP>
__global__ void k_lift(const double* in, double* out, Grid g, Bc bc, double tau, double sign) {
    const int jj = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (jj >= g.nin) return;
    const long long o = (long long)row * g.pitch + jj;
    const double disc = exp(-bc.r * tau);
    out[o] = in[o] + sign * coons<CHEAP>(bc, g.n, bc.h, row + 1, jj + 1, tau, disc);
}

// Network input plane: interior from the restricted field (62 x 62), ring 0;
// and the model parameters (sigma1, sigma2, rho, r).
__global__ void k_fno_in(const double* __restrict__ wc, float* __restrict__ win,
                         float* __restrict__ meta, Bc bc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 4) meta[t] = (float)(t == 0 ? bc.s1 : t == 1 ? bc.s2 : t == 2 ? bc.rho : bc.r);
    if (t >= kFG * kFG) return;
    const int x = t / kFG, y = t % kFG;
    const bool in = x > 0 && x < kFG - 1 && y > 0 && y < kFG - 1;
    win[t] = in ? (float)wc[(x - 1) * kFI + (y - 1)] : 0.0f;
}

// Coarse state after the slice: wo = base + scale * out on the 62 x 62
// interior (base: w_in, the LOD prediction, or nothing when null).
__global__ void k_fno_out(const double* __restrict__ base, const float* __restrict__ fout,
                          double scale, double* __restrict__ wo) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kFI * kFI) return;
    const int i = t / kFI, j = t % kFI;
    wo[t] = (base ? base[t] : 0.0) + scale * (double)fout[(i + 1) * kFG + (j + 1)];
}

// Training pair on the 64 x 64 grid from two restricted fields:
// [w_in, B1 (+ wb), V_in, V_tgt] = [w0, Bc(tau1) (+ wb), Bc(tau0) + w0, Bc(tau1) + w1]
// (wb: the LOD prediction's w, or null).
template <bool CHEAP>
__global__ void k_pair(const double* __restrict__ w0, const double* __restrict__ w1,
                       const double* __restrict__ wb, float* __restrict__ out, Bc bc,
                       double s_max, double tau0, double tau1) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kFG * kFG) return;
    const int x = t / kFG, y = t % kFG;
    const double h = s_max / (kFG - 1);
    const bool in = x > 0 && x < kFG - 1 && y > 0 && y < kFG - 1;
    const double a = in ? w0[(x - 1) * kFI + (y - 1)] : 0.0;
    const double b = in ? w1[(x - 1) * kFI + (y - 1)] : 0.0;
    const double B0 = coons<CHEAP>(bc, kFG, h, x, y, tau0, exp(-bc.r * tau0));
    const double B1 = coons<CHEAP>(bc, kFG, h, x, y, tau1, exp(-bc.r * tau1));
    out[t] = (float)a;
    out[kFG * kFG + t] = (float)(B1 + (wb && in ? wb[(x - 1) * kFI + (y - 1)] : 0.0));
    out[2 * kFG * kFG + t] = (float)(B0 + a);
    out[3 * kFG * kFG + t] = (float)(B1 + b);
}

hipError_t launch_lift(const double* in, double* out, const Grid& g, const Bc& bc, double tau,
                       double sign, hipStream_t st) {
    dim3 grid((g.nin + 255) / 256, g.nin);
    if (bc.kind == 2)
        hipLaunchKernelGGL(k_lift<false>, grid, dim3(256), 0, st, in, out, g, bc, tau, sign);
    else
        hipLaunchKernelGGL(k_lift<true>, grid, dim3(256), 0, st, in, out, g, bc, tau, sign);
    return hipGetLastError();
}

hipError_t launch_fno_in(const double* wc, float* win, float* meta, const Bc& bc, hipStream_t st) {
    hipLaunchKernelGGL(k_fno_in, dim3(kFG * kFG / 256), dim3(256), 0, st, wc, win, meta, bc);
    return hipGetLastError();
}

hipError_t launch_fno_out(const double* base, const float* fout, double scale, double* wo,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_fno_out, dim3((kFI * kFI + 255) / 256), dim3(256), 0, st, base, fout,
                       scale, wo);
    return hipGetLastError();
}

hipError_t launch_pair(const double* w0, const double* w1, const double* wb, float* out,
                       const Bc& bc, double s_max, double tau0, double tau1, hipStream_t st) {
    if (bc.kind == 2)
        hipLaunchKernelGGL(k_pair<false>, dim3(kFG * kFG / 256), dim3(256), 0, st, w0, w1, wb, out,
                           bc, s_max, tau0, tau1);
    else
        hipLaunchKernelGGL(k_pair<true>, dim3(kFG * kFG / 256), dim3(256), 0, st, w0, w1, wb, out,
                           bc, s_max, tau0, tau1);
    return hipGetLastError();
}

// Host: restriction (62 x nf) and prolongation (nf x 62) matrices.
//   restriction: a_k = 2/(nf+1) sum_i w_i sin(pi k i/(nf+1)), k = 1..62, then
//                wc_m = sum_k a_k sin(pi k m/63), m = 1..62
//   prolongation: b_k = 2/63 sum_m wc_m sin(pi k m/63), then
//                wf_i = sum_k b_k sin(pi k i/(nf+1))
void sine_transfer_matrices(int nf, std::vector<double>& R, std::vector<double>& P) {
    const double pf = M_PI / (nf + 1), pc = M_PI / (kFI + 1);
    std::vector<double> sc((size_t)kFI * kFI);
    for (int k = 1; k <= kFI; ++k)
        for (int m = 1; m <= kFI; ++m) sc[(size_t)(k - 1) * kFI + (m - 1)] = std::sin(pc * k * m);
    R.assign((size_t)kFI * nf, 0.0);
    P.assign((size_t)nf * kFI, 0.0);
    std::vector<double> sf(kFI);
    for (int i = 1; i <= nf; ++i) {
        for (int k = 1; k <= kFI; ++k) sf[k - 1] = std::sin(pf * k * i);
        for (int m = 1; m <= kFI; ++m) {
            double r = 0.0, p = 0.0;
            for (int k = 1; k <= kFI; ++k) {
                const double s = sc[(size_t)(k - 1) * kFI + (m - 1)];
                r += s * sf[k - 1];
                p += sf[k - 1] * s;
            }
            R[(size_t)(m - 1) * nf + (i - 1)] = r * 2.0 / (nf + 1);
            P[(size_t)(i - 1) * kFI + (m - 1)] = p * 2.0 / (kFI + 1);
        }
    }
}

}  // namespace pr
