// device.hpp -- gfx950 device helpers: Dirichlet data, payoff, wavefront shifts.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace pr {

// Payoff at tau = 0 (Sec. 3.2 gives the cash-or-nothing payoff; this solver
// prices the basket call max(w1 S1 + w2 S2 - K, 0) and the exchange option
// max(S1 - S2, 0)).
__device__ __host__ inline double payoff_at(const Bc& b, double x, double y) {
    double v = (b.payoff == 1) ? (x - y) : (b.w1 * x + b.w2 * y - b.K);
    return v > 0.0 ? v : 0.0;
}

__device__ inline double ncdf(double z) { return 0.5 * erfc(-z * 0.70710678118654752440); }

// Exchange option max(S1 - S2, 0): Margrabe's formula (r cancels).
__device__ inline double margrabe_d(double x, double y, double tau, double s1, double s2,
                                    double rho) {
    if (tau <= 0.0) return x > y ? x - y : 0.0;
    if (x <= 0.0) return 0.0;
    if (y <= 0.0) return x;
    double sd = sqrt((s1 * s1 + s2 * s2 - 2.0 * rho * s1 * s2) * tau);
    double d1 = (log(x / y) + 0.5 * sd * sd) / sd;
    return x * ncdf(d1) - y * ncdf(d1 - sd);
}

// One-asset call on S with strike K.
__device__ inline double bs_call_d(double S, double K, double r, double s, double tau) {
    if (tau <= 0.0) return S > K ? S - K : 0.0;
    if (S <= 0.0) return 0.0;
    double sd = s * sqrt(tau);
    double d1 = (log(S / K) + (r + 0.5 * s * s) * tau) / sd;
    return S * ncdf(d1) - K * exp(-r * tau) * ncdf(d1 - sd);
}

// Closed-form ring values (Margrabe / one-asset call), kept out of line so the
// stencil kernels do not carry their registers.
__device__ __noinline__ double ring_exact(const Bc& b, double x, double y, double tau) {
    if (b.payoff == 1) return margrabe_d(x, y, tau, b.s1, b.s2, b.rho);
    return b.w1 * bs_call_d(x, b.K / b.w1, b.r, b.s1, tau);
}

// Dirichlet value g(x, y, tau); disc = exp(-r tau) precomputed by the caller.
// CHEAP = true compiles only the forward-intrinsic and discounted-payoff kinds.
template <bool CHEAP = false>
__device__ inline double ring_value(const Bc& b, double x, double y, double tau, double disc) {
    if (b.kind == 1) return disc * payoff_at(b, x, y);
    if (!CHEAP && b.kind == 2) return ring_exact(b, x, y, tau);
    if (b.payoff == 1) return x > y ? x - y : 0.0;
    double v = b.w1 * x + b.w2 * y - b.K * disc;
    return v > 0.0 ? v : 0.0;
}

// Wavefront shifts through DPP (no LDS traffic): shr1 gives lane l the value
// of lane l-1, shl1 the value of lane l+1.  Lanes whose source is outside the
// wavefront receive 0 (bound_ctrl: the hardware writes zero, so no old value
// has to be materialised and the shift can become a DPP operand of the
// instruction that consumes it); callers patch those lanes.
__device__ inline float shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ inline float shl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ inline double shr1(double v) {
    int2 p = *reinterpret_cast<int2*>(&v);
    p.x = __builtin_amdgcn_update_dpp(0, p.x, 0x138, 0xF, 0xF, true);
    p.y = __builtin_amdgcn_update_dpp(0, p.y, 0x138, 0xF, 0xF, true);
    return *reinterpret_cast<double*>(&p);
}
__device__ inline double shl1(double v) {
    int2 p = *reinterpret_cast<int2*>(&v);
    p.x = __builtin_amdgcn_update_dpp(0, p.x, 0x130, 0xF, 0xF, true);
    p.y = __builtin_amdgcn_update_dpp(0, p.y, 0x130, 0xF, 0xF, true);
    return *reinterpret_cast<double*>(&p);
}

// Broadcast lane `src` (a constant) to the whole wavefront.
__device__ inline float bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double bcast(double v, int src) {
    int2 p = *reinterpret_cast<int2*>(&v);
    p.x = __builtin_amdgcn_readlane(p.x, src);
    p.y = __builtin_amdgcn_readlane(p.y, src);
    return *reinterpret_cast<double*>(&p);
}

// Broadcast lane `src` (uniform across the wavefront, not necessarily a
// compile-time constant) to the whole wavefront.
__device__ inline float bcast_u(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double bcast_u(double v, int src) {
    int2 p = *reinterpret_cast<int2*>(&v);
    p.x = __builtin_amdgcn_readlane(p.x, src);
    p.y = __builtin_amdgcn_readlane(p.y, src);
    return *reinterpret_cast<double*>(&p);
}

// Workgroup-to-XCD-aware remap: the hardware hands consecutive workgroup ids
// to the 8 XCDs in turn; renumber so each XCD sees a contiguous range of
// logical tiles (neighbouring tiles share halo rows in that XCD's L2).
__device__ inline int xcd_remap(int bid, int nblocks) {
    const int nx = 8;
    int per = nblocks / nx;
    int full = per * nx;
    if (bid >= full) return bid;
    return (bid % nx) * per + bid / nx;
}

}  // namespace pr
