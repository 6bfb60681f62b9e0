// device.hpp -- gfx950 device helpers: Dirichlet data, payoff, wavefront shifts.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace pr {

// Payoff at tau = 0: the basket call max(w1 S1 + w2 S2 - K, 0), the exchange
// option max(S1 - S2, 0), or the paper's two-asset cash-or-nothing option
// (Sec. 3.2): the cash amount c if S1 >= K1 and S2 >= K2, else 0.
__device__ __host__ inline double payoff_at(const Bc& b, double x, double y) {
    if (b.payoff == 2) return (x >= b.K && y >= b.K2) ? b.cash : 0.0;
    double v = (b.payoff == 1) ? (x - y) : (b.w1 * x + b.w2 * y - b.K);
    return v > 0.0 ? v : 0.0;
}

// 20-point Gauss-Legendre rule on [-1, 1], computed at compile time: Newton's
// iteration on P_20 from the usual initial guesses cos(pi (i + 3/4) / 20.5),
// weights 2 / ((1 - x^2) P_20'(x)^2).
struct GaussLegendre20 {
    double x[20], w[20];
};
constexpr double cx_cos(double t) {   // |t| <= pi: Taylor series
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 30; ++k) {
        term *= -t * t / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
constexpr GaussLegendre20 make_gauss_legendre20() {
    GaussLegendre20 r{};
    const int n = 20;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double x = cx_cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (dx < 1e-17 && dx > -1e-17) break;
        }
        r.x[i] = x;
        r.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return r;
}
constexpr GaussLegendre20 kGL20 = make_gauss_legendre20();

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

// Bivariate standard normal CDF P(X <= h, Y <= k) for correlation |rho| <=
// 0.925, from Plackett's identity d/drho B = phi_2(h, k; rho): with rho = sin t,
//   B(h, k; rho) = Phi(h) Phi(k) + 1/(2 pi) int_0^{asin rho}
//                  exp(-(h^2 - 2 h k sin t + k^2) / (2 cos^2 t)) dt,
// the integral by the 20-point Gauss-Legendre rule (the integrand is smooth on
// the whole interval for |rho| <= 0.925).
template <int I = 0>
__device__ inline double plackett_sum(double h, double k, double half) {
    if constexpr (I < 20) {
        const double t = half * (1.0 + kGL20.x[I]);
        const double sn = sin(t), c2 = 1.0 - sn * sn;
        return kGL20.w[I] * exp(-(h * h - 2.0 * h * k * sn + k * k) / (2.0 * c2)) +
               plackett_sum<I + 1>(h, k, half);
    } else {
        return 0.0;
    }
}
__device__ inline double bvn_lower(double h, double k, double rho) {
    if (h == -INFINITY || k == -INFINITY) return 0.0;
    if (h == INFINITY) return ncdf(k);
    if (k == INFINITY) return ncdf(h);
    const double base = ncdf(h) * ncdf(k);
    if (rho == 0.0) return base;
    const double half = 0.5 * asin(rho);
    return base + half * plackett_sum(h, k, half) * 0.15915494309189533577;   // 1/(2 pi)
}

// The paper's closed form, Eq. (solution): c e^{-r tau} B(d1, d2; rho) with
// d_i = (ln(S_i / K_i) + (r - sigma_i^2 / 2) tau) / (sigma_i sqrt(tau)).
__device__ inline double cash_or_nothing_d(const Bc& b, double x, double y, double tau) {
    if (tau <= 0.0) return payoff_at(b, x, y);
    if (x <= 0.0 || y <= 0.0) return 0.0;
    const double st = sqrt(tau);
    const double d1 = (log(x / b.K) + (b.r - 0.5 * b.s1 * b.s1) * tau) / (b.s1 * st);
    const double d2 = (log(y / b.K2) + (b.r - 0.5 * b.s2 * b.s2) * tau) / (b.s2 * st);
    return b.cash * exp(-b.r * tau) * bvn_lower(d1, d2, b.rho);
}

// Closed-form ring values (Margrabe / one-asset call / cash-or-nothing), kept
// out of line so the stencil kernels do not carry their registers.
__device__ __noinline__ double ring_exact(const Bc& b, double x, double y, double tau) {
    if (b.payoff == 2) return cash_or_nothing_d(b, x, y, tau);
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
