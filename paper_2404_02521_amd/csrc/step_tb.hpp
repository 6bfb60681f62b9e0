// step_tb.hpp -- device body of the temporally blocked explicit Euler step
// (S steps of Eq. (fd) per launch), shared by the per-solver kernel and the
// ragged multi-request kernel.  Included by HIP sources only.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace pr {

enum { MODE_DIRECT = 0, MODE_INCR = 1 };
enum { P_GEN = 0, P_MID = 1, P_FAST = 2 };   // row paths of the temporally blocked kernel

// f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>), unrolled.
template <int N, int I = 0, class Fn>
__device__ __attribute__((always_inline)) inline void static_for(Fn&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// ---------------------------------------------------------------------------
// Temporally blocked fine steps: S explicit steps of the same operator per
// launch, the intermediate time levels kept in registers.
//
// A wavefront owns 64 consecutive columns jl = j0 - S + lane and walks rows
// top to bottom.  Level 0 is the input state; level q (1..S) is the state
// after q steps.  When level-0 row x arrives, level q computes its row x - q
// from the three newest rows of level q-1, so one pass over the rows advances
// every level.  DPP shifts supply the j +- 1 neighbours; lane 0 / lane 63 have
// no outer neighbour, so level q is valid on lanes [q, 63-q] and the output
// columns are the middle W = 64 - 2S lanes.  Row chunks overlap by S rows on
// each side for the same reason.  Each input element is read once and each
// output element written once per S steps.  The Dirichlet ring of every level
// is evaluated in place at that level's time.
// MODE_INCR: FP32 increments d over an FP64 base (d+ = d + dt (Lb + L d), with
// dt Lb stored); MODE_DIRECT: FP64 state (u+ = u + dt L u).
//
// The update is applied as neighbour weights with dt folded in:
//   u+ = [dt Lb] + (cR_i - b2_j) u + wP_i u_{i+1} + wM_i u_{i-1} + wR_j u_{j+1}
//        + wL_j u_{j-1} + gI_i j (mixed four-corner difference),
// cR = 1 - dt (2 alpha_i + r), wP/wM = dt (alpha_i +- mu_i), gI = dt rho s1 s2 i / 4
// per row (from this wavefront's LDS copy of the table `wt`), b2 = 2 dt beta_j,
// wR/wL = dt (beta_j +- nu_j) per column (registers).  The j +- 1 terms are
// summed on the neighbour's lane (vr = wR_{j-1} u + gI (j-1) (u_{i+1} - u_{i-1})
// and vl likewise) and enter as the DPP operands of the last two additions,
// so a point-step is ten vector operations plus the per-row products.  Every
// row path evaluates the same expressions in the same order.
// ---------------------------------------------------------------------------
// Longest row chunk of the temporally blocked kernel and the rows of its
// per-wavefront weight table (chunk + 3 S + 1 for S <= 8).
constexpr int kTbMaxRows = 128;
constexpr int kTbWRows = kTbMaxRows + 3 * 8 + 1;

template <int MODE, bool CHEAP, typename T, int S, int PF>
__device__ __attribute__((always_inline)) inline void tb_body(const T* __restrict__ in,
                                                              const float* __restrict__ lb,
                                                              T* __restrict__ out,
                                                              const T* __restrict__ wt,
                                                              const StepArgs& a, const int wid) {
    // multiply-adds are fused only within a statement, so every instance (S,
    // row path) evaluates a point-step with the same roundings: the result does
    // not depend on the launch geometry
#pragma clang fp contract(on)
    constexpr int W = kWave - 2 * S;
    static_assert(S < 32, "ring lanes: columns 0 and M-1 use lanes 0..S and 32..32+S");
    const int lane = threadIdx.x & 63;
    const int strip = wid % a.nstrips;
    const int t = wid / a.nstrips;
    const int chunk = t % a.nchunks;
    const int s = t / a.nchunks;
    if (s >= a.count) return;

    const int M = a.g.n;
    const int P = a.g.pitch;
    const int n = a.first + s;
    const double Tn = n * a.dT;
    const double disc_T = exp(-a.bc.r * Tn);
    const int j0 = 1 + strip * W;
    const int jl = j0 - S + lane;
    const bool in_col = (jl >= 1) && (jl <= M - 2);
    const bool out_lane = (lane >= S) && (lane < S + W) && in_col;
    // ring columns (0 and M-1) that fall inside this wavefront's 64 columns
    const bool rc_left = j0 - S <= 0, rc_right = j0 - S + kWave - 1 >= M - 1;
    const int n_rc = (rc_left ? 1 : 0) + (rc_right ? 1 : 0);
    const int jring = rc_right ? M - 1 : 0;   // the ring column when n_rc == 1
    const int ia = 1 + chunk * a.rows;
    const int ib = min(ia + a.rows, M - 1);
    const T* src = in + (long long)s * a.g.stride;
    const float* lbs = lb + (long long)s * a.g.stride;
    T* dst = out + (long long)s * a.g.stride;
    const int x0 = max(0, ia - S);
    const int x1 = ib - 1 + S;   // last iteration (level S row ib-1)

    // Row weights of rows x0 - S .. x1 - 1 (every row a level evaluates; rows
    // outside the grid take a clamped row, whose result is never used) copied
    // once into this wavefront's slice of LDS: a level then reads its row's
    // four weights with one LDS load at an immediate offset.
    using W4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;
    __shared__ W4 wlds[kBlock / kWave][kTbWRows];
    W4* wrow = wlds[threadIdx.x >> 6];
    const int nrow = x1 - x0 + S;
    for (int e = lane; e < nrow; e += kWave) {
        const int rr = min(max(x0 - S + e, 0), M - 1);
        wrow[e] = *reinterpret_cast<const W4*>(wt + 4 * rr);
    }
    // Row iterations of the unrolled paths: x in [S+1, M-2] for wavefronts
    // with at most one ring column (P_MID also evaluates rows up to x + 2 <=
    // M - 2).
    const bool interior = n_rc <= 1;
    const int fb = interior ? max(x0, S + 1) : x1 + 1;
    const int fe = interior ? min(x1, M - 2) : x1;

    // P_MID: the ring column's values for every iteration x in [fb, fe] and
    // level q (0..S: row x - q at level q's time), in this wavefront's slice
    // of LDS at entry (x - x0) (S + 1) + q, evaluated once by all lanes.
    constexpr int RS = S + 1;
    __shared__ T rtab[kBlock / kWave][kTbWRows * RS];
    T* rring = rtab[threadIdx.x >> 6];
    if (n_rc == 1 && fb <= fe) {
        const double yr = jring * a.bc.h;
        const int nv = (fe - fb + 1) * RS;
        for (int e = lane; e < nv; e += kWave) {
            const int x = fb + e / RS, q = e % RS;
            const double tq = Tn + (a.step + q) * a.dt;
            const double xr = (x - q) * a.bc.h;
            double v = ring_value<CHEAP>(a.bc, xr, yr, tq, exp(-a.bc.r * tq));
            if (MODE == MODE_INCR) v -= ring_value<CHEAP>(a.bc, xr, yr, Tn, disc_T);
            rring[(x - x0) * RS + q] = (T)v;
        }
    }
    // the LDS writes of this wavefront complete before its reads below
    __builtin_amdgcn_s_waitcnt(0xC07F);

    // ring value at node (i, jl), level q; only the ring rows use it, so the
    // level's time and discount are formed on the spot
    auto ring = [&](int i, int q) __attribute__((always_inline)) -> T {
        const double x = i * a.bc.h, y = jl * a.bc.h;
        const double tq = Tn + (a.step + q) * a.dt;
        double v = ring_value<CHEAP>(a.bc, x, y, tq, exp(-a.bc.r * tq));
        if (MODE == MODE_INCR) v -= ring_value<CHEAP>(a.bc, x, y, Tn, disc_T);
        return (T)v;
    };
    // Ring columns inside interior rows.  When the newest level-0 row is x,
    // level q needs the ring value at row x - q.  One pass over the lanes
    // evaluates them for three consecutive newest rows x + k (k = 0..2), both
    // ring columns c and every level q: lane RS (2k + c) + q holds column c
    // (0: column 0, 1: column M-1), level q, row x + k - q; P_GEN evaluates
    // them per row and its levels pick up the lanes with k = 0 by readlane.
    // The values are the same expressions as ring(x + k - q, q).
    static_assert(6 * RS <= kWave, "ring lanes: 3 rows x 2 columns x (S + 1) levels");
    const int bl = min(lane, 6 * RS - 1);
    const int bq = bl % RS;
    const int boff = bl / (2 * RS) - bq;   // row offset k - q
    const bool bcol = (bl / RS) & 1;
    const double btau = Tn + (a.step + bq) * a.dt;
    const double bdisc = exp(-a.bc.r * btau);
    auto ring_batch = [&](int x) __attribute__((always_inline)) -> T {
        const double xx = (x + boff) * a.bc.h, yy = (bcol ? M - 1 : 0) * a.bc.h;
        double v = ring_value<CHEAP>(a.bc, xx, yy, btau, bdisc);
        if (MODE == MODE_INCR) v -= ring_value<CHEAP>(a.bc, xx, yy, Tn, disc_T);
        return (T)v;
    };
    const bool ring_lane = jl == jring;   // P_MID: this lane is the ring column

    // column weights (FP64, then rounded once).  The j +- 1 terms are formed
    // on the neighbour's lane and shifted once: lane k holds the weights of
    // columns k - 1 (the right-hand term of that column) and k + 1 (its
    // left-hand term), so wR_j u_{j+1} = shl1(wRs u)_j and wL_j u_{j-1} =
    // shr1(wLs u)_j, and likewise the mixed term with (j -+ 1) in place of j.
    auto colw = [&](int jj, double sgn) -> T {
        const double B = a.c.a2 * (double)jj * (double)jj, N = a.c.hr * (double)jj;
        return (T)(a.dt * (B + sgn * N));
    };
    const T wRs = colw(jl - 1, 1.0), wLs = colw(jl + 1, -1.0);
    const T b2 = (T)(2.0 * a.dt * (a.c.a2 * (double)jl * (double)jl));
    const T fjm = (T)(jl - 1), fjp = (T)(jl + 1);

    // Window of level q (0..S-1): three rows in slots 0..2; with the row loop
    // unrolled by 3 the newest row of iteration x sits in slot x % 3, so
    // rotating the window costs no moves.  Only the lane's own column is
    // kept: the j +- 1 neighbours come from DPP shifts when a level is
    // evaluated (the mixed term needs only the shifts of u_{i+1} - u_{i-1}).
    T wc[S][3];
    float lbw[S];   // Lb rows x-1 .. x-S (lbw[q-1] -> row x-q)
#pragma unroll
    for (int q = 0; q < S; ++q) {
        lbw[q] = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) wc[q][k] = T(0);
    }

    // Prefetch queue: raw loads of rows x..x+PF-1 and Lb rows x-1..x+PF-2 in
    // flight (PF a multiple of 3; row x in slot x % PF).
    // Loads are unconditional, with row and column clamped into the interior,
    // so no branch surrounds them.  A clamped value is never used as data:
    // level 0 masks rows and columns outside the interior when it takes the
    // row in, and Lb only enters rows and lanes whose result is replaced by
    // ring values or zero, or that feed no output lane.
    const int jc = min(max(jl, 1), M - 2) - 1;
    auto raw = [&](int x) -> T { return src[(long long)(min(max(x, 1), M - 2) - 1) * P + jc]; };
    auto rawlb = [&](int rl) -> float {
        if (MODE != MODE_INCR) return 0.f;
        return lbs[(long long)(min(max(rl, 1), M - 2) - 1) * P + jc];
    };
    static_assert(PF % 3 == 0, "prefetch depth must be a multiple of the window");
    T pq[PF];
    float lq[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int xr = x0 + ((k - x0 % PF) + PF) % PF;   // the row in [x0, x0+PF) with xr % PF == k
        pq[k] = raw(xr);
        lq[k] = rawlb(xr - 1);
    }

    // One row iteration; the newest window slot is x % 3 = K and the prefetch
    // slot x % PF = KP (both compile time).  PATH (compile time):
    //  P_FAST: every row touched (x-S .. x) is interior and no lane is on the
    //          ring, so no boundary logic is compiled in;
    //  P_MID : rows as for P_FAST, one ring column in the wavefront; its values
    //          come from the wavefront's LDS table (one broadcast read each);
    //  P_GEN : anything (ring rows, rows outside the grid, both ring columns).
    auto iter = [&](auto KPc, auto Pc, int x) __attribute__((always_inline)) {
        constexpr int KP = decltype(KPc)::value;
        constexpr int K = KP % 3;
        constexpr int PATH = decltype(Pc)::value;
        constexpr int K1 = (K + 2) % 3;   // previous row
        constexpr int K2 = (K + 1) % 3;   // row before that
        const T cur_raw = pq[KP];
        const float cur_lb = lq[KP];
        if (PATH == P_GEN) {   // the unrolled paths refill the queue per PF rows
            pq[KP] = raw(x + PF);
            lq[KP] = rawlb(x + PF - 1);
        }
        if (MODE == MODE_INCR) {
#pragma unroll
            for (int q = S - 1; q > 0; --q) lbw[q] = lbw[q - 1];
            lbw[0] = cur_lb;
        }
        T rv = T(0);   // P_GEN: ring values of this row (lanes with k = 0)
        if (PATH == P_GEN && n_rc > 0) rv = ring_batch(x);
        // value of the wavefront's ring column at level q (P_MID)
        auto mid_ring = [&](int q) __attribute__((always_inline)) -> T {
            return rring[(x - x0) * RS + q];
        };
        {
            T c = cur_raw;
            // ring values are read by the whole wavefront before the select:
            // under a lane condition the read would become a branch
            if (PATH == P_MID) {
                const T rv0 = mid_ring(0);
                c = ring_lane ? rv0 : c;
            } else if (PATH == P_GEN) {
                if (x > M - 1)
                    c = T(0);
                else if (x == 0 || x == M - 1)
                    c = (jl >= 0 && jl <= M - 1) ? ring(x, 0) : T(0);
                else {
                    c = in_col ? cur_raw : T(0);
                    if (n_rc > 0) {
                        const T rl = bcast(rv, 0), rr_ = bcast(rv, RS);
                        c = (jl == 0) ? rl : ((jl == M - 1) ? rr_ : c);
                    }
                }
            }
            wc[0][K] = c;
        }
#pragma unroll
        for (int q = 1; q <= S; ++q) {
            const int row = x - q;
            const T um = wc[q - 1][K2], u0 = wc[q - 1][K1], up = wc[q - 1][K];
            // row weights from the LDS copy: entry row - (x0 - S)
            const W4 w = wrow[x - x0 + S - q];
            const T wP = w.x, wM = w.y, cR = w.z, gI = w.w;
            const T dd = up - um;
            // right-hand and left-hand neighbour terms of the neighbouring
            // columns (u_{i,j} and the mixed difference u_{i+1,j} - u_{i-1,j})
            const T vr = wRs * u0 + (gI * fjm) * dd;
            const T vl = wLs * u0 - (gI * fjp) * dd;
            const T cc = cR - b2;
            T acc = (MODE == MODE_INCR) ? cc * u0 + (T)lbw[q - 1] : cc * u0;
            acc = acc + wP * up;
            acc = acc + wM * um;
            acc = acc + shl1(vr);
            acc = acc + shr1(vl);
            T c = acc;
            if (PATH == P_MID) {
                const T rvq = mid_ring(q);
                c = ring_lane ? rvq : c;
            } else if (PATH == P_GEN) {
                if (row < 0 || row > M - 1) {
                    c = T(0);
                } else if (row == 0 || row == M - 1) {
                    c = (jl >= 0 && jl <= M - 1) ? ring(row, q) : T(0);
                } else if (n_rc > 0) {
                    const T rl = bcast(rv, q), rr_ = bcast(rv, RS + q);
                    c = (jl == 0) ? rl : ((jl == M - 1) ? rr_ : c);
                }
            }
            if (q == S) {
                if (row >= ia && row < ib && out_lane) dst[(long long)(row - 1) * P + (jl - 1)] = c;
            } else {
                wc[q][K] = c;
            }
        }
    };
    auto general = [&](int x) __attribute__((always_inline)) {
        static_for<PF>([&](auto Kc) {
            if (x % PF == decltype(Kc)::value) iter(Kc, std::integral_constant<int, P_GEN>{}, x);
        });
    };
    int x = x0;
    while (x <= x1 && (x < fb || x % PF != 0)) general(x++);
    // The unrolled paths issue the loads of the next PF rows at the top of
    // the PF rows they evaluate and move them into the queue at the bottom:
    // the move at the loop's back edge then waits on loads issued PF rows
    // earlier, not on loads just issued.
    auto unrolled = [&](auto Pc) __attribute__((always_inline)) {
        for (; x + PF - 1 <= fe; x += PF) {
            T pn[PF];
            float ln[PF];
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                pn[k] = raw(x + PF + k);
                ln[k] = rawlb(x + PF + k - 1);
            }
            static_for<PF>([&](auto Kc) { iter(Kc, Pc, x + decltype(Kc)::value); });
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                pq[k] = pn[k];
                lq[k] = ln[k];
            }
        }
    };
    if (n_rc == 0)
        unrolled(std::integral_constant<int, P_FAST>{});
    else
        unrolled(std::integral_constant<int, P_MID>{});
    while (x <= x1) general(x++);
}

}  // namespace pr
