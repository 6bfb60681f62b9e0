// fno.hip -- the Fourier neural operator coarse propagator on gfx950.
//
// Network (Sec. 3.4; sizes of include/parareal.h): per sample a 64 x 64 grid,
//   lift     z1 = inp L1 + l1, h1 = GELU(z1), v0 = h1 L2 + l2   (7 -> 64 -> 32)
//   layer l  z_l = SpecConv_l(v_l) + v_l W_l + b_l, v_{l+1} = GELU(z_l) (none after the last)
//   project  zq = v4 P1 + p1, hq = GELU(zq), out = hq P2 + p2  (32 -> 128 -> 1)
// SpecConv: truncated DFT to modes kx in {0..11, -12..-1}, ky in {0..11}, a
// complex 32 x 32 multiplier per mode, inverse DFT of the retained half
// spectrum (weights c_0 = 1, c_q = 2, divided by 64^2).
//
// Everything is a strided batched GEMM (k_gemm) plus a few elementwise
// kernels.  The truncated DFTs are real GEMMs against cos/sin tables (FP32).
// The channel contractions (lift, pointwise W, per-mode multipliers,
// projection, and their gradients) run either in FP32 or in BF16 on MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation; operands are rounded to bf16
// as they are staged, the master copies stay FP32).  FP64 instances of the
// same GEMM carry the sine transfers between a fine grid and the FNO grid.
//
// Activation layout: channel-last, sample b, node (x, y), channel c at
// ((b*64 + x)*64 + y)*C + c.  Spectral intermediates (o = output channel):
//   T1[b][x][re/im][q][c]   after the y transform  (rows (x, re/im) = 2x + re/im)
//   X [k][q][b][re/im][c]   after the x transform  (mode-major, for the mixing)
//   Y [b][re/im][k][q][o]   after the mixing
//   Z [b][x][re/im][q][o]   after the inverse x transform
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "parareal.h"

namespace pr {
namespace fno {

constexpr int G = PR_FNO_GRID;     // 64
constexpr int GG = G * G;          // nodes per sample
constexpr int C = PR_FNO_WIDTH;    // 32
constexpr int MX = PR_FNO_MODES;   // 12: kx in {0..11, -12..-1}, ky in {0..11}
constexpr int NKX = 2 * MX;        // 24
constexpr int NMODE = NKX * MX;    // 288
constexpr int CIN = PR_FNO_CIN;    // 7
constexpr int LH = PR_FNO_LIFT;    // 64
constexpr int PH = PR_FNO_PROJ;    // 128
constexpr int NL = PR_FNO_LAYERS;  // 4
constexpr int KT = 32;             // GEMM k tile
constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// GEMM: C[b] (M x N) = alpha * A[b] (M x K) * B[b] (K x N)  (+ beta C + bias),
// every operand addressed by (row stride, column stride, three batch strides)
// in elements, so transposes and the spectral layouts need no copies.
// Epilogue, in order: alpha * acc, + beta * C, + bias[n], * GELU'(Z) (Z in
// C's layout), store; and D = GELU(result) when D is given.
// ---------------------------------------------------------------------------
struct Opnd {
    long long off, rs, cs, b0, b1, b2;
};

template <typename T>
struct GemmArgs {
    const T* A;
    const T* B;
    T* C;
    T* D;
    const T* Z;
    const T* bias;
    Opnd a, b, c;
    long long bias_s;
    int M, N, K;
    int n1, n2;   // batch = n0 x n1 x n2, blockIdx.z = (i0 * n1 + i1) * n2 + i2
    int ones_row; // row of A read as all ones (-1: none)
    T alpha, beta;
};

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}
__device__ inline double gelu_f(double z) { return 0.5 * z * (1.0 + erf(z * 0.70710678118654752)); }
__device__ inline double gelu_grad_f(double z) {
    return 0.5 * (1.0 + erf(z * 0.70710678118654752)) + z * exp(-0.5 * z * z) * 0.39894228040143268;
}

// float -> bf16 bits, round to nearest even (finite inputs).
__device__ inline short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// MF = true: BF16 MFMA (T = float only).  Block tile BM x BN (32x32, 64x32,
// 128x32 or 64x64), 256 threads.
//   FMA : thread (tx, ty) of a 16 x 16 grid owns rows ty + 16 i, columns tx + 16 j.
//   MFMA: four wavefronts in a WM x WN grid, each a (16 PM) x (16 QN) sub-tile of
//         16x16x16 blocks.
template <typename T, int BM, int BN, bool MF>
__global__ __launch_bounds__(kThreads) void k_gemm(GemmArgs<T> g) {
    // FMA: FP32 tiles, k-major.  MFMA: bf16 tiles, k fastest (rounded once when
    // staged), rows padded to 40 elements so that a lane's eight consecutive k
    // are one aligned 16-byte LDS read.
    constexpr int KP = KT + 8;
    __shared__ T As[MF ? 1 : KT][MF ? 1 : BM + 1];
    __shared__ T Bs[MF ? 1 : KT][MF ? 1 : BN + 1];
    __shared__ __attribute__((aligned(16))) short Ab[MF ? BM : 1][MF ? KP : 1];
    __shared__ __attribute__((aligned(16))) short Bb[MF ? BN : 1][MF ? KP : 1];
    auto put_a = [&](int kk, int mm, T v) __attribute__((always_inline)) {
        if constexpr (MF) Ab[mm][kk] = to_bf16((float)v);
        else As[kk][mm] = v;
    };
    auto put_b = [&](int kk, int nn, T v) __attribute__((always_inline)) {
        if constexpr (MF) Bb[nn][kk] = to_bf16((float)v);
        else Bs[kk][nn] = v;
    };
    const int tid = threadIdx.x;
    const int bz = blockIdx.z;
    const int i2 = bz % g.n2;
    const int i1 = (bz / g.n2) % g.n1;
    const int i0 = bz / (g.n2 * g.n1);
    const T* A = g.A + g.a.off + i0 * g.a.b0 + i1 * g.a.b1 + i2 * g.a.b2;
    const T* B = g.B + g.b.off + i0 * g.b.b0 + i1 * g.b.b1 + i2 * g.b.b2;
    const long long coff = g.c.off + i0 * g.c.b0 + i1 * g.c.b1 + i2 * g.c.b2;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const bool a_kfast = g.a.cs == 1;
    const bool b_nfast = g.b.cs == 1;

    constexpr int TM = BM / 16, TN = BN / 16;
    constexpr int WN = (BN >= 64 || BM < 128) ? 2 : 1;   // MFMA wave grid WM x WN = 4 waves
    constexpr int WM = 4 / WN;
    constexpr int PM = BM / (16 * WM), QN = BN / (16 * WN);
    static_assert(PM >= 1 && QN >= 1 && PM * 16 * WM == BM && QN * 16 * WN == BN, "tile");
    const int tx = tid & 15, ty = tid >> 4;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave / WN, wn = wave % WN;

    T acc[TM][TN];
    f32x4 macc[PM][QN];
    if constexpr (MF) {
#pragma unroll
        for (int p = 0; p < PM; ++p)
#pragma unroll
            for (int q = 0; q < QN; ++q) macc[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = T(0);
    }

    // 16-byte loads along a contiguous, aligned fast dimension (FP32 operands)
    bool a_vec = false, b_vec = false;
    if constexpr (std::is_same<T, float>::value) {
        a_vec = a_kfast && g.ones_row < 0 && (g.a.rs % 4 == 0) &&
                ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
        b_vec = b_nfast && (g.b.rs % 4 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    }

    for (int k0 = 0; k0 < g.K; k0 += KT) {
        if (a_vec) {
            for (int e = tid; e < BM * (KT / 4); e += kThreads) {
                const int kk = (e % (KT / 4)) * 4, mm = e / (KT / 4);
                const int m = m0 + mm, k = k0 + kk;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (m < g.M) {
                    const float* src = reinterpret_cast<const float*>(A) + (long long)m * g.a.rs + k;
                    if (k + 3 < g.K) {
                        v = *reinterpret_cast<const float4*>(src);
                    } else {
                        if (k < g.K) v.x = src[0];
                        if (k + 1 < g.K) v.y = src[1];
                        if (k + 2 < g.K) v.z = src[2];
                    }
                }
                put_a(kk, mm, (T)v.x); put_a(kk + 1, mm, (T)v.y);
                put_a(kk + 2, mm, (T)v.z); put_a(kk + 3, mm, (T)v.w);
            }
        } else {
            for (int e = tid; e < BM * KT; e += kThreads) {
                int mm, kk;
                if (a_kfast) { kk = e % KT; mm = e / KT; } else { mm = e % BM; kk = e / BM; }
                const int m = m0 + mm, k = k0 + kk;
                put_a(kk, mm, (m < g.M && k < g.K)
                                  ? (m == g.ones_row ? T(1) : A[(long long)m * g.a.rs + (long long)k * g.a.cs])
                                  : T(0));
            }
        }
        if (b_vec) {
            for (int e = tid; e < KT * (BN / 4); e += kThreads) {
                const int nn = (e % (BN / 4)) * 4, kk = e / (BN / 4);
                const int n = n0 + nn, k = k0 + kk;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (k < g.K) {
                    const float* src = reinterpret_cast<const float*>(B) + (long long)k * g.b.rs + n;
                    if (n + 3 < g.N) {
                        v = *reinterpret_cast<const float4*>(src);
                    } else {
                        if (n < g.N) v.x = src[0];
                        if (n + 1 < g.N) v.y = src[1];
                        if (n + 2 < g.N) v.z = src[2];
                    }
                }
                put_b(kk, nn, (T)v.x); put_b(kk, nn + 1, (T)v.y);
                put_b(kk, nn + 2, (T)v.z); put_b(kk, nn + 3, (T)v.w);
            }
        } else {
            for (int e = tid; e < KT * BN; e += kThreads) {
                int kk, nn;
                if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % KT; nn = e / KT; }
                const int n = n0 + nn, k = k0 + kk;
                put_b(kk, nn, (n < g.N && k < g.K) ? B[(long long)k * g.b.rs + (long long)n * g.b.cs] : T(0));
            }
        }
        __syncthreads();
        if constexpr (MF) {
            // one 16x16x32 product per output block and k tile: lane group
            // lane / 16 holds k = 8 (lane / 16) .. + 7 of its row (A) or column (B)
            static_assert(KT == 32, "one 16x16x32 MFMA per k tile");
            const int kb = (lane >> 4) * 8;
            bf16x8 af[PM], bfr[QN];
#pragma unroll
            for (int p = 0; p < PM; ++p)
                af[p] = *reinterpret_cast<const bf16x8*>(&Ab[wm * 16 * PM + p * 16 + (lane & 15)][kb]);
#pragma unroll
            for (int q = 0; q < QN; ++q)
                bfr[q] = *reinterpret_cast<const bf16x8*>(&Bb[wn * 16 * QN + q * 16 + (lane & 15)][kb]);
#pragma unroll
            for (int p = 0; p < PM; ++p)
#pragma unroll
                for (int q = 0; q < QN; ++q)
                    macc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[p], bfr[q], macc[p][q],
                                                                        0, 0, 0);
        } else {
#pragma unroll 8
            for (int kk = 0; kk < KT; ++kk) {
                T av[TM], bv[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) av[i] = As[kk][ty + 16 * i];
#pragma unroll
                for (int j = 0; j < TN; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[i][j] += av[i] * bv[j];
            }
        }
        __syncthreads();
    }

    auto store = [&](int m, int n, T v) {
        if (m >= g.M || n >= g.N) return;
        const long long ci = coff + (long long)m * g.c.rs + (long long)n * g.c.cs;
        v = g.alpha * v;
        if (g.beta != T(0)) v += g.beta * g.C[ci];
        if (g.bias) v += g.bias[(long long)n * g.bias_s];
        if (g.Z) v *= gelu_grad_f(g.Z[ci]);
        g.C[ci] = v;
        if (g.D) g.D[ci] = gelu_f(v);
    };
    if constexpr (MF) {
#pragma unroll
        for (int p = 0; p < PM; ++p)
#pragma unroll
            for (int q = 0; q < QN; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    store(m0 + wm * 16 * PM + p * 16 + (lane >> 4) * 4 + e,
                          n0 + wn * 16 * QN + q * 16 + (lane & 15), (T)macc[p][q][e]);
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) store(m0 + ty + 16 * i, n0 + tx + 16 * j, acc[i][j]);
    }
}

// Host-side description of one GEMM call.
template <typename T>
struct Gemm {
    GemmArgs<T> g{};
    int n0 = 1;
    Gemm(int M, int N, int K) {
        g.M = M; g.N = N; g.K = K; g.n1 = 1; g.n2 = 1; g.ones_row = -1;
        g.alpha = T(1); g.beta = T(0);
    }
    Gemm& A(const T* p, long long rs, long long cs, long long off = 0) {
        g.A = p; g.a.rs = rs; g.a.cs = cs; g.a.off = off; return *this;
    }
    Gemm& B(const T* p, long long rs, long long cs, long long off = 0) {
        g.B = p; g.b.rs = rs; g.b.cs = cs; g.b.off = off; return *this;
    }
    Gemm& Cm(T* p, long long rs, long long cs, long long off = 0) {
        g.C = p; g.c.rs = rs; g.c.cs = cs; g.c.off = off; return *this;
    }
    // batch level: sizes and the strides of A, B, C along it
    Gemm& batch(int level, int n, long long sa, long long sb, long long sc) {
        if (level == 0) { n0 = n; g.a.b0 = sa; g.b.b0 = sb; g.c.b0 = sc; }
        if (level == 1) { g.n1 = n; g.a.b1 = sa; g.b.b1 = sb; g.c.b1 = sc; }
        if (level == 2) { g.n2 = n; g.a.b2 = sa; g.b.b2 = sb; g.c.b2 = sc; }
        return *this;
    }
    Gemm& scale(T alpha, T beta) { g.alpha = alpha; g.beta = beta; return *this; }
    Gemm& bias(const T* p, long long s = 1) { g.bias = p; g.bias_s = s; return *this; }
    Gemm& act_out(T* d) { g.D = d; return *this; }
    Gemm& dact(const T* z) { g.Z = z; return *this; }
    Gemm& ones(int row) { g.ones_row = row; return *this; }
};

template <typename T, int BM, int BN, bool MF>
static void launch_tile(const Gemm<T>& q, hipStream_t st) {
    dim3 grid((q.g.M + BM - 1) / BM, (q.g.N + BN - 1) / BN, q.n0 * q.g.n1 * q.g.n2);
    hipLaunchKernelGGL((k_gemm<T, BM, BN, MF>), grid, dim3(kThreads), 0, st, q.g);
}

template <typename T>
static hipError_t run(const Gemm<T>& q, bool mfma, hipStream_t st) {
    if (q.g.M <= 0 || q.g.N <= 0 || q.g.K <= 0) return hipErrorInvalidValue;
    if ((long long)q.n0 * q.g.n1 * q.g.n2 > 65535) return hipErrorInvalidValue;
    // tile by output shape: small outputs (the truncated transforms) would
    // leave most of a 64 x 64 tile idle
    const int M = q.g.M, N = q.g.N;
    const int shape = (N <= 32) ? (M <= 32 ? 0 : (M <= 64 ? 1 : 2)) : 3;
    if constexpr (std::is_same<T, float>::value) {
        if (mfma) {
            switch (shape) {
                case 0: launch_tile<float, 32, 32, true>(q, st); break;
                case 1: launch_tile<float, 64, 32, true>(q, st); break;
                case 2: launch_tile<float, 128, 32, true>(q, st); break;
                default: launch_tile<float, 64, 64, true>(q, st); break;
            }
        } else {
            switch (shape) {
                case 0: launch_tile<float, 32, 32, false>(q, st); break;
                case 1: launch_tile<float, 64, 32, false>(q, st); break;
                case 2: launch_tile<float, 128, 32, false>(q, st); break;
                default: launch_tile<float, 64, 64, false>(q, st); break;
            }
        }
    } else {
        (void)mfma; (void)shape;
        launch_tile<T, 64, 64, false>(q, st);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Elementwise kernels.
// ---------------------------------------------------------------------------
// Network input of sample b: channels [w, s1, s2, rho, r, x/63, y/63].
// w of sample b at w + src(b)*wstride, its parameters at meta + src(b)*4,
// src(b) = idx ? idx[b] (clamped to [0, nsrc)) : b.
__global__ void k_input(const float* __restrict__ w, long long wstride,
                        const float* __restrict__ meta, const int* __restrict__ idx, int nsrc,
                        float* __restrict__ inp, int B) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * GG) return;
    const int b = (int)(t / GG), p = (int)(t % GG);
    const int sb = idx ? min(max(idx[b], 0), nsrc - 1) : b;
    const float* mt = meta + (long long)sb * 4;
    float* o = inp + t * CIN;
    o[0] = w[(long long)sb * wstride + p];
    o[1] = mt[0]; o[2] = mt[1]; o[3] = mt[2]; o[4] = mt[3];
    o[5] = (float)(p / G) / (float)(G - 1);
    o[6] = (float)(p % G) / (float)(G - 1);
}

// Stacked real form of the complex multipliers of every layer:
// Rs[l][mode] (64 x 64) = [[Rr, Ri], [-Ri, Rr]], so that [Yre Yim] = [Xre Xim] Rs.
__global__ void k_stack(const float* __restrict__ params, const long long* __restrict__ offs,
                        float* __restrict__ Rs) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)NL * NMODE * 4 * C * C) return;
    const int col = (int)(t % (2 * C));
    const int row = (int)((t / (2 * C)) % (2 * C));
    const int mode = (int)((t / (4 * C * C)) % NMODE);
    const int l = (int)(t / ((long long)NMODE * 4 * C * C));
    const int ri = row / C, i = row % C, ro = col / C, o = col % C;
    const long long e = (long long)mode * C * C + i * C + o;
    const float rr = params[offs[2 * l] + e], im = params[offs[2 * l + 1] + e];
    Rs[t] = (ri == ro) ? rr : (ri == 0 ? im : -im);
}

// Gradient of the stacked multipliers back to (Rr, Ri) of layer l:
// gRr = g00 + g11, gRi = g01 - g10.
__global__ void k_fold(const float* __restrict__ gRs, float* __restrict__ gRr,
                       float* __restrict__ gRi) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NMODE * C * C) return;
    const int o = t % C, i = (t / C) % C, mode = t / (C * C);
    const float* s = gRs + (long long)mode * 4 * C * C;
    const float g00 = s[i * 2 * C + o], g01 = s[i * 2 * C + C + o];
    const float g10 = s[(C + i) * 2 * C + o], g11 = s[(C + i) * 2 * C + C + o];
    gRr[t] = g00 + g11;
    gRi[t] = g01 - g10;
}

// Loss of Sec. 3.5 on the 64^2 grid, pass 1 (one workgroup per sample row x):
// V1 = B1 + w_in + s*out (interior), d = V1 - V_tgt,
// R = (V1 - V_in) - dT L_h((V1 + V_in)/2) on the interior; per-row sums of d^2
// and R^2; gpred = s * (2 d + 2 lam R) / (B n_int); cc = -dT lam R / (B n_int).
// A training pair is four 64^2 planes [w_in, B1, V_in, V_tgt] at
// pairs + src(b) * 4 * 4096.
struct LossArgs {
    const float* out;
    const float* pairs;
    const float* meta;
    const int* idx;
    int nsrc;      // pairs addressable through idx (indices are clamped to [0, nsrc))
    float* gpred;
    float* cc;
    double* part;
    int B;
    double scale, dT, lam;
    double skip;   // 1: the prediction is a change of w_in, 0: the new w
};

__device__ inline double v1_at(const LossArgs& a, const float* pr, const float* ob, int x, int y) {
    const int p = x * G + y;
    const bool in = x > 0 && x < G - 1 && y > 0 && y < G - 1;
    return (double)pr[GG + p] + a.skip * (double)pr[p] + (in ? a.scale * (double)ob[p] : 0.0);
}

__global__ __launch_bounds__(64) void k_loss1(LossArgs a) {
    const int b = blockIdx.x / G, x = blockIdx.x % G, y = threadIdx.x;
    const int sb = a.idx ? min(max(a.idx[b], 0), a.nsrc - 1) : b;
    const float* pr = a.pairs + (long long)sb * 4 * GG;
    const float* ob = a.out + (long long)b * GG;
    const float* mt = a.meta + (long long)sb * 4;
    const double s1 = mt[0], s2 = mt[1], rho = mt[2], r = mt[3];
    const double nint = (double)(G - 2) * (G - 2);
    const double norm = 1.0 / (a.B * nint);
    double dsq = 0.0, rsq = 0.0, gp = 0.0, c = 0.0;
    if (x > 0 && x < G - 1 && y > 0 && y < G - 1) {
        auto avg = [&](int i, int j) {
            return 0.5 * (v1_at(a, pr, ob, i, j) + (double)pr[2 * GG + i * G + j]);
        };
        const double I = x, J = y;
        const double al = 0.5 * s1 * s1 * I * I, be = 0.5 * s2 * s2 * J * J;
        const double ga = 0.25 * rho * s1 * s2 * I * J, hr = 0.5 * r;
        const double u0 = avg(x, y);
        const double lh = al * (avg(x + 1, y) - 2.0 * u0 + avg(x - 1, y)) +
                          be * (avg(x, y + 1) - 2.0 * u0 + avg(x, y - 1)) +
                          ga * (avg(x + 1, y + 1) + avg(x - 1, y - 1) - avg(x + 1, y - 1) -
                                avg(x - 1, y + 1)) +
                          hr * I * (avg(x + 1, y) - avg(x - 1, y)) +
                          hr * J * (avg(x, y + 1) - avg(x, y - 1)) - r * u0;
        const double v1 = v1_at(a, pr, ob, x, y);
        const double d = v1 - (double)pr[3 * GG + x * G + y];
        const double R = (v1 - (double)pr[2 * GG + x * G + y]) - a.dT * lh;
        dsq = d * d;
        rsq = R * R;
        gp = 2.0 * d * norm + a.lam * 2.0 * R * norm;
        c = -0.5 * a.dT * a.lam * 2.0 * R * norm;
    }
    a.gpred[(long long)b * GG + x * G + y] = (float)gp;   // scaled in pass 2
    a.cc[(long long)b * GG + x * G + y] = (float)c;
    // row sums: wavefront reduction in a fixed order
    for (int off = 32; off > 0; off >>= 1) {
        dsq += __shfl_down(dsq, off);
        rsq += __shfl_down(rsq, off);
    }
    if (y == 0) {
        a.part[2 * blockIdx.x] = dsq;
        a.part[2 * blockIdx.x + 1] = rsq;
    }
}

// Pass 2: add the adjoint of -dT L_h(V1 / 2) (a gather of cc through the
// nine-point stencil of every interior centre), mask the ring, scale.
__global__ __launch_bounds__(64) void k_loss2(LossArgs a) {
    const int b = blockIdx.x / G, x = blockIdx.x % G, y = threadIdx.x;
    const int sb = a.idx ? min(max(a.idx[b], 0), a.nsrc - 1) : b;
    const float* mt = a.meta + (long long)sb * 4;
    const double s1 = mt[0], s2 = mt[1], rho = mt[2], r = mt[3];
    const float* cb = a.cc + (long long)b * GG;
    const long long o = (long long)b * GG + x * G + y;
    if (!(x > 0 && x < G - 1 && y > 0 && y < G - 1)) { a.gpred[o] = 0.0f; return; }
    auto cc = [&](int i, int j) -> double { return (double)cb[i * G + j]; };
    auto al = [&](int i) { return 0.5 * s1 * s1 * i * i; };
    auto be = [&](int j) { return 0.5 * s2 * s2 * j * j; };
    auto ga = [&](int i, int j) { return 0.25 * rho * s1 * s2 * i * j; };
    const double hr = 0.5 * r;
    double gw = cc(x, y) * (-2.0 * al(x) - 2.0 * be(y) - r);
    gw += cc(x - 1, y) * (al(x - 1) + hr * (x - 1));       // centre (x-1, y), node x = its i+1
    gw += cc(x + 1, y) * (al(x + 1) - hr * (x + 1));       // centre (x+1, y), its i-1
    gw += cc(x, y - 1) * (be(y - 1) + hr * (y - 1));
    gw += cc(x, y + 1) * (be(y + 1) - hr * (y + 1));
    gw += cc(x - 1, y - 1) * ga(x - 1, y - 1);             // (i+1, j+1) of that centre
    gw += cc(x + 1, y + 1) * ga(x + 1, y + 1);             // (i-1, j-1)
    gw -= cc(x - 1, y + 1) * ga(x - 1, y + 1);             // (i+1, j-1)
    gw -= cc(x + 1, y - 1) * ga(x + 1, y - 1);             // (i-1, j+1)
    a.gpred[o] = (float)(a.scale * ((double)a.gpred[o] + gw));
}

// Sum of the per-row partials in a fixed order; res = [loss, data, residual].
__global__ __launch_bounds__(256) void k_loss3(const double* __restrict__ part, int rows, double B,
                                               double lam, double* __restrict__ res) {
    __shared__ double sd[256], sr[256];
    double d = 0.0, r = 0.0;
    for (int i = threadIdx.x; i < rows; i += 256) { d += part[2 * i]; r += part[2 * i + 1]; }
    sd[threadIdx.x] = d;
    sr[threadIdx.x] = r;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) { sd[threadIdx.x] += sd[threadIdx.x + s]; sr[threadIdx.x] += sr[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nint = (double)(G - 2) * (G - 2);
        const double data = sd[0] / (B * nint), resid = sr[0] / (B * nint);
        res[0] = data + lam * resid;
        res[1] = data;
        res[2] = resid;
    }
}

// Adam (Kingma and Ba) over the flat parameter vector; c1 = 1 - b1^t, c2 = 1 - b2^t.
// out[g][c] = sum of in[s][c] over s in [g * per, min((g + 1) * per, S)), in
// order of s (rows of W floats); grid (ceil(W / 256), groups).
__global__ void k_colsum(const float* __restrict__ in, int S, int W, int per,
                         float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (c >= W) return;
    const int s0 = g * per, s1 = min((g + 1) * per, S);
    float acc = 0.f;
    int s = s0;
    // eight loads in flight per round; the adds stay in the order of s
    for (; s + 8 <= s1; s += 8) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = in[(long long)(s + e) * W + c];
#pragma unroll
        for (int e = 0; e < 8; ++e) acc += v[e];
    }
    for (; s < s1; ++s) acc += in[(long long)s * W + c];
    out[(long long)g * W + c] = acc;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

inline int blocks_for(long long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace fno
}  // namespace pr

// ===========================================================================
// The FNO runtime behind pr_fno_*.
// ===========================================================================
using namespace pr::fno;

namespace {

constexpr uint64_t kAlign = 256;
inline uint64_t al(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Parameter blocks in the order of the flat vector.
struct ParamIndex {
    long long L1, l1, L2, l2, Rr[NL], Ri[NL], W[NL], b[NL], P1, p1, P2, p2, total;
    ParamIndex() {
        long long o = 0;
        auto take = [&](long long n) { long long at = o; o += n; return at; };
        L1 = take(CIN * LH); l1 = take(LH); L2 = take(LH * C); l2 = take(C);
        for (int l = 0; l < NL; ++l) {
            Rr[l] = take((long long)NMODE * C * C);
            Ri[l] = take((long long)NMODE * C * C);
            W[l] = take(C * C);
            b[l] = take(C);
        }
        P1 = take(C * PH); p1 = take(PH); P2 = take(PH); p2 = take(1);
        total = o;
    }
};

// Weight-gradient reductions over the Q = batch x 4096 nodes are split into
// chunks of kSplitRows nodes (one product per chunk, many workgroups in
// flight), then the chunk partials are summed in a fixed order in groups of
// kSumGroup and the group sums again.
constexpr int kSplitRows = 128;
constexpr int kSumGroup = 32;

struct Layout {
    uint64_t params, grads, m, v, Rs, gRs, tabs, offs, ones;
    uint64_t inp, z1, h1, vv[NL], zz[NL], T1, X[NL], Y, Z, zq, hq, out;
    uint64_t gA, gB, gbig, gT, gX, gY, part, part2, gpred, cc, lpart, lres;
    uint64_t total;
};

Layout make_layout(int Bm) {
    const ParamIndex pi;
    const uint64_t Q = (uint64_t)Bm * GG;
    Layout L{};
    uint64_t p = 0;
    auto take = [&](uint64_t bytes) { uint64_t at = p; p = al(p + bytes); return at; };
    const uint64_t f = 4;
    L.params = take(pi.total * f);
    L.grads = take(pi.total * f);
    L.m = take(pi.total * f);
    L.v = take(pi.total * f);
    L.Rs = take((uint64_t)NL * NMODE * 4 * C * C * f);
    L.gRs = take((uint64_t)NMODE * 4 * C * C * f);
    L.tabs = take((uint64_t)(2 * MX * G + 2 * NKX * 2 * G + 2 * G * 2 * NKX + G * 2 * MX) * f);
    L.offs = take(2 * NL * 8);
    L.ones = take(f);
    L.inp = take(Q * CIN * f);
    L.z1 = take(Q * LH * f);
    L.h1 = take(Q * LH * f);
    for (int l = 0; l < NL; ++l) L.vv[l] = take(Q * C * f);
    for (int l = 0; l < NL; ++l) L.zz[l] = take(Q * C * f);
    L.T1 = take((uint64_t)Bm * G * 2 * MX * C * f);
    for (int l = 0; l < NL; ++l) L.X[l] = take((uint64_t)NMODE * Bm * 2 * C * f);
    L.Y = take((uint64_t)Bm * 2 * NMODE * C * f);
    L.Z = take((uint64_t)Bm * G * 2 * MX * C * f);
    L.zq = take(Q * PH * f);
    L.hq = take(Q * PH * f);
    L.out = take(Q * f);
    L.gA = take(Q * C * f);
    L.gB = take(Q * C * f);
    L.gbig = take(Q * PH * f);
    L.gT = take((uint64_t)Bm * G * 2 * MX * C * f);
    L.gX = take((uint64_t)NMODE * Bm * 2 * C * f);
    L.gY = take((uint64_t)Bm * 2 * NMODE * C * f);
    // largest (K+1) x N: P1 and p1
    const uint64_t nsplit = (Q + kSplitRows - 1) / kSplitRows;
    L.part = take(nsplit * (C + 1) * PH * f);
    L.part2 = take((nsplit + kSumGroup - 1) / kSumGroup * (C + 1) * PH * f);
    L.gpred = take(Q * f);
    L.cc = take(Q * f);
    L.lpart = take((uint64_t)Bm * G * 2 * 8);
    L.lres = take(4 * 8);
    L.total = p;
    return L;
}

// cos / sin tables of the truncated transforms (host, double -> float).
//   EyF (24 x 64)   [re/im * 12 + q][y]:  cos(th q y), -sin(th q y)
//   ExF (2 x 24 x 128) [ro][k][2x + ri]:  ro=0: (c, s), ro=1: (-s, c), c/s of th kx x
//   ExI (128 x 48)  [2x + rz][ri * 24 + k]: rz=0: (c, -s), rz=1: (s, c)
//   EyI (64 x 24)   [y][ri * 12 + q]: w_q cos(th q y), -w_q sin(th q y), w_q = c_q / 4096
std::vector<float> make_tables() {
    const double th = 2.0 * M_PI / G;
    auto kx = [](int k) { return k < MX ? k : k - NKX; };
    std::vector<float> t;
    for (int ri = 0; ri < 2; ++ri)
        for (int q = 0; q < MX; ++q)
            for (int y = 0; y < G; ++y)
                t.push_back((float)(ri == 0 ? std::cos(th * q * y) : -std::sin(th * q * y)));
    for (int ro = 0; ro < 2; ++ro)
        for (int k = 0; k < NKX; ++k)
            for (int x = 0; x < G; ++x) {
                const double c = std::cos(th * kx(k) * x), s = std::sin(th * kx(k) * x);
                if (ro == 0) { t.push_back((float)c); t.push_back((float)s); }
                else { t.push_back((float)-s); t.push_back((float)c); }
            }
    for (int x = 0; x < G; ++x)
        for (int rz = 0; rz < 2; ++rz)
            for (int ri = 0; ri < 2; ++ri)
                for (int k = 0; k < NKX; ++k) {
                    const double c = std::cos(th * kx(k) * x), s = std::sin(th * kx(k) * x);
                    double v;
                    if (rz == 0) v = (ri == 0) ? c : -s;
                    else v = (ri == 0) ? s : c;
                    t.push_back((float)v);
                }
    for (int y = 0; y < G; ++y)
        for (int ri = 0; ri < 2; ++ri)
            for (int q = 0; q < MX; ++q) {
                const double w = (q == 0 ? 1.0 : 2.0) / (double)GG;
                t.push_back((float)(ri == 0 ? w * std::cos(th * q * y) : -w * std::sin(th * q * y)));
            }
    return t;
}

}  // namespace

struct pr_fno {
    int Bm = 0;
    hipStream_t st = nullptr;
    char* ws = nullptr;
    Layout L{};
    ParamIndex pi;
    float* params = nullptr;
    float* grads = nullptr;
    float *EyF = nullptr, *ExF = nullptr, *ExI = nullptr, *EyI = nullptr, *ones = nullptr;
    bool stacked = false;   // Rs matches params
    int fwd_batch = 0;      // batch of the last forward (0: none)
    int fwd_prec = 0;       // precision of the last forward
    int infer_prec = 0;     // precision of the coarse-propagator inference
    double out_scale = 1.0;
    int base = PR_FNO_BASE_IDENTITY;
    double skip = 1.0;      // 1 when the prediction is a change of w_in
    std::string err;
    template <typename T = float>
    T* at(uint64_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

pr_status fail(pr_fno* f, pr_status st, const std::string& m) {
    if (f) f->err = m;
    return st;
}

#define FNO_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) return fail(f, PR_EDEVICE, hipGetErrorString(e_));   \
    } while (0)

hipError_t ensure_stacked(pr_fno* f) {
    if (f->stacked) return hipSuccess;
    const long long n = (long long)NL * NMODE * 4 * C * C;
    hipLaunchKernelGGL(k_stack, dim3(blocks_for(n, 256)), dim3(256), 0, f->st, f->params,
                       f->at<long long>(f->L.offs), f->at(f->L.Rs));
    f->stacked = true;
    return hipGetLastError();
}

#define TRY(x)                                    \
    do {                                          \
        hipError_t e_ = (x);                      \
        if (e_ != hipSuccess) return e_;          \
    } while (0)

// Pointwise layer over Q rows: out (Q x N) = in (Q x K) Wt (K x N) + bias.
hipError_t dense(pr_fno* f, const float* in, int K, const float* W, const float* bias, int N,
                 float* out, float* act, long long Q, bool mf, float beta = 0.0f) {
    Gemm<float> q((int)Q, N, K);
    q.A(in, K, 1).B(W, N, 1).Cm(out, N, 1).scale(1.0f, beta);
    if (bias) q.bias(bias);
    if (act) q.act_out(act);
    return run(q, mf, f->st);
}

// gW (K x N) = in^T (K x Q) g (Q x N), written to dst; split over Q, then summed
// in a fixed order.  bias: also the column sums of g, as row K (the flat
// parameter vector keeps every bias block right after its weight block).
hipError_t wgrad(pr_fno* f, const float* in, int K, const float* g, int N, float* dst,
                 long long Q, bool mf, bool bias = true) {
    const int KB = bias ? K + 1 : K;   // rows of the product; row K reads ones
    const long long kc = kSplitRows;
    const int S = (int)((Q + kc - 1) / kc);
    float* part = f->at(f->L.part);
    // the last split may be short: K bounds are per split, so run the full
    // splits and the tail separately
    const int full = (int)(Q / kc);
    if (full > 0) {
        Gemm<float> a(KB, N, (int)kc);
        a.A(in, 1, K).B(g, N, 1).Cm(part, N, 1).batch(0, full, kc * K, kc * N, (long long)KB * N);
        if (bias) a.ones(K);
        TRY(run(a, mf, f->st));
    }
    if (full < S) {
        const long long rem = Q - (long long)full * kc;
        Gemm<float> a(KB, N, (int)rem);
        a.A(in, 1, K, (long long)full * kc * K).B(g, N, 1, (long long)full * kc * N)
            .Cm(part, N, 1, (long long)full * KB * N);
        if (bias) a.ones(K);
        TRY(run(a, mf, f->st));
    }
    // dst = sum over the S partials (KB * N each), in a fixed order
    const int W = KB * N, NG = (S + kSumGroup - 1) / kSumGroup;
    float* part2 = f->at(f->L.part2);
    hipLaunchKernelGGL(k_colsum, dim3((W + 255) / 256, NG), dim3(256), 0, f->st, part, S, W,
                       kSumGroup, part2);
    hipLaunchKernelGGL(k_colsum, dim3((W + 255) / 256, 1), dim3(256), 0, f->st, part2, NG, W, NG,
                       dst);
    return hipGetLastError();
}

// Spectral convolution of layer l, accumulated onto z (which holds v W + b);
// act (optional) receives GELU of the sum.
hipError_t spectral_fwd(pr_fno* f, int l, const float* v, float* z, float* act, int B, bool mf) {
    float* T1 = f->at(f->L.T1);
    float* X = f->at(f->L.X[l]);
    float* Y = f->at(f->L.Y);
    float* Z = f->at(f->L.Z);
    const float* Rs = f->at(f->L.Rs) + (long long)l * NMODE * 4 * C * C;
    const long long sT1 = (long long)G * 2 * MX * C;   // per sample in T1 / Z
    const long long sY = 2LL * NMODE * C;              // per sample in Y
    // y transform, batch (b, x): T1[b][x] (24 x C) = EyF (24 x 64) v[b][x] (64 x C)
    {
        Gemm<float> q(2 * MX, C, G);
        q.A(f->EyF, G, 1).B(v, C, 1).Cm(T1, C, 1).batch(0, B * G, 0, (long long)G * C, 2LL * MX * C);
        TRY(run(q, false, f->st));
    }
    // x transform, batch (b, q, ro): X[k][q][b][ro][c] = sum_{x,ri} ExF[ro][k][2x+ri] T1[b][x][ri][q][c]
    {
        Gemm<float> q(NKX, C, 2 * G);
        q.A(f->ExF, 2 * G, 1).B(T1, (long long)MX * C, 1)
            .Cm(X, (long long)MX * B * 2 * C, 1)
            .batch(0, B, 0, sT1, 2 * C)
            .batch(1, MX, 0, C, (long long)B * 2 * C)
            .batch(2, 2, (long long)NKX * 2 * G, 0, C);
        TRY(run(q, false, f->st));
    }
    // mixing, batch (k, q, ro): Y[b][ro][k][q][:] = X[k][q][b][:] (B x 2C) Rs[k][q][:, ro C : ro C + C]
    {
        Gemm<float> q(B, C, 2 * C);
        q.A(X, 2 * C, 1).B(Rs, 2 * C, 1).Cm(Y, sY, 1)
            .batch(0, NKX, (long long)MX * B * 2 * C, (long long)MX * 4 * C * C, (long long)MX * C)
            .batch(1, MX, (long long)B * 2 * C, 4LL * C * C, C)
            .batch(2, 2, 0, C, (long long)NMODE * C);
        TRY(run(q, mf, f->st));
    }
    // inverse x transform, batch (b, q): Z[b][2x+rz][q][:] = ExI (128 x 48) Y[b][ri*24+k][q][:]
    {
        Gemm<float> q(2 * G, C, 2 * NKX);
        q.A(f->ExI, 2 * NKX, 1).B(Y, (long long)MX * C, 1).Cm(Z, (long long)MX * C, 1)
            .batch(0, B, 0, sY, sT1)
            .batch(1, MX, 0, C, C);
        TRY(run(q, false, f->st));
    }
    // inverse y transform, batch (b, x): z[b][x] (64 x C) += EyI (64 x 24) Z[b][x] (24 x C)
    {
        Gemm<float> q(G, C, 2 * MX);
        q.A(f->EyI, 2 * MX, 1).B(Z, C, 1).Cm(z, C, 1).scale(1.0f, 1.0f)
            .batch(0, B * G, 0, 2LL * MX * C, (long long)G * C);
        if (act) q.act_out(act);
        TRY(run(q, false, f->st));
    }
    return hipSuccess;
}

// Backward of the spectral convolution of layer l: gz (B, 64, 64, C) is the
// gradient at its output; writes gRr, gRi of layer l into the gradient vector
// and gv (beta 0) = gradient at its input v.
hipError_t spectral_bwd(pr_fno* f, int l, const float* gz, float* gv, int B, bool mf) {
    float* gT = f->at(f->L.gT);
    float* gY = f->at(f->L.gY);
    float* gX = f->at(f->L.gX);
    float* gRs = f->at(f->L.gRs);
    const float* X = f->at(f->L.X[l]);
    const float* Rs = f->at(f->L.Rs) + (long long)l * NMODE * 4 * C * C;
    const long long sT1 = (long long)G * 2 * MX * C;
    const long long sY = 2LL * NMODE * C;
    // gZ[b][x] (24 x C) = EyI^T (24 x 64) gz[b][x] (64 x C)
    {
        Gemm<float> q(2 * MX, C, G);
        q.A(f->EyI, 1, 2 * MX).B(gz, C, 1).Cm(gT, C, 1).batch(0, B * G, 0, (long long)G * C, 2LL * MX * C);
        TRY(run(q, false, f->st));
    }
    // gY[b][ri*24+k][q][:] = ExI^T (48 x 128) gZ[b][2x+rz][q][:]
    {
        Gemm<float> q(2 * NKX, C, 2 * G);
        q.A(f->ExI, 1, 2 * NKX).B(gT, (long long)MX * C, 1).Cm(gY, (long long)MX * C, 1)
            .batch(0, B, 0, sT1, sY)
            .batch(1, MX, 0, C, C);
        TRY(run(q, false, f->st));
    }
    // gX[k][q] (B x 2C) = sum_ri gY[b][ri][k][q][:] (B x C) Rs[k][q]^T[ri C : ri C + C, :]
    for (int ri = 0; ri < 2; ++ri) {
        Gemm<float> q(B, 2 * C, C);
        q.A(gY, sY, 1, (long long)ri * NMODE * C).B(Rs, 1, 2 * C, (long long)ri * C)
            .Cm(gX, 2 * C, 1).scale(1.0f, ri ? 1.0f : 0.0f)
            .batch(0, NKX, (long long)MX * C, (long long)MX * 4 * C * C, (long long)MX * B * 2 * C)
            .batch(1, MX, C, 4LL * C * C, (long long)B * 2 * C);
        TRY(run(q, mf, f->st));
    }
    // gRs[k][q][:, ro C : ro C + C] (2C x C) = X[k][q]^T (2C x B) gY[b][ro][k][q][:] (B x C)
    {
        Gemm<float> q(2 * C, C, B);
        q.A(X, 1, 2 * C).B(gY, sY, 1).Cm(gRs, 2 * C, 1)
            .batch(0, NKX, (long long)MX * B * 2 * C, (long long)MX * C, (long long)MX * 4 * C * C)
            .batch(1, MX, (long long)B * 2 * C, C, 4LL * C * C)
            .batch(2, 2, 0, (long long)NMODE * C, C);
        TRY(run(q, mf, f->st));
    }
    hipLaunchKernelGGL(k_fold, dim3(blocks_for((long long)NMODE * C * C, 256)), dim3(256), 0, f->st,
                       gRs, f->grads + f->pi.Rr[l], f->grads + f->pi.Ri[l]);
    TRY(hipGetLastError());
    // gT1[b][2x+ri][q][:] = sum_ro ExF[ro]^T (128 x 24) gX[k][q][b][ro][:] (24 x C)
    for (int ro = 0; ro < 2; ++ro) {
        Gemm<float> q(2 * G, C, NKX);
        q.A(f->ExF, 1, 2 * G, (long long)ro * NKX * 2 * G)
            .B(gX, (long long)MX * B * 2 * C, 1, (long long)ro * C)
            .Cm(gT, (long long)MX * C, 1).scale(1.0f, ro ? 1.0f : 0.0f)
            .batch(0, B, 0, 2 * C, sT1)
            .batch(1, MX, 0, (long long)B * 2 * C, C);
        TRY(run(q, false, f->st));
    }
    // gv[b][x] (64 x C) = EyF^T (64 x 24) gT1[b][x] (24 x C)
    {
        Gemm<float> q(G, C, 2 * MX);
        q.A(f->EyF, 1, G).B(gT, C, 1).Cm(gv, C, 1)
            .batch(0, B * G, 0, 2LL * MX * C, (long long)G * C);
        TRY(run(q, false, f->st));
    }
    return hipSuccess;
}

hipError_t forward(pr_fno* f, const float* w, long long wstride, const float* meta, const int* idx,
                   int nsrc, int B, bool mf, float* out) {
    TRY(ensure_stacked(f));
    const long long Q = (long long)B * GG;
    float* inp = f->at(f->L.inp);
    hipLaunchKernelGGL(k_input, dim3(blocks_for(Q, 256)), dim3(256), 0, f->st, w, wstride, meta, idx,
                       nsrc, inp, B);
    TRY(hipGetLastError());
    const float* P = f->params;
    const ParamIndex& pi = f->pi;
    TRY(dense(f, inp, CIN, P + pi.L1, P + pi.l1, LH, f->at(f->L.z1), f->at(f->L.h1), Q, mf));
    TRY(dense(f, f->at(f->L.h1), LH, P + pi.L2, P + pi.l2, C, f->at(f->L.vv[0]), nullptr, Q, mf));
    for (int l = 0; l < NL; ++l) {
        float* v = f->at(f->L.vv[l]);
        float* z = f->at(f->L.zz[l]);
        TRY(dense(f, v, C, P + pi.W[l], P + pi.b[l], C, z, nullptr, Q, mf));
        float* act = (l < NL - 1) ? f->at(f->L.vv[l + 1]) : nullptr;
        TRY(spectral_fwd(f, l, v, z, act, B, mf));
    }
    const float* v4 = f->at(f->L.zz[NL - 1]);
    TRY(dense(f, v4, C, P + pi.P1, P + pi.p1, PH, f->at(f->L.zq), f->at(f->L.hq), Q, mf));
    TRY(dense(f, f->at(f->L.hq), PH, P + pi.P2, P + pi.p2, 1, out, nullptr, Q, mf));
    return hipSuccess;
}

hipError_t backward(pr_fno* f, const float* gout, int B, bool mf) {
    const long long Q = (long long)B * GG;
    const float* P = f->params;
    float* Gd = f->grads;
    const ParamIndex& pi = f->pi;
    float* gbig = f->at(f->L.gbig);
    float* gA = f->at(f->L.gA);
    float* gB = f->at(f->L.gB);
    // projection
    TRY(wgrad(f, f->at(f->L.hq), PH, gout, 1, Gd + pi.P2, Q, mf));   // and p2
    {   // gzq = gout P2^T * GELU'(zq)
        Gemm<float> q((int)Q, PH, 1);
        q.A(gout, 1, 0).B(P + pi.P2, 0, 1).Cm(gbig, PH, 1).dact(f->at(f->L.zq));
        TRY(run(q, false, f->st));
    }
    const float* v4 = f->at(f->L.zz[NL - 1]);
    TRY(wgrad(f, v4, C, gbig, PH, Gd + pi.P1, Q, mf));   // and p1
    {   // gv4 = gzq P1^T (no activation after the last layer)
        Gemm<float> q((int)Q, C, PH);
        q.A(gbig, PH, 1).B(P + pi.P1, 1, PH).Cm(gA, C, 1);
        TRY(run(q, mf, f->st));
    }
    // layers: gA holds dL/dz_l on entry
    for (int l = NL - 1; l >= 0; --l) {
        const float* v = f->at(f->L.vv[l]);
        TRY(wgrad(f, v, C, gA, C, Gd + pi.W[l], Q, mf));   // and b_l
        TRY(spectral_bwd(f, l, gA, gB, B, mf));
        // gB += gA W^T, times GELU'(z_{l-1}) when v_l = GELU(z_{l-1})
        Gemm<float> q((int)Q, C, C);
        q.A(gA, C, 1).B(P + pi.W[l], 1, C).Cm(gB, C, 1).scale(1.0f, 1.0f);
        if (l > 0) q.dact(f->at(f->L.zz[l - 1]));
        TRY(run(q, mf, f->st));
        std::swap(gA, gB);
    }
    // lift: gA = dL/dv0
    TRY(wgrad(f, f->at(f->L.h1), LH, gA, C, Gd + pi.L2, Q, mf));   // and l2
    {   // gz1 = gv0 L2^T * GELU'(z1)
        Gemm<float> q((int)Q, LH, C);
        q.A(gA, C, 1).B(P + pi.L2, 1, C).Cm(gbig, LH, 1).dact(f->at(f->L.z1));
        TRY(run(q, mf, f->st));
    }
    TRY(wgrad(f, f->at(f->L.inp), CIN, gbig, LH, Gd + pi.L1, Q, mf));   // and l1
    return hipSuccess;
}

hipError_t loss(pr_fno* f, const float* out, const float* pairs, const float* meta, const int* idx,
                int nsrc, int B, double scale, double dT, double lam) {
    LossArgs a{out, pairs, meta, idx, nsrc, f->at(f->L.gpred), f->at(f->L.cc),
               f->at<double>(f->L.lpart), B, scale, dT, lam, f->skip};
    hipLaunchKernelGGL(k_loss1, dim3(B * G), dim3(64), 0, f->st, a);
    hipLaunchKernelGGL(k_loss2, dim3(B * G), dim3(64), 0, f->st, a);
    hipLaunchKernelGGL(k_loss3, dim3(1), dim3(256), 0, f->st, f->at<double>(f->L.lpart), B * G,
                       (double)B, lam, f->at<double>(f->L.lres));
    return hipGetLastError();
}

hipError_t adam(pr_fno* f, double lr, int step) {
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
    const long long n = f->pi.total;
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 256)), dim3(256), 0, f->st, f->params, f->grads,
                       f->at(f->L.m), f->at(f->L.v), n, (float)lr, (float)b1, (float)b2,
                       (float)eps, (float)c1, (float)c2);
    f->stacked = false;
    return hipGetLastError();
}

bool valid_prec(int p) { return p == PR_FNO_FP32 || p == PR_FNO_BF16; }

}  // namespace

// Used by the solver's FNO coarse propagator (solver.hip).
namespace pr {
namespace fno {
hipError_t infer(pr_fno* f, const float* w, const float* meta, int B, float* out, hipStream_t st) {
    hipStream_t keep = f->st;
    f->st = st;
    hipError_t e = forward(f, w, GG, meta, nullptr, 0, B, f->infer_prec == PR_FNO_BF16, out);
    f->st = keep;
    return e;
}
int max_batch(const pr_fno* f) { return f->Bm; }
double out_scale(const pr_fno* f) { return f->out_scale; }
int base(const pr_fno* f) { return f->base; }

hipError_t gemm_f64(const double* A, long long ars, long long acs, const double* B, long long brs,
                    long long bcs, double* Cp, long long crs, int M, int N, int K, double beta,
                    hipStream_t st) {
    Gemm<double> q(M, N, K);
    q.A(A, ars, acs).B(B, brs, bcs).Cm(Cp, crs, 1).scale(1.0, beta);
    return run(q, false, st);
}
}  // namespace fno
}  // namespace pr

extern "C" {

uint64_t pr_fno_param_count(void) { return (uint64_t)ParamIndex().total; }

uint64_t pr_fno_workspace_bytes(int32_t max_batch) {
    if (max_batch < 1 || max_batch > PR_FNO_MAX_BATCH) return 0;
    return make_layout(max_batch).total;
}

pr_status pr_fno_create(const pr_fno_config* cfg, void* ws, uint64_t bytes, void* stream,
                        pr_fno** out) {
    if (!out) return PR_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->max_batch < 1 || cfg->max_batch > PR_FNO_MAX_BATCH) return PR_EINVAL;
    if (!valid_prec(cfg->precision)) return PR_EINVAL;
    if (!(cfg->out_scale > 0.0) || !std::isfinite(cfg->out_scale)) return PR_EINVAL;
    if (cfg->base < PR_FNO_BASE_ZERO || cfg->base > PR_FNO_BASE_FINE_LOD) return PR_EINVAL;
    const Layout L = make_layout(cfg->max_batch);
    if (!ws || bytes < L.total) return PR_ENOMEM;
    if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return PR_EINVAL;
    pr_fno* f = new (std::nothrow) pr_fno();
    if (!f) return PR_ENOMEM;
    f->Bm = cfg->max_batch;
    f->st = reinterpret_cast<hipStream_t>(stream);
    f->ws = static_cast<char*>(ws);
    f->L = L;
    f->params = f->at(L.params);
    f->grads = f->at(L.grads);
    f->infer_prec = cfg->precision;
    f->out_scale = cfg->out_scale;
    f->base = cfg->base;
    f->skip = cfg->base == PR_FNO_BASE_IDENTITY ? 1.0 : 0.0;
    float* tabs = f->at(L.tabs);
    f->EyF = tabs;
    f->ExF = f->EyF + 2 * MX * G;
    f->ExI = f->ExF + 2 * NKX * 2 * G;
    f->EyI = f->ExI + 2 * G * 2 * NKX;
    f->ones = f->at(L.ones);
    const std::vector<float> t = make_tables();
    long long offs[2 * NL];
    for (int l = 0; l < NL; ++l) { offs[2 * l] = f->pi.Rr[l]; offs[2 * l + 1] = f->pi.Ri[l]; }
    const float one = 1.0f;
    hipError_t e = hipMemcpyAsync(tabs, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice, f->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f->at(L.offs), offs, sizeof(offs), hipMemcpyHostToDevice, f->st);
    if (e == hipSuccess) e = hipMemcpyAsync(f->ones, &one, sizeof(float), hipMemcpyHostToDevice, f->st);
    if (e == hipSuccess) e = hipMemsetAsync(f->at(L.m), 0, (L.v - L.m) + f->pi.total * 4, f->st);
    if (e == hipSuccess) e = hipStreamSynchronize(f->st);
    if (e != hipSuccess) { delete f; return PR_EDEVICE; }
    *out = f;
    return PR_OK;
}

pr_status pr_fno_set_params(pr_fno* f, const float* src) {
    if (!f || !src) return PR_EINVAL;
    FNO_HIP(hipMemcpyAsync(f->params, src, f->pi.total * sizeof(float), hipMemcpyDeviceToDevice, f->st));
    FNO_HIP(hipMemsetAsync(f->at(f->L.m), 0, (f->L.v - f->L.m) + f->pi.total * 4, f->st));
    f->stacked = false;
    f->fwd_batch = 0;
    return PR_OK;
}

pr_status pr_fno_get_params(pr_fno* f, float* dst) {
    if (!f || !dst) return PR_EINVAL;
    FNO_HIP(hipMemcpyAsync(dst, f->params, f->pi.total * sizeof(float), hipMemcpyDeviceToDevice, f->st));
    return PR_OK;
}

pr_status pr_fno_get_grads(pr_fno* f, float* dst) {
    if (!f || !dst) return PR_EINVAL;
    FNO_HIP(hipMemcpyAsync(dst, f->grads, f->pi.total * sizeof(float), hipMemcpyDeviceToDevice, f->st));
    return PR_OK;
}

pr_status pr_fno_forward(pr_fno* f, const float* w, const float* meta, int32_t batch,
                         int32_t precision, float* out) {
    if (!f) return PR_EINVAL;
    if (!w || !meta || !out || batch < 1 || batch > f->Bm) return fail(f, PR_EINVAL, "bad forward arguments");
    if (!valid_prec(precision)) return fail(f, PR_EINVAL, "unknown precision");
    FNO_HIP(forward(f, w, GG, meta, nullptr, 0, batch, precision == PR_FNO_BF16, out));
    f->fwd_batch = batch;
    f->fwd_prec = precision;
    return PR_OK;
}

pr_status pr_fno_backward(pr_fno* f, const float* gout) {
    if (!f) return PR_EINVAL;
    if (!gout) return fail(f, PR_EINVAL, "null gradient");
    if (f->fwd_batch < 1) return fail(f, PR_EINVAL, "backward without a preceding forward");
    FNO_HIP(backward(f, gout, f->fwd_batch, f->fwd_prec == PR_FNO_BF16));
    return PR_OK;
}

pr_status pr_fno_loss(pr_fno* f, const float* pred, const float* pairs, const float* meta,
                      int32_t batch, double scale, double dT, double lam, float* gpred,
                      double* host_loss) {
    if (!f) return PR_EINVAL;
    if (!pred || !pairs || !meta || batch < 1 || batch > f->Bm || !(dT > 0.0) || !(lam >= 0.0))
        return fail(f, PR_EINVAL, "bad loss arguments");
    FNO_HIP(loss(f, pred, pairs, meta, nullptr, 0, batch, scale, dT, lam));
    if (gpred)
        FNO_HIP(hipMemcpyAsync(gpred, f->at(f->L.gpred), (size_t)batch * GG * sizeof(float),
                               hipMemcpyDeviceToDevice, f->st));
    if (host_loss) {
        FNO_HIP(hipMemcpyAsync(host_loss, f->at<double>(f->L.lres), 3 * sizeof(double),
                               hipMemcpyDeviceToHost, f->st));
        FNO_HIP(hipStreamSynchronize(f->st));
    }
    return PR_OK;
}

pr_status pr_fno_adam(pr_fno* f, double lr, int32_t step) {
    if (!f) return PR_EINVAL;
    if (step < 1 || !(lr >= 0.0)) return fail(f, PR_EINVAL, "bad Adam arguments");
    FNO_HIP(adam(f, lr, step));
    return PR_OK;
}

pr_status pr_fno_train_step(pr_fno* f, const float* pairs, const float* meta, int64_t n_pairs,
                            const int32_t* idx, int32_t batch, double dT, double lam, double lr, int32_t step,
                            int32_t precision, double* host_loss) {
    if (!f) return PR_EINVAL;
    if (!pairs || !meta || !idx || n_pairs < 1 || n_pairs > INT32_MAX || batch < 1 ||
        batch > f->Bm || !(dT > 0.0) || !(lam >= 0.0) ||
        step < 1 || !(lr >= 0.0))
        return fail(f, PR_EINVAL, "bad train-step arguments");
    if (!valid_prec(precision)) return fail(f, PR_EINVAL, "unknown precision");
    const bool mf = precision == PR_FNO_BF16;
    float* out = f->at(f->L.out);
    FNO_HIP(forward(f, pairs, 4LL * GG, meta, idx, (int)n_pairs, batch, mf, out));
    FNO_HIP(loss(f, out, pairs, meta, idx, (int)n_pairs, batch, f->out_scale, dT, lam));
    FNO_HIP(backward(f, f->at(f->L.gpred), batch, mf));
    FNO_HIP(adam(f, lr, step));
    f->fwd_batch = 0;
    if (host_loss) {
        FNO_HIP(hipMemcpyAsync(host_loss, f->at<double>(f->L.lres), 3 * sizeof(double),
                               hipMemcpyDeviceToHost, f->st));
        FNO_HIP(hipStreamSynchronize(f->st));
    }
    return PR_OK;
}

// ---------------------------------------------------------------------------
// Weight file (pr_fno_save / pr_fno_load / pr_fno_check_file).  Little-endian:
//   [0, 8)   magic "PRFNOW01"
//   [8, 12)  uint32 version (1)            [12, 16) uint32 header bytes (96)
//   [16, 44) int32 grid, width, modes, layers, c_in, lift, proj
//   [44, 48) int32 base                    [48, 52) int32 inference precision
//   [52, 56) int32 0                       [56, 64) double out_scale
//   [64, 72) uint64 parameter count        [72, 80) uint64 training-config hash
//   [80, 88) uint64 FNV-1a 64 of bytes [0, 80) followed by the parameters
//   [88, 96) uint64 0
//   [96, ..) parameter count FP32 master weights (the flat vector of set_params)
// ---------------------------------------------------------------------------
namespace {

constexpr char kFileMagic[8] = {'P', 'R', 'F', 'N', 'O', 'W', '0', '1'};
constexpr uint32_t kFileVersion = 1;
constexpr uint32_t kFileHeader = 96;

uint64_t fnv1a(uint64_t h, const unsigned char* p, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

const int32_t kArch[7] = {PR_FNO_GRID, PR_FNO_WIDTH, PR_FNO_MODES, PR_FNO_LAYERS,
                          PR_FNO_CIN, PR_FNO_LIFT, PR_FNO_PROJ};

// Reads and validates a weight file; params receives the weights when non-null.
pr_status read_weight_file(const char* path, pr_fno_file_info* info, std::vector<float>* params,
                           std::string* why) {
    auto bad = [&](const std::string& m) { if (why) *why = m; return PR_EMODEL; };
    if (!path) return bad("null path");
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return bad(std::string("cannot open ") + path);
    unsigned char hdr[kFileHeader];
    const size_t got = std::fread(hdr, 1, kFileHeader, fp);
    if (got != kFileHeader) { std::fclose(fp); return bad("truncated header"); }
    if (std::memcmp(hdr, kFileMagic, 8) != 0) { std::fclose(fp); return bad("not an FNO weight file (magic)"); }
    uint32_t ver, hb;
    int32_t arch[7], base, prec;
    double scale;
    uint64_t count, thash, sum;
    std::memcpy(&ver, hdr + 8, 4);
    std::memcpy(&hb, hdr + 12, 4);
    std::memcpy(arch, hdr + 16, 28);
    std::memcpy(&base, hdr + 44, 4);
    std::memcpy(&prec, hdr + 48, 4);
    std::memcpy(&scale, hdr + 56, 8);
    std::memcpy(&count, hdr + 64, 8);
    std::memcpy(&thash, hdr + 72, 8);
    std::memcpy(&sum, hdr + 80, 8);
    if (ver != kFileVersion || hb != kFileHeader) { std::fclose(fp); return bad("unsupported file version"); }
    if (std::memcmp(arch, kArch, sizeof(kArch)) != 0) { std::fclose(fp); return bad("architecture differs from this library's"); }
    if (count != (uint64_t)ParamIndex().total) { std::fclose(fp); return bad("parameter count differs"); }
    if (base < PR_FNO_BASE_ZERO || base > PR_FNO_BASE_FINE_LOD || !valid_prec(prec) ||
        !(scale > 0.0) || !std::isfinite(scale)) {
        std::fclose(fp);
        return bad("invalid header field");
    }
    std::vector<float> w(count);
    const size_t gw = std::fread(w.data(), sizeof(float), count, fp);
    unsigned char extra;
    const bool trailing = std::fread(&extra, 1, 1, fp) == 1;
    std::fclose(fp);
    if (gw != count) return bad("truncated parameters");
    if (trailing) return bad("trailing bytes after the parameters");
    uint64_t h = fnv1a(1469598103934665603ull, hdr, 80);
    h = fnv1a(h, reinterpret_cast<const unsigned char*>(w.data()), count * sizeof(float));
    if (h != sum) return bad("checksum mismatch");
    for (float v : w)
        if (!std::isfinite(v)) return bad("non-finite parameter");
    if (info) {
        info->version = ver;
        info->base = base;
        info->precision = prec;
        info->pad_ = 0;
        info->out_scale = scale;
        info->param_count = count;
        info->train_hash = thash;
    }
    if (params) params->swap(w);
    return PR_OK;
}

}  // namespace

pr_status pr_fno_check_file(const char* path, pr_fno_file_info* info) {
    return read_weight_file(path, info, nullptr, nullptr);
}

pr_status pr_fno_save(pr_fno* f, const char* path, uint64_t train_hash) {
    if (!f || !path) return PR_EINVAL;
    const uint64_t count = (uint64_t)f->pi.total;
    std::vector<float> w(count);
    FNO_HIP(hipMemcpyAsync(w.data(), f->params, count * sizeof(float), hipMemcpyDeviceToHost, f->st));
    FNO_HIP(hipStreamSynchronize(f->st));
    unsigned char hdr[kFileHeader];
    std::memset(hdr, 0, sizeof(hdr));
    const int32_t base = f->base, prec = f->infer_prec;
    const double scale = f->out_scale;
    std::memcpy(hdr, kFileMagic, 8);
    std::memcpy(hdr + 8, &kFileVersion, 4);
    std::memcpy(hdr + 12, &kFileHeader, 4);
    std::memcpy(hdr + 16, kArch, 28);
    std::memcpy(hdr + 44, &base, 4);
    std::memcpy(hdr + 48, &prec, 4);
    std::memcpy(hdr + 56, &scale, 8);
    std::memcpy(hdr + 64, &count, 8);
    std::memcpy(hdr + 72, &train_hash, 8);
    uint64_t h = fnv1a(1469598103934665603ull, hdr, 80);
    h = fnv1a(h, reinterpret_cast<const unsigned char*>(w.data()), count * sizeof(float));
    std::memcpy(hdr + 80, &h, 8);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return fail(f, PR_EMODEL, "cannot create " + tmp);
    bool ok = std::fwrite(hdr, 1, kFileHeader, fp) == kFileHeader &&
              std::fwrite(w.data(), sizeof(float), count, fp) == count;
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(f, PR_EMODEL, std::string("cannot write ") + path);
    }
    return PR_OK;
}

pr_status pr_fno_load(pr_fno* f, const char* path, pr_fno_file_info* info) {
    if (!f || !path) return PR_EINVAL;
    pr_fno_file_info fi{};
    std::vector<float> w;
    std::string why;
    const pr_status st = read_weight_file(path, &fi, &w, &why);
    if (st != PR_OK) return fail(f, st, why);
    if (fi.base != f->base || fi.out_scale != f->out_scale)
        return fail(f, PR_EMODEL, "the file's base or out_scale differs from the handle's configuration");
    FNO_HIP(hipMemcpyAsync(f->params, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice, f->st));
    FNO_HIP(hipMemsetAsync(f->at(f->L.m), 0, (f->L.v - f->L.m) + f->pi.total * 4, f->st));
    FNO_HIP(hipStreamSynchronize(f->st));
    f->stacked = false;
    f->fwd_batch = 0;
    if (info) *info = fi;
    return PR_OK;
}

pr_status pr_fno_destroy(pr_fno* f) {
    if (!f) return PR_EINVAL;
    (void)hipStreamSynchronize(f->st);
    delete f;
    return PR_OK;
}

const char* pr_fno_last_error(const pr_fno* f) { return f ? f->err.c_str() : "null handle"; }

}  // extern "C"
