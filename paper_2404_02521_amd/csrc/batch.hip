// batch.hip -- the temporally blocked explicit step (S steps of Eq. (fd) per
// launch, body in step_tb.hpp) over the slices of several independent solvers
// in one launch: the ragged per-tick fine launch of the serving loop.  Each
// entry keeps the launch geometry of its own solver; workgroups are assigned to
// entries in order, so every workgroup belongs to exactly one entry and runs
// the same code as the single-solver kernel (the result is bitwise the same).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"
#include "step_tb.hpp"

namespace pr {

template <int MODE, bool CHEAP, typename T, int S, int PF>
__global__ __launch_bounds__(kBlock) void k_fine_tb_batch(const TbBatch b) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    // the entry of this workgroup: uniform, held in scalar registers
    int r = 0;
#pragma unroll
    for (int e = 1; e < kTbBatchMax; ++e)
        if (e < b.n && bid >= b.e[e].block0) r = e;
    const int wid = (bid - b.e[r].block0) * (kBlock / kWave) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    tb_body<MODE, CHEAP, T, S, PF>(static_cast<const T*>(b.e[r].in), b.e[r].lb,
                                   static_cast<T*>(b.e[r].out), static_cast<const T*>(b.e[r].wt),
                                   b.e[r].a, wid);
}

namespace {

// rows in flight per wavefront, as in the single-solver launch
constexpr int kPf = 3;

template <int MODE, typename T, int S>
void launch_s(const TbBatch& b, hipStream_t st) {
    hipLaunchKernelGGL((k_fine_tb_batch<MODE, true, T, S, kPf>), dim3(b.nblocks), dim3(kBlock), 0,
                       st, b);
}

template <int MODE, typename T>
hipError_t launch_t(const TbBatch& b, int S, hipStream_t st) {
    switch (S) {
        case 1: launch_s<MODE, T, 1>(b, st); break;
        case 2: launch_s<MODE, T, 2>(b, st); break;
        case 3: launch_s<MODE, T, 3>(b, st); break;
        case 4: launch_s<MODE, T, 4>(b, st); break;
        case 5: launch_s<MODE, T, 5>(b, st); break;
        case 6: launch_s<MODE, T, 6>(b, st); break;
        case 7: launch_s<MODE, T, 7>(b, st); break;
        case 8: launch_s<MODE, T, 8>(b, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

// S fused steps for every entry of b (FP32 increment form when fp32, else FP64
// states).  Solvers whose ring takes the out-of-line closed forms (PR_BC_EXACT)
// are not batched: that call takes the address of the entry's arguments, which
// would copy the whole table to scratch memory; they keep their own launches.
// Entry e's workgroups start at b.e[e].block0, which the caller sets to the
// running sum of ceil(count * nchunks * nstrips / 4) over the entries before it.
hipError_t launch_fine_tb_batch(const TbBatch& b, bool fp32, int S, hipStream_t st) {
    if (b.n < 1 || b.n > kTbBatchMax || b.nblocks < 1) return hipErrorInvalidValue;
    int blocks = 0;
    for (int e = 0; e < b.n; ++e) {
        const StepArgs& a = b.e[e].a;
        if (a.rows > kTbMaxRows || b.e[e].block0 != blocks) return hipErrorInvalidValue;
        if (fp32 != (b.e[e].lb != nullptr) || a.bc.kind == 2) return hipErrorInvalidValue;
        blocks += (a.count * a.nchunks * a.nstrips + kBlock / kWave - 1) / (kBlock / kWave);
    }
    if (blocks != b.nblocks) return hipErrorInvalidValue;
    return fp32 ? launch_t<MODE_INCR, float>(b, S, st) : launch_t<MODE_DIRECT, double>(b, S, st);
}

}  // namespace pr
