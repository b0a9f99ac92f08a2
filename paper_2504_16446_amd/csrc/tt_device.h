// Device-only helpers shared by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>

namespace tt {

// Block-wide float64 sum; the result is valid in thread 0.  ws must hold
// blockDim.x / 64 doubles of shared memory.  Contains barriers: every thread
// of the block must call it.
__device__ __forceinline__ double block_sum(double v, double *ws)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += ws[i];
    __syncthreads();
    return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map the hardware block id to a logical id so that every XCD receives
// one contiguous range of logical blocks: neighbouring tiles, which share
// data, then share an L2.  A bijection on [0, nblk).
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int nblk)
{
    const int xcd = b % kNumXcd, idx = b / kNumXcd;
    const int base = nblk / kNumXcd, extra = nblk % kNumXcd;
    return xcd * base + min(xcd, extra) + idx;
}

}  // namespace tt
