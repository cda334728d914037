// Device helpers shared by the HIP translation units of libgks.
#pragma once

#include <hip/hip_runtime.h>

namespace gks {

__device__ __forceinline__ int gid() { return blockIdx.x * blockDim.x + threadIdx.x; }

// Workgroups go to the chip's 8 XCDs round-robin (workgroup b to XCD b mod 8),
// and each XCD has its own L2.  The kernels that gather neighbours renumber
// their workgroups so that each XCD takes one contiguous range of cells or
// faces: ranges adjacent in the space-filling order, whose neighbour gathers
// then hit the L2 that loaded them.  A bijection of [0, gridDim.x).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q = nb / kXcds, r = nb % kXcds, x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}
__device__ __forceinline__ int xcd_gid() { return xcd_block() * blockDim.x + threadIdx.x; }

}  // namespace gks
