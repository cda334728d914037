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

// No-slip walls (Sec. 4.4): the prescribed value of component q (1-3
// momentum, 4 energy) at a wall point is rho times this factor, rho the
// density reconstructed there: U_wall, or |U_wall|^2/2 + T_wall/(gamma - 1)
// with T = p / rho.
template <typename R>
__device__ __forceinline__ R wall_factor(int q, const R u[3], R gamma, R Tw)
{
    if (q <= 3) return u[q - 1];
    return R(0.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + Tw / (gamma - R(1));
}
template <typename R>
__device__ __forceinline__ R wall_value(int q, R rho, const R u[3], R gamma, R Tw)
{
    return rho * wall_factor(q, u, gamma, Tw);
}

// a cell polynomial about its centroid, coefficients (c0, G, Hxx, Hyy, Hzz,
// Hxy, Hxz, Hyz), at offset r; and the coefficients' weights at r
template <typename R>
__device__ __forceinline__ void quad_basis(const R r[3], R e[10])
{
    e[0] = R(1);
    e[1] = r[0];
    e[2] = r[1];
    e[3] = r[2];
    e[4] = R(0.5) * r[0] * r[0];
    e[5] = R(0.5) * r[1] * r[1];
    e[6] = R(0.5) * r[2] * r[2];
    e[7] = r[0] * r[1];
    e[8] = r[0] * r[2];
    e[9] = r[1] * r[2];
}
template <typename R>
__device__ __forceinline__ R quad_value(const R c[10], const R r[3])
{
    return c[0] + c[1] * r[0] + c[2] * r[1] + c[3] * r[2] +
           R(0.5) * (c[4] * r[0] * r[0] + c[5] * r[1] * r[1] + c[6] * r[2] * r[2]) + c[7] * r[0] * r[1] +
           c[8] * r[0] * r[2] + c[9] * r[1] * r[2];
}

}  // namespace gks
