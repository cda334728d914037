// Conservation sums that allocate nothing: the variant of gks_conservation_sums
// behind gks_conservation_sums_noalloc, for callers that cannot allocate
// device memory or synchronise (code under HIP graph capture, tight serving
// loops).  Its per-block partial sums live in a fixed device array of this
// translation unit instead of the context's workspace, and the result is
// written to a caller's device pointer without a host synchronisation.
//
// The array is one per device and shared by every call on that device: calls
// that overlap on one GPU race.  Every call overwrites all the partials it
// reads (one per block and component), so nothing needs clearing between
// calls.
#include "gks_device.h"
#include "gks_internal.h"

#include <mutex>

namespace gks {

// per-block partials: 5 components x kNoAllocMaxBlocks blocks of kBlock cells
// (2.5 MiB per device, held until the process ends)
constexpr int kNoAllocMaxBlocks = 65536;
constexpr size_t kNoAllocScratchDoubles = (size_t)5 * kNoAllocMaxBlocks;

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

// device address of `scratch` per device, from hipGetSymbolAddress (the
// array's name is not a device address in host code)
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
double *scratch_ptr[kMaxDevices] = {};

__device__ __forceinline__ double block_sum(double v, double *sm)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sm[k];  // fixed order
    __syncthreads();
    return t;
}

// one thread per cell: |Omega_i| W_i summed per block, in a fixed order
__global__ __launch_bounds__(kBlock) void noalloc_sums_pass1(DevMesh m, DevState s, double *part)
{
    __shared__ double sm[kBlock / 64];
    const int n = m.nc, i = gid();
    const double v = i < n ? m.geoD[(size_t)G_VOL * n + i] : 0.0;
    for (int q = 0; q < 5; ++q) {
        const double t = block_sum(i < n ? v * s.W[(size_t)q * n + i] : 0.0, sm);
        if (threadIdx.x == 0) part[(size_t)q * gridDim.x + blockIdx.x] = t;
    }
}

// one block: the partials of each component in a fixed order
__global__ __launch_bounds__(kBlock) void noalloc_sums_pass2(const double *part, int nblocks, double *out)
{
    __shared__ double sm[kBlock / 64];
    for (int q = 0; q < 5; ++q) {
        double t = 0.0;
        for (int k = threadIdx.x; k < nblocks; k += blockDim.x) t += part[(size_t)q * nblocks + k];
        t = block_sum(t, sm);
        if (threadIdx.x == 0) out[q] = t;
    }
}

}  // namespace

int64_t noalloc_max_cells() { return (int64_t)kNoAllocMaxBlocks * kBlock; }

hipError_t launch_sums_noalloc(const DevMesh &m, const DevState &s, double *out, hipStream_t st)
{
    if ((int64_t)m.nc > noalloc_max_cells() || m.nc <= 0) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    double *ptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mutex);
        if (!scratch_ptr[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            scratch_ptr[dev] = static_cast<double *>(p);
        }
        ptr = scratch_ptr[dev];
    }
    const int blocks = (m.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(noalloc_sums_pass1, dim3(blocks), dim3(kBlock), 0, st, m, s, ptr);
    hipLaunchKernelGGL(noalloc_sums_pass2, dim3(1), dim3(kBlock), 0, st, ptr, blocks, out);
    return hipGetLastError();
}

}  // namespace gks
