// Streaming of the per-cell step-2 operators M2 through LDS, shared by the
// reconstruction kernel and its reverse: one workgroup handles one tile of
// kRecCells cells with one wavefront per conservative component, and the
// tile's 144 x 64 operator entries (contiguous in memory) are staged in
// kM2Chunk-row chunks that all five wavefronts read.
#pragma once

#include "gks_internal.h"

namespace gks {

constexpr int kRecCells = kM2Tile;
constexpr int kRecThreads = 5 * kRecCells;
constexpr int kM2Chunk = 48;                 // three output rows of 16 operator rows
constexpr int kM2Chunks = kM2Rows / kM2Chunk;
static_assert(kM2Chunk * kM2Chunks == kM2Rows && kM2Chunk % 16 == 0, "M2 chunking");

// one chunk of a tile as 16-byte vectors, spread over the block
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename R>
struct M2Chunk {
    static constexpr int kVec = kM2Chunk * kRecCells * (int)sizeof(R) / 16;
    static constexpr int kPer = (kVec + kRecThreads - 1) / kRecThreads;
    u32x4 v[kPer];
    __device__ __forceinline__ void load(const R *tile, int chunk)
    {
        const u32x4 *src = reinterpret_cast<const u32x4 *>(tile + (size_t)chunk * kM2Chunk * kRecCells);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int t = threadIdx.x + j * kRecThreads;
            if (t < kVec) v[j] = src[t];
        }
    }
    __device__ __forceinline__ void store(R *lds) const
    {
        u32x4 *dst = reinterpret_cast<u32x4 *>(lds);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int t = threadIdx.x + j * kRecThreads;
            if (t < kVec) dst[t] = v[j];
        }
    }
};

}  // namespace gks
