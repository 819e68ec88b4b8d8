// merf_ingest.hip -- device-side scene ingest: packing of stored blocks into
// apron bricks, and max-pooling of a binary occupancy mask into the coarser
// levels of the empty-space hierarchy (Sec. 6 builds its occupancy grids by
// max-pooling the full-resolution mask; Sec. 5.3 stores the grid in a
// block-sparse format).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "merf_device.h"

namespace merf {

namespace {

constexpr int kBrickVoxels = kBrick * kBrick * kBrick;   // 729

// One thread per voxel of a brick: copy the 8 channels of voxel
// (8 b + l) from its stored block, or zeros for an absent block, outside the
// grid, or for the shared zero brick (slot == nbricks).
__global__ void k_pack_bricks(const uint8_t *__restrict__ blocks, const int32_t *__restrict__ block_index,
                              const int32_t *__restrict__ brick_pos, int nbricks, int L, int nbl,
                              uint8_t *__restrict__ bricks) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)(nbricks + 1) * kBrickVoxels;
    if (gid >= total) return;
    const int slot = (int)(gid / kBrickVoxels), v = (int)(gid % kBrickVoxels);
    uint2 val = make_uint2(0u, 0u);
    if (slot < nbricks) {
        const int pos = brick_pos[slot];
        const int bx = pos & 1023, by = (pos >> 10) & 1023, bz = pos >> 20;
        const int lz = v / (kBrick * kBrick), ly = (v / kBrick) % kBrick, lx = v % kBrick;
        const int x = bx * kBlock + lx, y = by * kBlock + ly, z = bz * kBlock + lz;
        if (x < L && y < L && z < L) {
            const int src = block_index[((size_t)(z / kBlock) * nbl + (y / kBlock)) * nbl + (x / kBlock)];
            if (src >= 0) {
                const size_t off = ((((size_t)src * kBlock + (z % kBlock)) * kBlock + (y % kBlock)) * kBlock +
                                    (x % kBlock)) * kChannels;
                val = *reinterpret_cast<const uint2 *>(blocks + off);
            }
        }
    }
    *reinterpret_cast<uint2 *>(bricks + (size_t)slot * kBrickBytes + (size_t)v * kChannels) = val;
}

// One thread per output cell: 1 if any of the f^3 input cells is nonzero.
__global__ void k_maxpool(const uint8_t *__restrict__ in, int rin, int f, uint8_t *__restrict__ out) {
    const int rout = rin / f;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)rout * rout * rout) return;
    const int x = (int)(gid % rout), y = (int)((gid / rout) % rout), z = (int)(gid / ((int64_t)rout * rout));
    uint32_t any = 0;
    for (int dz = 0; dz < f && !any; ++dz)
        for (int dy = 0; dy < f && !any; ++dy) {
            const uint8_t *row = in + (((size_t)z * f + dz) * rin + ((size_t)y * f + dy)) * rin + (size_t)x * f;
            for (int dx = 0; dx < f; ++dx) any |= row[dx];
        }
    out[gid] = any ? 1 : 0;
}

}  // namespace

hipError_t launch_pack_bricks(const uint8_t *blocks, const int32_t *block_index, const int32_t *brick_pos,
                              int nbricks, int L, uint8_t *bricks, hipStream_t stream) {
    const int64_t total = (int64_t)(nbricks + 1) * kBrickVoxels;
    const int64_t grid = (total + 255) / 256;
    hipLaunchKernelGGL(k_pack_bricks, dim3((unsigned)grid), dim3(256), 0, stream, blocks, block_index, brick_pos,
                       nbricks, L, L / kBlock, bricks);
    return hipGetLastError();
}

hipError_t launch_maxpool(const uint8_t *in, int rin, int f, uint8_t *out, hipStream_t stream) {
    const int64_t rout = rin / f, n = rout * rout * rout;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_maxpool, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, rin, f, out);
    return hipGetLastError();
}

}  // namespace merf
