// merf_ingest.hip -- device-side scene ingest: packing of stored blocks into
// apron bricks, and max-pooling of a binary occupancy mask into the coarser
// levels of the empty-space hierarchy (Sec. 6 builds its occupancy grids by
// max-pooling the full-resolution mask; Sec. 5.3 stores the grid in a
// block-sparse format); and the empty-space distance grid the renderer skips
// with, derived from the occupancy levels.
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

// Empty-space distance grid, step 1: the cell of the finest level is
// occupied when every level marks the cell containing it (the levels nest,
// so each finest cell lies in one cell of every level).  Output is the seed
// of the distance transform: 0 for occupied, 255 for empty.
__global__ void k_occ_combine(const OccLevels lv, uint8_t *__restrict__ out) {
    const int rf = lv.res[lv.n - 1];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)rf * rf * rf) return;
    const int x = (int)(gid % rf), y = (int)((gid / rf) % rf), z = (int)(gid / ((int64_t)rf * rf));
    bool occ = true;
    for (int l = 0; l < lv.n && occ; ++l) {
        const int r = lv.res[l], k = rf / r;
        occ = lv.occ[l][((size_t)(z / k) * r + (y / k)) * r + (x / k)] != 0;
    }
    out[gid] = occ ? 0 : 255;
}

// Step 2, one pass per axis: the Chebyshev (L-infinity) distance to the
// nearest occupied cell is separable,
//   d(c) = min over cells t of the line through c along the axis of
//          max(|c_a - t_a|, d_prev(t)),
// starting from the seed and applied along x, then y, then z; values are
// capped at 255 (a cap only shortens skips).  One workgroup per line, the
// line staged in LDS; each cell scans outwards and stops once the offset
// reaches its best distance.
__global__ void k_dist_axis(const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int r, int axis) {
    __shared__ uint8_t line[kMaxDistRes];
    const int64_t lid = blockIdx.x;
    int64_t base, stride;
    if (axis == 0) { base = lid * r; stride = 1; }
    else if (axis == 1) { base = (lid / r) * r * r + lid % r; stride = r; }
    else { base = lid; stride = (int64_t)r * r; }
    for (int c = (int)threadIdx.x; c < r; c += (int)blockDim.x) line[c] = in[base + c * stride];
    __syncthreads();
    for (int c = (int)threadIdx.x; c < r; c += (int)blockDim.x) {
        int best = line[c];
        for (int dd = 1; dd < best; ++dd) {
            if (c - dd >= 0) best = min(best, max(dd, (int)line[c - dd]));
            if (c + dd < r) best = min(best, max(dd, (int)line[c + dd]));
        }
        out[base + c * stride] = (uint8_t)best;
    }
}

// Forward empty extents, step 1: inclusive prefix sums of the occupancy
// (seed 0 = occupied) along x, then y, then z -- one thread per line.
__global__ void k_occ_prefix_x(const uint8_t *__restrict__ seed, int32_t *__restrict__ sat, int r) {
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= (int64_t)r * r) return;
    int32_t acc = 0;
    for (int x = 0; x < r; ++x) {
        acc += seed[line * r + x] == 0 ? 1 : 0;
        sat[line * r + x] = acc;
    }
}

__global__ void k_prefix_axis(int32_t *__restrict__ sat, int r, int axis) {
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= (int64_t)r * r) return;
    const int64_t base = axis == 1 ? (line / r) * r * r + line % r : line;   // y: (z, x) lines; z: (y, x)
    const int64_t stride = axis == 1 ? (int64_t)r : (int64_t)r * r;
    int32_t acc = 0;
    for (int i = 0; i < r; ++i) {
        acc += sat[base + i * stride];
        sat[base + i * stride] = acc;
    }
}

__device__ __forceinline__ int32_t sat_at(const int32_t *sat, int r, int x, int y, int z) {
    return (x < 0 || y < 0 || z < 0) ? 0 : sat[((int64_t)z * r + y) * r + x];
}

// Occupied cells in the box [x0, x1] x [y0, y1] x [z0, z1] (inclusive).
__device__ __forceinline__ int32_t box_count(const int32_t *sat, int r, int x0, int y0, int z0, int x1, int y1,
                                             int z1) {
    return sat_at(sat, r, x1, y1, z1) - sat_at(sat, r, x0 - 1, y1, z1) - sat_at(sat, r, x1, y0 - 1, z1) -
           sat_at(sat, r, x1, y1, z0 - 1) + sat_at(sat, r, x0 - 1, y0 - 1, z1) + sat_at(sat, r, x0 - 1, y1, z0 - 1) +
           sat_at(sat, r, x1, y0 - 1, z0 - 1) - sat_at(sat, r, x0 - 1, y0 - 1, z0 - 1);
}

// Step 2: for each cell and each octant o (bit 0: -x, bit 1: -y, bit 2: -z)
// the largest k <= 255 such that the cube of k cells on a side with a corner
// at the cell and extending in the octant's directions holds no occupied
// cell (cells outside the grid are empty); 0 for an occupied cell.  Found by
// bisection, since the count only grows with k.
__global__ void k_octant_extent(const int32_t *__restrict__ sat, int r, uint8_t *__restrict__ out) {
    const int64_t n = (int64_t)r * r * r;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 8 * n) return;
    const int o = (int)(gid / n);
    const int64_t cell = gid % n;
    const int x = (int)(cell % r), y = (int)((cell / r) % r), z = (int)(cell / ((int64_t)r * r));
    if (box_count(sat, r, x, y, z, x, y, z) != 0) {
        out[gid] = 0;
        return;
    }
    auto empty = [&](int k) {
        const int x0 = (o & 1) ? max(x - k + 1, 0) : x, x1 = (o & 1) ? x : min(x + k - 1, r - 1);
        const int y0 = (o & 2) ? max(y - k + 1, 0) : y, y1 = (o & 2) ? y : min(y + k - 1, r - 1);
        const int z0 = (o & 4) ? max(z - k + 1, 0) : z, z1 = (o & 4) ? z : min(z + k - 1, r - 1);
        return box_count(sat, r, x0, y0, z0, x1, y1, z1) == 0;
    };
    int lo = 1, hi = 255;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (empty(mid)) lo = mid;
        else hi = mid - 1;
    }
    out[gid] = (uint8_t)lo;
}

}  // namespace

hipError_t launch_octant_extents(const OccLevels &lv, uint8_t *seed, int32_t *sat, uint8_t *out, hipStream_t stream) {
    const int r = lv.res[lv.n - 1];
    const int64_t n = (int64_t)r * r * r;
    if (n <= 0 || r > kMaxDistRes) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_occ_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, lv, seed);
    const unsigned lines = (unsigned)(((int64_t)r * r + 255) / 256);
    hipLaunchKernelGGL(k_occ_prefix_x, dim3(lines), dim3(256), 0, stream, seed, sat, r);
    hipLaunchKernelGGL(k_prefix_axis, dim3(lines), dim3(256), 0, stream, sat, r, 1);
    hipLaunchKernelGGL(k_prefix_axis, dim3(lines), dim3(256), 0, stream, sat, r, 2);
    hipLaunchKernelGGL(k_octant_extent, dim3((unsigned)((8 * n + 255) / 256)), dim3(256), 0, stream, sat, r, out);
    return hipGetLastError();
}

hipError_t launch_pack_bricks(const uint8_t *blocks, const int32_t *block_index, const int32_t *brick_pos,
                              int nbricks, int L, uint8_t *bricks, hipStream_t stream) {
    const int64_t total = (int64_t)(nbricks + 1) * kBrickVoxels;
    const int64_t grid = (total + 255) / 256;
    hipLaunchKernelGGL(k_pack_bricks, dim3((unsigned)grid), dim3(256), 0, stream, blocks, block_index, brick_pos,
                       nbricks, L, L / kBlock, bricks);
    return hipGetLastError();
}

hipError_t launch_distance_grid(const OccLevels &lv, uint8_t *tmp0, uint8_t *tmp1, uint8_t *dist,
                                hipStream_t stream) {
    const int r = lv.res[lv.n - 1];
    const int64_t n = (int64_t)r * r * r;
    if (n <= 0 || r > kMaxDistRes) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_occ_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, lv, tmp0);
    const dim3 lines((unsigned)((int64_t)r * r)), block(256);
    hipLaunchKernelGGL(k_dist_axis, lines, block, 0, stream, tmp0, tmp1, r, 0);
    hipLaunchKernelGGL(k_dist_axis, lines, block, 0, stream, tmp1, tmp0, r, 1);
    hipLaunchKernelGGL(k_dist_axis, lines, block, 0, stream, tmp0, dist, r, 2);
    return hipGetLastError();
}

hipError_t launch_maxpool(const uint8_t *in, int rin, int f, uint8_t *out, hipStream_t stream) {
    const int64_t rout = rin / f, n = rout * rout * rout;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_maxpool, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, rin, f, out);
    return hipGetLastError();
}

}  // namespace merf
