// merf_device.h -- device-side scene layout and launch descriptors shared by
// the host API (merf_api.hip) and the kernels (merf_render.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace merf {

constexpr int kBlock = 8;                        // stored block edge (voxels)
constexpr int kBrick = kBlock + 1;               // block plus a one-voxel apron on the high side
constexpr int kChannels = 8;                     // density, rgb, 4 features
constexpr int kBrickBytes = kBrick * kBrick * kBrick * kChannels;   // 5832
constexpr int kMaxLevels = 4;
constexpr int kMlpIn = 34;
constexpr int kMlpHidden = 16;
constexpr int kMlpOut = 3;
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden * kMlpOut + kMlpOut;
constexpr int kTile = 8;                         // a wave renders an 8x8 pixel tile
constexpr int kCamsPerLaunch = 16;               // cameras carried in one launch's arguments
constexpr int kMaxDistRes = 1024;                // finest occupancy resolution (distance grid)
constexpr int kOctMaxRes = 256;                  // up to this r_f the grid has eight octant forms
// Tile order of a launch: a prepass estimates each tile's cost from
// kCostRays of its rays, and the tiles run heaviest first.  Launches of fewer
// than kOrderMinTiles tiles (1.5 waves per wave slot of the device; measured
// to gain nothing below) or more than kOrderMaxTiles (the work buffers' size;
// there the end of the launch is a small part of it) keep the plain order.
constexpr int kCostRays = 4;
constexpr int kCostKeys = kCostRays + 1;         // keys 0 .. 4: classes of estimated effort (k_tile_cost)
constexpr int kOrderMinTiles = 6144;
constexpr int kOrderMaxTiles = 1 << 17;

// Scene as laid out in device memory.
//   brick_index  int32 [(L/8)^3] z-major: brick slot; blocks whose brick would
//                hold only zeros point at a shared all-zero brick.
//   bricks       uint8 [n][9][9][9][8] (z, y, x, c): voxels 8b .. 8b+8 of each
//                axis, so the 2x2x2 trilinear footprint whose low corner lies
//                in block b is inside brick b.
//   planes       uint8 [3][R][R][8]: P_x[z][y], P_y[z][x], P_z[y][x].
//   occ[l]       uint8 [r^3] z-major, coarse to fine; each resolution divides
//                the next finer one.
//   dist         empty-space grid at the finest resolution r_f, z-major; 0
//                marks a cell occupied at every level.  Either (r_f <= 256)
//                eight octant grids uint8 [8][r_f^3]: octant o (bit 0: -x,
//                bit 1: -y, bit 2: -z) holds E, the largest cube of E cells
//                a side with a corner at the cell, extending in the
//                octant's directions, that is empty (capped at 255); or one
//                grid uint8 [r_f^3] of the Chebyshev distance D to the
//                nearest occupied cell, shared by all octants
//                (dist_oct_stride = 0): the same forward cube with E = D.
//   mlp          float32 W0[34][16] b0 W1[16][16] b1 W2[16][3] b2.
// A scene without a grid carries a stand-in grid (L = 8, one index entry
// pointing at the zero brick); a scene without planes carries all-zero 2x2
// stand-in planes (R = 2).  Stand-ins read code 0, and nsrc counts only the
// present sources (the fp16-feature path instead gives stand-in texels weight
// grid_w / planes_w = 0), so the kernels gather both kinds without branching.
struct DevScene {
    const int32_t *brick_index;
    const uint8_t *bricks;
    const uint8_t *planes;
    const uint8_t *occ[kMaxLevels];
    const uint8_t *dist;
    const float *mlp;
    int32_t L, R, nbl, occ_levels;
    int32_t occ_res[kMaxLevels];
    float occ_cell[kMaxLevels];                  // cell edge 4 / r of each level
    int32_t dist_res;                            // r_f
    float dist_cell;                             // 4 / r_f
    uint32_t dist_oct_stride;                    // bytes between octant grids (0: one shared grid)
    float m_density, m_feature;
    float nsrc;                                  // present sources: grid 1 + planes 3
    float grid_w, planes_w;                      // 1 for a present source, 0 for a stand-in
    int32_t res;                                 // finest present resolution max(L, R) of the scene
    // constants of the kernels, computed once on the host in float32 exactly
    // as the kernels would (uniform values the compiler would otherwise hold
    // in vector registers):
    float p_scale, p_off, p_max;                 // plane texel coordinate fma(p, R/4, R/2 - 1/2), max R - 1
    float g_scale, g_off, g_max;                 // grid voxel coordinate, the same with L
    float d_scale, d_off;                        // density: 2 m_d / 255 and -nsrc m_d
    float f_scale, f_off;                        // appearance: 2 m_f / 255 and -nsrc m_f
    float d_scale24, f_scale24;                  // d_scale, f_scale times 2^24 (codes read as b * 2^-24)
    float dist_scale, dist_off;                  // empty-space cell: fma(p, r_f/4, r_f/2)
};

struct DevCamera {
    float c2w[12];
    float fx, fy, cx, cy;
    float inv_fx, inv_fy;
    int32_t width, height, tiles_x, tile_start;  // tile_start: first tile of this camera in the launch
    float *out;                                  // device RGBA of this camera's first pixel (row-major)
};

struct RenderBatch {
    int32_t n_cams, total_tiles;
    float step, inv_step, t_min;
    int32_t delta_mode, mlp_prec, feat_prec, skip_mode;
    unsigned long long *stats;
    // gather record (statistics variant only; null = off): evaluated sample
    // k of launch slot q = 64 tile + lane writes its texel offsets to
    // rec[k * 64 total_tiles + q] when k < rec_cap; rec_count[q] = samples
    uint32_t *rec;
    int32_t *rec_count;
    int32_t rec_cap;
    // phase profile (null = off; needs stats): every wave adds the
    // shader-clock cycles it spent in each phase and its loop counts
    // (layout: enum PhaseSlot)
    unsigned long long *phases;
    // tile order (null = plain): workgroup slot i renders tile order[i]
    const int32_t *order;
    DevCamera cams[kCamsPerLaunch];
};

// Served launches (merf_serve.hip): one launch renders requests of several
// resident scenes.  The descriptors live in device memory, so a
// captured graph replays a launch unchanged (its first node copies the
// descriptors in).
struct ServeWork {
    DevCamera cam;                               // tile_start: first tile of this request in the launch
    int32_t scene;                               // slot of its scene in the server's scene table
    float step, inv_step, t_min;
    int32_t delta_mode;
};
struct ServeLaunch {
    int32_t n_work, total_tiles;
    ServeWork work[kCamsPerLaunch];
};
// Workgroup b of a served launch of G workgroups takes tiles from the share
// of XCD x = b % 8 (the runs of 4 consecutive tiles that xcd_remap deals to
// that XCD): first position b / 8, then, when the launch has more than G / 8
// positions per XCD, G / 8 + the positions it takes from the XCD's counter,
// until the share is exhausted.  Each counter has a 256-byte line of its
// own, zeroed before each launch that may take positions from it.
constexpr int kXcds = 8;
constexpr int kCtlStride = 64;                   // uint32 per counter line
struct ServeCtl {
    uint32_t next[kXcds * kCtlStride];           // next[x * kCtlStride]: positions taken by XCD x
};

// Slots of RenderBatch::phases (uint64 each, summed over the waves of a launch).
enum PhaseSlot {
    kPhSetup = 0,        // cycles: ray set-up and the first segment
    kPhMarch,            // cycles: march passes, segment openings excluded
    kPhOpen,             // cycles: segment openings during the march
    kPhShade,            // cycles: gather, dequantise, decode of parked samples
    kPhComposite,        // cycles: compositing and parking-queue upkeep
    kPhMlp,              // cycles: deferred MLP and output (slots 0..5 tile the wave's time)
    kPhWaves,            // waves
    kPhMarchPasses,      // wave-level march passes
    kPhOpenPasses,       // march passes in which some lane opened a segment
    kPhOpenLanes,        // segment openings (lanes)
    kPhShadePasses,      // shading passes
    kPhShadeLanes,       // samples shaded (lanes busy in shading passes)
    kPhRounds,           // march-shade-composite rounds
    kPhSlots = 16
};

// Launchers (merf_render.hip).
hipError_t launch_render(const DevScene &sc, const RenderBatch &rb, hipStream_t stream);
// Served launch: grid workgroups (a multiple of kXcds) render the tiles of
// *launch (device) with the scenes of table (device, indexed by
// ServeWork::scene), in the kernel variant of (mlp_prec, feat_prec,
// skip_mode); ctl (device) is the slot's control block.
const void *served_kernel(int mlp_prec, int feat_prec, int skip_mode);
// Zero the counters of a served launch's control block.
hipError_t launch_zero_ctl(ServeCtl *ctl, hipStream_t stream);
hipError_t launch_render_served(const DevScene *table, const ServeLaunch *launch, ServeCtl *ctl, int mlp_prec,
                                int feat_prec, int skip_mode, int grid, hipStream_t stream);
// Heaviest-first tile order of a launch: keys (uint8 [kOrderMaxTiles])
// receive the cost keys, group_counts (uint32 [kOrderMaxTiles / 16]) their
// counts per group of tiles, order (int32 [total_tiles]) the tiles sorted by
// key, highest first, ascending tile within a key.  Needs total_tiles <=
// kOrderMaxTiles.
hipError_t launch_tile_order(const DevScene &sc, const RenderBatch &rb, uint8_t *keys, uint32_t *group_counts,
                             int32_t *order, hipStream_t stream);
// order[i] = i for i < n (the plain order, for the gather replay).
hipError_t launch_identity_order(int32_t *order, int n, hipStream_t stream);
// The kernel a batch runs and its launch shape (for graph nodes).
const void *render_kernel(const RenderBatch &rb);
dim3 render_grid(const RenderBatch &rb);
constexpr int kRenderBlock = 64;
// Gather replay (measurement): re-issues the recorded texel loads of a
// launch of total_tiles tiles with no arithmetic, in the launch's tile order
// (null: plain); out: float4 per slot.
hipError_t launch_gather_replay(const DevScene &sc, const uint32_t *rec, const int32_t *rec_count, int cap,
                                const int32_t *order, int total_tiles, float *out, hipStream_t stream);
// Eq. 8 of n codes with range m and scale a = eq8_scale(m): prec 0 / 2 the
// correctly rounded float32 / bfloat16 value, prec 1 the float16 routine of
// the fp16-feature render path (deq_f16 with the scale the upload computes).
hipError_t launch_dequant(const uint8_t *codes, int64_t n, float m, float a, int prec, void *out,
                          hipStream_t stream);
// merf_ingest.hip: brick_pos[i] = bx | by << 10 | bz << 20 of brick slot i.
hipError_t launch_pack_bricks(const uint8_t *blocks, const int32_t *block_index, const int32_t *brick_pos,
                              int nbricks, int L, uint8_t *bricks, hipStream_t stream);
hipError_t launch_maxpool(const uint8_t *in, int rin, int f, uint8_t *out, hipStream_t stream);
// Distance grid of DevScene::dist from the occupancy levels (tmp0, tmp1:
// scratch of r_f^3 bytes each).
struct OccLevels {
    const uint8_t *occ[kMaxLevels];
    int32_t res[kMaxLevels];
    int32_t n;
};
hipError_t launch_distance_grid(const OccLevels &lv, uint8_t *tmp0, uint8_t *tmp1, uint8_t *dist,
                                hipStream_t stream);
// Forward empty extents of DevScene::dist in its eight-octant form (seed:
// scratch of r_f^3 bytes; sat: scratch of r_f^3 int32; out: 8 r_f^3 bytes).
hipError_t launch_octant_extents(const OccLevels &lv, uint8_t *seed, int32_t *sat, uint8_t *out, hipStream_t stream);

}  // namespace merf
