/*
 * merf.h -- C ABI of the MI355X (gfx950) MERF renderer.
 *
 * Renders a baked MERF scene (Reiser et al., "MERF: Memory-Efficient Radiance
 * Fields for Real-time View Synthesis in Unbounded Scenes", arXiv 2302.12249)
 * by deferred volume rendering on one GPU:
 *   per pixel: cast a ray; map it through the piecewise-projective
 *   contraction (Sec. 4.2, Eq. 7); march a uniform lattice in contracted
 *   space, skipping empty space with a max-pooled occupancy hierarchy (Sec. 6);
 *   at each occupied sample, gather the sparse low-resolution 3D grid
 *   (trilinear) and the three high-resolution planes (bilinear) (Sec. 4.1,
 *   Eq. 5) from uint8 codes dequantised by Eq. 8; decode density, diffuse
 *   colour and features (Eq. 6); composite front to back (Eq. 1-2) until the
 *   transmittance falls below a threshold (Sec. 6); then evaluate the small
 *   view-dependent MLP once per pixel (Eq. 3, App. B).
 *
 * All functions return 0 (MERF_OK) or a negative error code; a message for
 * the calling thread's last error is available from merf_last_error().
 * Every error path releases whatever the failing call had allocated.
 * Pointers passed in are read during the call only; the caller keeps
 * ownership.
 */
#ifndef MERF_H
#define MERF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MERF_OK 0
#define MERF_E_INVALID (-1)   /* bad argument, descriptor, handle or double free */
#define MERF_E_OOM (-2)       /* device allocation failed or HBM budget exceeded  */
#define MERF_E_DEVICE (-3)    /* a HIP runtime call failed                        */

#define MERF_MAX_OCC_LEVELS 4

/* Opaque handle of a scene resident in device memory (owned by the library
 * from merf_scene_upload until merf_free). */
typedef struct merf_scene *merf_scene_t;

/*
 * Baked scene (Sec. 4.1 representation, Sec. 5.3 baking, Sec. 6
 * occupancy hierarchy).  Channel order of every texel: [density, diffuse r,
 * g, b, feature 0..3] (C = 4 + K with K = 4).
 *
 *  grid_res L      resolution of the low-resolution 3D grid V; multiple of 8.
 *  block_size      edge of a stored block; must be 8.
 *  plane_res R     resolution of the three 2D planes.
 *  channels        must be 8.
 *  num_blocks      number of stored blocks (may be 0).
 *  block_index     int32 [(L/8)^3], z-major ((bz*nb + by)*nb + bx); -1 marks
 *                  an absent block (all of its voxels read code 0), otherwise
 *                  a slot in [0, num_blocks).
 *  blocks          uint8 [num_blocks][8][8][8][8], indexed [z][y][x][c].
 *  planes          uint8 [3][R][R][8]: plane 0 = P_x indexed [z][y],
 *                  plane 1 = P_y indexed [z][x], plane 2 = P_z indexed [y][x].
 *  occ_levels      number of occupancy levels, 1..4, coarse to fine.
 *  occ_res[l]      level resolution r; a cell covers a box of edge 4/r of the
 *                  contracted domain [-2, 2]^3.  Each resolution divides the
 *                  next finer one (a max-pool pyramid, Sec. 6).  A sample is
 *                  rendered only if every level marks the cell containing it.
 *  occ[l]          uint8 [r^3] z-major, nonzero = occupied.
 *  m_density,
 *  m_feature       Eq. 8 ranges: code b means 2 m b / 255 - m (14 and 7).
 *  mlp_in,
 *  mlp_hidden      deferred MLP shape; must be 34 and 16 (App. B: 3 layers,
 *                  16 hidden units, 4 direction frequencies).
 *  mlp_params      float32 W0[in][h], b0[h], W1[h][h], b1[h], W2[h][3], b2[3].
 *
 * block_index must be host memory (the upload reads it to lay the bricks
 * out).  blocks, planes, occ[l] and mlp_params may be host memory or device
 * memory of the current device: an occupancy pyramid built on the device by
 * merf_occupancy_pyramid is uploaded without a trip through the host.
 */
typedef struct {
    uint32_t struct_size;                 /* = sizeof(merf_scene_desc) */
    int32_t grid_res;
    int32_t block_size;
    int32_t plane_res;
    int32_t channels;
    int32_t num_blocks;
    const int32_t *block_index;
    const uint8_t *blocks;
    const uint8_t *planes;
    int32_t occ_levels;
    int32_t occ_res[MERF_MAX_OCC_LEVELS];
    const uint8_t *occ[MERF_MAX_OCC_LEVELS];
    float m_density;
    float m_feature;
    int32_t mlp_in;
    int32_t mlp_hidden;
    const float *mlp_params;
} merf_scene_desc;

/*
 * Pinhole camera, OpenCV axes (x right, y down, z forward).  c2w is the
 * row-major 3x4 camera-to-world matrix [R | centre].  The ray of pixel
 * (row i, column j) starts at the centre and has direction
 * normalize(R * ((j + 1/2 - cx)/fx, (i + 1/2 - cy)/fy, 1)).
 */
typedef struct {
    float c2w[12];
    float fx, fy, cx, cy;
    int32_t width, height;                /* 1..16384 each */
} merf_camera;

/* Render parameters. */
typedef struct {
    uint32_t struct_size;                 /* = sizeof(merf_render_params) */
    float step;                           /* contracted distance between samples; <= 0: 4/R */
    float t_min;                          /* stop when transmittance < t_min (Sec. 6: 2e-4) */
    int32_t delta_mode;                   /* 0: delta = contracted interval length;
                                             1: world length of its preimage */
    int32_t mlp_prec;                     /* deferred MLP: 0 = fp32, 1 = fp16, 2 = bf16 */
    int32_t feat_prec;                    /* 0 = codes interpolated in fp32; 1 = every code
                                             dequantised to float16 first (sums stay fp32);
                                             2 = appearance interpolated from float16
                                             operands (weights rounded to float16, codes
                                             exact) by dot products with fp32 sums, density
                                             as in 0 (the fast reduced-precision mode) */
    int32_t skip_mode;                    /* empty-space skipping, same image either way:
                                             0 = empty-space grid derived from the occupancy
                                             levels at upload (the largest empty cube ahead
                                             of a sample is left in one step);
                                             1 = the levels themselves, coarse to fine,
                                             leaving one empty cell per step (Sec. 6) */
    int32_t tile_order;                   /* order in which the 8x8 tiles of a launch run,
                                             same image either way: 0 = estimated
                                             heaviest first for launches of 6144 to
                                             131072 tiles (a prepass marches 4 rays of
                                             each tile and, up to 65536 tiles, counts
                                             the samples they evaluate before
                                             terminating, up to 4 each;
                                             calls on a device allocate up to 64 work
                                             buffers of 672 KB, kept until the process
                                             ends; with all 64 in flight, the call
                                             keeps the plain order and never waits),
                                             plain order otherwise; 1 = plain order */
    uint64_t *stats_dev;                  /* NULL, or device uint64[8] to which the render
                                             ADDS: [0] rays, [1] occupancy lookups
                                             (skip_mode 0: distance-grid lookups),
                                             [2] lattice samples visited, [3] samples
                                             evaluated, [4] samples with alpha > 0,
                                             [5] rays terminated early, [6..7] 0 */
} merf_render_params;

/*
 * Copy a baked scene into device memory and return its handle.
 * desc and the arrays it points to (host or device memory, see
 * merf_scene_desc) are read during the call.
 * The library re-lays the data out for the GPU (sparse grid blocks padded
 * with a one-voxel apron so a trilinear footprint never spans two blocks)
 * and derives the empty-space distance grid of skip_mode 0 (one byte per
 * cell of the finest occupancy level).
 * Synchronous: the scene is resident when the call returns.
 * Errors: MERF_E_INVALID for an inconsistent descriptor (sizes, block index
 * entries out of range, NULL arrays); MERF_E_OOM when the device bytes would
 * exceed the budget set by merf_set_hbm_budget or allocation fails.
 */
int merf_scene_upload(const merf_scene_desc *desc, merf_scene_t *out);

/*
 * Render n_cams cameras (host array) of scene s into out_rgba_dev, a device
 * float32 buffer of sum_i(width_i * height_i) * 4 values owned by the caller:
 * camera i's pixels start at the sum of the pixel counts of cameras 0..i-1,
 * row-major, each pixel (R, G, B, 1 - T).  RGB = C_d + h(C_d, F, d) is not
 * clamped.  Asynchronous and ordered on hip_stream (a hipStream_t; NULL =
 * the null stream); host arguments may be released when the call returns.
 * n_cams == 0 is a no-op.
 * Errors: MERF_E_INVALID for a bad handle, camera, parameter or NULL
 * buffer; MERF_E_DEVICE if a launch fails.
 */
int merf_render(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                float *out_rgba_dev, void *hip_stream);

/*
 * merf_render for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, image and errors as merf_render, bit for bit, but it calls
 * no hipMalloc, hipFree or other allocating routine, and every kernel runs on
 * hip_stream (merf_render runs the tile-order prepass on a stream of the
 * library's own, with work buffers it allocates).  The tile-order prepass
 * instead uses one fixed device array of 672 KiB per GPU, held until the
 * process ends, which bounds a launch run in tile order (tile_order 0) to
 * 131072 8x8 tiles (four 1920x1080 frames): a call with such a launch is
 * rejected with MERF_E_INVALID before anything runs (tile_order 1 has no
 * bound).  Every call on a GPU shares that GPU's array; each launch rewrites
 * all of it that it reads, so nothing carries over from an earlier call, but
 * calls that overlap on one GPU (different streams) race and must not be
 * issued.  hip_stream must belong to the current device.
 */
int merf_render_noalloc(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                        float *out_rgba_dev, void *hip_stream);

/*
 * Release a scene.  Waits for all work queued on the device before freeing
 * (renders that read the scene may be queued on any stream, and hipFree
 * waits for the device in any case); the serving runtime (merf_serve.h)
 * releases its scenes stream-ordered instead, without blocking.
 * Errors: MERF_E_INVALID for NULL, an unknown handle or a second free.
 */
int merf_free(merf_scene_t s);

/* Message of the calling thread's most recent error ("" if none). */
const char *merf_last_error(void);

/* Cap on device bytes held by all resident scenes (default: no cap).
 * Uploads that would exceed it fail with MERF_E_OOM. */
int merf_set_hbm_budget(size_t bytes);

/* Device bytes currently held by resident scenes. */
size_t merf_hbm_in_use(void);

/* Device bytes held by scene s (0 for an invalid handle). */
size_t merf_scene_bytes(merf_scene_t s);

/*
 * Eq. 8 dequantisation (Sec. 5.2) of n device codes with range m:
 * out[i] = 2 m codes[i] / 255 - m, correctly rounded to the output format,
 * which is what each precision of the renderer is checked against bit for
 * bit.  out_dev holds n elements of the format.
 *   prec 1 (float16): runs the device routine of the fp16-feature render path
 *     (merf_render_params.feat_prec = 1), which dequantises every code it
 *     reads with this routine, with the scale RN32(2m/255) that
 *     merf_scene_upload computes for it.
 *   prec 0 (float32) / 2 (bfloat16): the correctly rounded value.  The fp32
 *     render path (feat_prec = 0) does not dequantise code by code: it
 *     interpolates the codes of each source and applies Eq. 8's affine map
 *     once per channel, which equals the interpolation of the dequantised
 *     values in exact arithmetic because the weights of each source sum to 1
 *     (the two differ by float32 rounding only).  The fp16-interpolation
 *     path (feat_prec = 2) applies the same affine map after interpolating
 *     the codes with float16 weights.
 * Asynchronous on hip_stream.
 * Errors: MERF_E_INVALID for n < 0, NULL buffers, m <= 0 or a bad prec.
 */
int merf_dequantize(const uint8_t *codes_dev, int64_t n, float m, int32_t prec, void *out_dev,
                    void *hip_stream);

/*
 * Occupancy hierarchy by max-pooling (Sec. 6: the renderer's occupancy grids
 * are max-pools of the full-resolution binary mask A of Sec. 5.3).
 * mask_dev: device uint8 [res^3] z-major, nonzero = occupied.  For each level
 * l, out_dev[l] (device, (res / factors[l])^3 bytes, caller-owned) receives 1
 * where any cell of the factors[l]^3 block is occupied, else 0.  factors[l]
 * must divide res; factor 1 copies the mask as 0/1.  Host arrays factors and
 * out_dev are read during the call.  Asynchronous on hip_stream.
 * Errors: MERF_E_INVALID for res outside [1, 2048], n_levels outside [1, 8],
 * a factor that does not divide res, or NULL buffers.
 */
int merf_occupancy_pyramid(const uint8_t *mask_dev, int32_t res, const int32_t *factors, int32_t n_levels,
                           uint8_t *const *out_dev, void *hip_stream);

/*
 * Empty-space distance grid: the acceleration structure behind skip_mode 0 of
 * merf_render, derived from the occupancy hierarchy of Sec. 6 (the upload
 * builds it itself; this entry point exposes the same routine).
 * occ_dev[l] (device, res[l]^3 bytes, z-major, nonzero = occupied) for
 * l = 0 .. n_levels - 1, coarse to fine, each res[l] dividing res[l + 1].
 * out_dev (device, r^3 bytes, r = res[n_levels - 1], caller-owned) receives
 * for every cell of the finest level the Chebyshev distance, in cells, to the
 * nearest cell that every level marks occupied, capped at 255; 0 means the
 * cell itself is occupied at every level, 255 also means no such cell.  Host
 * arrays occ_dev and res are read during the call.  Allocates 2 r^3 bytes of
 * device scratch, runs on hip_stream and returns once the grid is complete.
 * Errors: MERF_E_INVALID for n_levels outside [1, 4], a resolution outside
 * [1, 1024] or not dividing the next, or NULL buffers; MERF_E_OOM if the
 * scratch cannot be allocated.
 */
int merf_distance_grid(const uint8_t *const *occ_dev, const int32_t *res, int32_t n_levels, uint8_t *out_dev,
                       void *hip_stream);

/*
 * Octant form of the empty-space grid (what the upload builds for skip_mode
 * 0 when the finest occupancy resolution is at most 256).  Same inputs as
 * merf_distance_grid; out_dev (device, 8 r^3 bytes, caller-owned) receives
 * eight grids, octant o = (bit 0: -x, bit 1: -y, bit 2: -z) at o r^3: for each
 * finest cell, the largest E <= 255 such that the cube of E cells on a side
 * with a corner at the cell, extending in the octant's directions (clipped to
 * the grid), holds no cell that every level marks occupied; 0 for such a cell
 * itself.  Allocates 5 r^3 bytes of device scratch, runs on hip_stream and
 * returns once the grids are complete.
 * Errors: as merf_distance_grid.
 */
int merf_octant_extent_grid(const uint8_t *const *occ_dev, const int32_t *res, int32_t n_levels, uint8_t *out_dev,
                            void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MERF_H */
