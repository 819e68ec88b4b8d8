/*
 * merf_measure.h -- measurement entry points of the MERF renderer (MI355X,
 * gfx950): the achievable-gather bound of a view, and where a wave's time
 * goes.
 *
 * The renderer's memory traffic is its texel gathers (Sec. 6: per evaluated
 * sample, 8 grid voxels and 3 x 4 plane texels of 8 uint8 channels).  To
 * bound what those gathers alone can reach, merf_record_gathers renders a
 * view while recording, for every evaluated sample, the texel offsets it
 * reads; merf_replay_gathers then re-issues exactly those loads, in the same
 * order, tile order, tile layout and wave shape, with no other arithmetic.
 * The ratio of replay time to render time is the fraction of the gather
 * bound the renderer reaches.
 *
 * Same error conventions as merf.h (0 = MERF_OK, negative codes,
 * merf_last_error()).
 */
#ifndef MERF_MEASURE_H
#define MERF_MEASURE_H

#include "merf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of recording slots (one per lane: 64 per 8x8 pixel tile) of a
 * launch of n_cams cameras (host array).  Errors: MERF_E_INVALID for a bad
 * camera or more cameras than one launch carries (16). */
int merf_gather_slots(const merf_camera *cams, int32_t n_cams, int32_t *n_slots);

/*
 * Render cams (at most 16, one launch) exactly as merf_render does, into
 * out_rgba_dev, and record the gathers.  p->stats_dev must be set (the
 * recording runs in the counting variant of the kernel, which also adds its
 * counters there).  count_dev: device int32[n_slots] receives the number of
 * evaluated samples of each slot.  rec_dev: device uint32[cap][n_slots][4]
 * receives, for evaluated sample k < cap of slot q, at [k][q]: the byte
 * offsets of the (u, v) texels of the three planes and (brick index entry
 * << 13 | byte offset in the brick) of the grid footprint.  Samples k >= cap
 * are counted but not recorded.  order_dev: device int32[n_slots / 64]
 * receives the tile order of the launch (entry i: the tile workgroup slot i
 * rendered; p->tile_order decides it as in merf_render).  Requires
 * (grid_res / 8)^3 <= 2^19 so that the grid word packs.  Asynchronous on
 * hip_stream.
 * Errors: MERF_E_INVALID for a bad handle, camera, parameter, cap < 1, NULL
 * buffers or a grid too large to pack; MERF_E_DEVICE if the launch fails.
 */
int merf_record_gathers(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                        uint32_t *rec_dev, int32_t cap, int32_t *count_dev, int32_t *order_dev, float *out_rgba_dev,
                        void *hip_stream);

/*
 * Render cams (at most 16, one launch) exactly as merf_render does, and
 * record ev_start and ev_end (hipEvent_t, created by the caller with timing
 * enabled) on hip_stream right before and right after the render kernel, so
 * that their elapsed time is that kernel's duration alone (the tile-order
 * prepass of the launch runs before ev_start).  Asynchronous on hip_stream.
 * Errors: MERF_E_INVALID for a bad handle, camera, parameter or NULL
 * argument; MERF_E_DEVICE if a launch or event record fails.
 */
int merf_render_timed(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                      float *out_rgba_dev, void *ev_start, void *ev_end, void *hip_stream);

/*
 * Re-issue the recorded loads of n_slots slots (rec_dev, count_dev, cap and
 * order_dev as given to merf_record_gathers for scene s), with the tiles in
 * the recorded order, and write one float4 per slot to
 * out_dev (device, n_slots * 4 floats): its recorded sample count, then
 * values with no meaning that keep the loads live.  Asynchronous on
 * hip_stream.
 * Errors: MERF_E_INVALID for a bad handle, n_slots not a positive multiple of
 * 64, cap < 1 or NULL buffers; MERF_E_DEVICE if the launch fails.
 */
int merf_replay_gathers(merf_scene_t s, const uint32_t *rec_dev, const int32_t *count_dev, int32_t cap,
                        const int32_t *order_dev, int32_t n_slots, float *out_dev, void *hip_stream);

/*
 * Phase profile of a view: render cams (at most 16, one launch) exactly as
 * merf_render does (same image), in the counting variant of the kernel
 * (p->stats_dev must be set), while every wave reads the shader clock at the
 * points its 64 lanes pass together and ADDS to phases_dev (device
 * uint64[16]), summed over the waves of the launch:
 *   [0] cycles of ray set-up and the first segment (Sec. 4.2 Eq. 7),
 *   [1] cycles of march passes (occupancy / empty-space steps, Sec. 6),
 *   [2] cycles of segment openings during the march (Eq. 7 breakpoints),
 *   [3] cycles of shading passes (gather, Eq. 8, Eq. 5, Eq. 6),
 *   [4] cycles of compositing and queue upkeep (Eq. 1-2),
 *   [5] cycles of the deferred MLP and the output (Eq. 3),
 *   [6] cycles of the whole wave, [7] waves, [8] march passes,
 *   [9] march passes in which some lane opened a segment, [10] segment
 *   openings (lanes), [11] shading passes, [12] samples shaded,
 *   [13] march-shade-composite rounds, [14..15] 0.
 * The clock reads perturb the timing slightly; the counts are exact.
 * Asynchronous on hip_stream.
 * Errors: MERF_E_INVALID for a bad handle, camera, parameter or NULL
 * buffer; MERF_E_DEVICE if a launch fails.
 */
int merf_render_phases(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                       float *out_rgba_dev, uint64_t *phases_dev, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MERF_MEASURE_H */
