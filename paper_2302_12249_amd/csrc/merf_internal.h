// merf_internal.h -- host helpers shared by the C ABI (merf_api.hip) and the
// serving runtime (merf_serve.hip).  Not part of the public interface.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "merf.h"
#include "merf_device.h"

namespace merf {

// Record the calling thread's error message; returns code.
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void clear_error();

// Eq. 8 scale a = 2 m / 255 in float32, correctly rounded: 2 m is exact and
// the division rounds once.  The upload derives the kernels' dequantisation
// constants from it and merf_dequantize uses the same value, so the routine
// that entry point runs is the renderer's own with the renderer's constant.
inline float eq8_scale(float m) { return (2.0f * m) / 255.0f; }

// Upload for the serving runtime: merf_scene_upload with every allocation,
// copy and kernel ordered on `stream` (stream-ordered allocation, so nothing
// waits for other work on the device); returns once the scene is resident.
int scene_upload_on(const merf_scene_desc *desc, hipStream_t stream, merf_scene_t *out);
// Release a scene of scene_upload_on, in order on `stream`, without waiting
// for other work on the device: the caller guarantees that no queued or
// running work reads it.
int scene_release_on(merf_scene_t s, hipStream_t stream);

// A scene's device image: the bytes of its device allocation once an upload
// has built it (packed bricks, occupancy levels, empty-space grids, planes,
// MLP) and its device view at the address it was taken from.  The arrays keep
// their offsets in the allocation, so the image restored at another address
// renders bit for bit as the scene it was taken from, with no build step.
struct SceneImage {
    DevScene ds;                 // device view at `base`
    uintptr_t base = 0;          // device address the image was taken from
    size_t bytes = 0;
    int32_t nbricks = 0;
};
// Copy live scene s's device bytes into host[0, host_bytes) in order on
// `stream` (pinned host memory makes it a plain DMA) and describe them in
// img; returns once the copy is done.
int scene_image_on(merf_scene_t s, void *host, size_t host_bytes, hipStream_t stream, SceneImage *img);
// A scene made resident from an image: one stream-ordered allocation and one
// host-to-device copy on `stream`, no kernels; returns once resident.  Counts
// against the device budget like an upload.
int scene_from_image_on(const SceneImage &img, const void *host, hipStream_t stream, merf_scene_t *out);

// Device view of a live scene handle, or nullptr.
const DevScene *scene_dev(merf_scene_t s);

// Device bytes merf_scene_upload would allocate for desc (0 if desc is invalid).
size_t scene_device_bytes(const merf_scene_desc *desc);

// Validate render parameters; res is the finest scene resolution max(R, L),
// whose texel size 4/res is the default step.  On success stores the
// effective contracted step.
int check_params(const merf_render_params *p, int res, float *step);
int check_camera(const merf_camera &c, int index);

// Start a launch descriptor (no cameras yet) / append one camera whose
// row-major RGBA pixels start at out.  add_camera fails when the launch is
// full or its tile count would overflow.
void begin_batch(RenderBatch &rb, const merf_render_params &p, float step);
bool add_camera(RenderBatch &rb, const merf_camera &c, float *out);

// Launch one render batch on stream: heaviest tiles first when tile_order is
// 0 and the launch has kOrderMinTiles..kOrderMaxTiles tiles (and the stream
// is not capturing a graph), plain order otherwise.  order_out (device
// int32[total_tiles], or null) receives the order used: order_out[i] is the
// tile of workgroup slot i.  ev_start / ev_end (or null) are recorded on
// stream right before and after the render kernel.  Returns MERF_OK or a
// recorded error.
int render_launch(const DevScene &ds, RenderBatch &rb, int tile_order, hipStream_t stream,
                  int32_t *order_out = nullptr, hipEvent_t ev_start = nullptr, hipEvent_t ev_end = nullptr);

}  // namespace merf
