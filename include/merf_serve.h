/*
 * merf_serve.h -- serving runtime of the MI355X MERF renderer (C ABI).
 *
 * Keeps baked scenes resident in device memory and renders a stream of
 * single-view requests with continuous batching.  This is the real-time use
 * MERF is built for (real-time view synthesis in a viewer, Sec. 6; compact
 * resident scenes, Sec. 7 Table 3), applied to many scenes and clients at
 * once.
 *
 *  - Registration and admission by memory: the server keeps a host copy of
 *    every registered scene.  A scene is made resident at registration if it
 *    fits the device-memory budget, otherwise when a request needs it.  The
 *    oldest waiting request whose scene is not resident gets it loaded as
 *    soon as the budget allows; with evict_idle, room is made by evicting
 *    resident scenes that no older request needs, least requested first
 *    (request counts decayed with a 2 s time constant; ties: least recently
 *    used), so that under a skewed popularity the rarely requested scenes
 *    take turns in the memory the popular ones leave (a scene still
 *    rendering is first drained: it takes no newer requests until it is
 *    evicted).  Requests older than the waiting one keep being
 *    served, so every request is eventually admitted.  Without evict_idle,
 *    only merf_server_remove_scene frees memory.  With evict_idle, after a
 *    scene's first upload the server's host copy is the device image that
 *    upload built (packed bricks, empty-space grids and all), so a
 *    re-admission is a single host-to-device copy and runs no kernels beside
 *    the renders.
 *  - Continuous batching: requests queue on the host.  A worker thread owns
 *    `slots` HIP streams.  Whenever a slot is free, it fuses the oldest
 *    request whose scene is resident with the following such requests that
 *    use the same kernel variant (MLP precision, feature precision, skip
 *    mode) -- any scenes, any image sizes, any step or t_min, at most
 *    max_batch -- into one launch.  Requests that arrive while others run
 *    are admitted as soon as a slot frees up, and the launches of different
 *    slots overlap on the device.
 *  - Launch classes: a served launch has a fixed number of workgroups,
 *    64 << 2c for c = 0 .. 6 (64 to 262144): the smallest class with a
 *    workgroup for each of its 8x8 tiles.  A launch of more tiles is
 *    persistent: 4096 workgroups go on taking tiles from a device-side
 *    counter per XCD until the launch's tiles are done.  It reads its work
 *    descriptors (per request: scene slot, camera, output, march parameters)
 *    and a device table of the resident scenes from device memory.  With
 *    use_graphs, each slot captures one hipGraph per kernel variant and grid
 *    size -- a copy of the descriptors into device memory, then the kernel --
 *    and replays it unchanged.
 *
 * Every pixel of a request is computed exactly as merf_render computes it
 * (same per-tile code, same arguments per camera), so a result does not
 * depend on the batch it ran in.
 *
 * Functions return MERF_OK or a negative MERF_E_* code; merf_last_error()
 * (merf.h) describes the calling thread's last error.  All functions are
 * thread-safe.
 */
#ifndef MERF_SERVE_H
#define MERF_SERVE_H

#include "merf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct merf_server *merf_server_t;

typedef struct {
    uint32_t struct_size;        /* = sizeof(merf_server_config) */
    int32_t slots;               /* launches in flight at once, 1..8 (one HIP stream each) */
    int32_t max_batch;           /* requests fused into one launch, 1..16 */
    int32_t use_graphs;          /* 1: replay captured hipGraphs; 0: plain launches */
    int32_t evict_idle;          /* 1: evict idle scenes (least requested first) to admit a new one */
    int32_t pad;
    size_t hbm_budget;           /* device bytes for resident scenes; 0 = no cap */
} merf_server_config;

typedef struct {
    uint64_t submitted;          /* requests accepted */
    uint64_t completed;          /* requests finished (or failed) */
    uint64_t launches;           /* kernel launches (plain or graph) */
    uint64_t graph_launches;     /* of which graph replays */
    uint64_t mixed_launches;     /* launches that rendered requests of more than one scene */
    uint64_t evictions;          /* scenes evicted to admit others */
    uint64_t admissions;         /* scenes made resident (at registration or for a request) */
    uint64_t admission_us;       /* host time spent making them resident (upload to table entry) */
    uint64_t image_admissions;   /* of the admissions, those copied from a kept device image */
    size_t resident_bytes;       /* device bytes of resident scenes */
    int32_t resident_scenes;
    int32_t registered;          /* registered scenes, resident or not */
    int32_t max_inflight;        /* most requests on the device at once */
    int32_t pad;
} merf_server_stats;

/* Create a server and its worker thread; streams are created on the
 * current device.  Errors: MERF_E_INVALID (config), MERF_E_DEVICE. */
int merf_server_create(const merf_server_config *cfg, merf_server_t *out);

/* Wait for every submitted request, stop the worker, free resident scenes
 * and streams.  Errors: MERF_E_INVALID for an unknown server. */
int merf_server_destroy(merf_server_t s);

/* Register a scene (host descriptor, as merf_scene_upload; its arrays are
 * copied and may be released when the call returns) and return its id.  The
 * scene is uploaded now if it fits the budget, otherwise when a request
 * needs it.  Errors: MERF_E_OOM if it alone exceeds the budget or its upload
 * fails; MERF_E_INVALID for a bad descriptor. */
int merf_server_add_scene(merf_server_t s, const merf_scene_desc *desc, int32_t *scene_id);

/* Unregister a scene and free its device memory if resident.  Errors:
 * MERF_E_INVALID if unknown, being loaded, or if requests on it are still
 * queued or running. */
int merf_server_remove_scene(merf_server_t s, int32_t scene_id);

/* Queue one view of a registered scene (resident or not).  cam and p are
 * copied; out_rgba_dev is caller-owned device memory of width * height * 4
 * floats that must stay valid until the request completes.  The request runs on the server's own
 * streams, not ordered after any work of the caller: out_rgba_dev must have
 * no pending writes when submitted.  p->tile_order is ignored: served
 * launches overlap one another and keep the plain tile order.  Errors:
 * MERF_E_INVALID (unknown scene, bad camera or parameters, NULL output). */
int merf_server_submit(merf_server_t s, int32_t scene_id, const merf_camera *cam, const merf_render_params *p,
                       float *out_rgba_dev, uint64_t *ticket);

/* 1 if the request has completed, 0 if it is queued or running.
 * Errors: MERF_E_INVALID for an unknown ticket. */
int merf_server_poll(merf_server_t s, uint64_t ticket);

/* Block until the request completes.  latency_ms (optional) receives the
 * time from submit to the host observing completion, and queue_ms (optional)
 * the part of it spent waiting for its scene and a slot.  Returns the
 * request's status: MERF_OK, MERF_E_DEVICE if its launch failed, or the
 * error of its scene's upload if that failed (MERF_E_OOM also when the
 * server is destroyed while the scene cannot fit without evictions). */
int merf_server_wait(merf_server_t s, uint64_t ticket, double *latency_ms, double *queue_ms);

/* Block until every submitted request has completed. */
int merf_server_drain(merf_server_t s);

int merf_server_get_stats(merf_server_t s, merf_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* MERF_SERVE_H */
