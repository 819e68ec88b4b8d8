/*
 * merf_serve.h -- serving runtime of the MI355X MERF renderer (C ABI).
 *
 * Keeps several baked scenes resident in device memory and renders a stream
 * of single-view requests with continuous batching.  This is the real-time
 * use MERF is built for (real-time view synthesis in a viewer, §6; compact
 * resident scenes, §7 Table 3), applied to many scenes and clients at once.
 *
 *  - Residency: scenes are admitted against a device-memory budget.  When a
 *    scene does not fit, idle scenes (no queued or running request) are
 *    evicted least recently used first if the server allows it; otherwise the
 *    add fails with MERF_E_OOM.
 *  - Continuous batching: requests queue on the host.  A worker thread owns
 *    `slots` HIP streams.  Whenever a slot is free, it fuses the oldest
 *    waiting request with the following waiting requests of the same scene
 *    and parameters (any image sizes, at most max_batch) into one launch of
 *    the render kernel.  Requests that arrive while others run are admitted
 *    as soon as a slot frees up, and the launches of different slots overlap
 *    on the device.
 *  - Graphs: with use_graphs, each slot captures its first launch of each
 *    kernel variant into a hipGraph; later batches update that graph's kernel
 *    node arguments and replay it.
 *
 * Every pixel of a request is computed exactly as merf_render computes it
 * (same kernel, same arguments per camera), so a result does not depend on
 * the batch it ran in.
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
    int32_t evict_idle;          /* 1: evict idle scenes (LRU) to admit a new one */
    int32_t pad;
    size_t hbm_budget;           /* device bytes for resident scenes; 0 = no cap */
} merf_server_config;

typedef struct {
    uint64_t submitted;          /* requests accepted */
    uint64_t completed;          /* requests finished */
    uint64_t launches;           /* kernel launches (plain or graph) */
    uint64_t graph_launches;     /* of which graph replays */
    uint64_t evictions;          /* scenes evicted to admit others */
    size_t resident_bytes;       /* device bytes of resident scenes */
    int32_t resident_scenes;
    int32_t max_inflight;        /* most requests on the device at once */
} merf_server_stats;

/* Create a server and its worker thread; streams are created on the
 * current device.  Errors: MERF_E_INVALID (config), MERF_E_DEVICE. */
int merf_server_create(const merf_server_config *cfg, merf_server_t *out);

/* Wait for every submitted request, stop the worker, free resident scenes
 * and streams.  Errors: MERF_E_INVALID for an unknown server. */
int merf_server_destroy(merf_server_t s);

/* Upload a scene (host descriptor, as merf_scene_upload) into the resident
 * set; returns its id.  Errors: MERF_E_OOM if it cannot be admitted under
 * the budget; MERF_E_INVALID for a bad descriptor. */
int merf_server_add_scene(merf_server_t s, const merf_scene_desc *desc, int32_t *scene_id);

/* Remove a resident scene.  Errors: MERF_E_INVALID if unknown or if
 * requests on it are still queued or running. */
int merf_server_remove_scene(merf_server_t s, int32_t scene_id);

/* Queue one view of a resident scene.  cam and p are copied; out_rgba_dev
 * is caller-owned device memory of width * height * 4 floats that must stay
 * valid until the request completes.  The request runs on the server's own
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
 * the part of it spent waiting for a slot.  Returns the request's status:
 * MERF_OK, or MERF_E_DEVICE if its launch failed. */
int merf_server_wait(merf_server_t s, uint64_t ticket, double *latency_ms, double *queue_ms);

/* Block until every submitted request has completed. */
int merf_server_drain(merf_server_t s);

int merf_server_get_stats(merf_server_t s, merf_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* MERF_SERVE_H */
