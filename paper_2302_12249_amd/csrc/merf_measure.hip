// merf_measure.hip -- host side of include/merf_measure.h: gather recording
// (a counting launch of the render kernel with its record pointers set) and
// the replay launch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "merf_internal.h"
#include "merf_measure.h"

using namespace merf;

extern "C" {

int merf_gather_slots(const merf_camera *cams, int32_t n_cams, int32_t *n_slots) {
    clear_error();
    if (!cams || !n_slots) return fail(MERF_E_INVALID, "NULL argument");
    if (n_cams < 1 || n_cams > kCamsPerLaunch)
        return fail(MERF_E_INVALID, "n_cams %d not in [1, %d]", n_cams, kCamsPerLaunch);
    RenderBatch rb;
    merf_render_params p{};
    p.struct_size = sizeof p;
    begin_batch(rb, p, 1.0f);
    for (int i = 0; i < n_cams; ++i) {
        int rc = check_camera(cams[i], i);
        if (rc) return rc;
        if (!add_camera(rb, cams[i], nullptr)) return fail(MERF_E_INVALID, "cameras exceed one launch");
    }
    if ((int64_t)rb.total_tiles * 64 > INT32_MAX) return fail(MERF_E_INVALID, "too many slots");
    *n_slots = rb.total_tiles * 64;
    return MERF_OK;
}

int merf_record_gathers(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                        uint32_t *rec_dev, int32_t cap, int32_t *count_dev, int32_t *order_dev, float *out_rgba_dev,
                        void *hip_stream) {
    clear_error();
    const DevScene *ds = scene_dev(s);
    if (!ds) return fail(MERF_E_INVALID, "merf_record_gathers: invalid scene handle");
    float step = 0.0f;
    int rc = check_params(p, ds->res, &step);
    if (rc) return rc;
    if (!p->stats_dev) return fail(MERF_E_INVALID, "recording needs stats_dev");
    if (cap < 1) return fail(MERF_E_INVALID, "cap %d < 1", cap);
    if (!cams || !rec_dev || !count_dev || !order_dev || !out_rgba_dev) return fail(MERF_E_INVALID, "NULL buffer");
    if ((int64_t)ds->nbl * ds->nbl * ds->nbl > ((int64_t)1 << 19))
        return fail(MERF_E_INVALID, "grid of %d^3 blocks too large to record", ds->nbl);
    if (n_cams < 1 || n_cams > kCamsPerLaunch)
        return fail(MERF_E_INVALID, "n_cams %d not in [1, %d]", n_cams, kCamsPerLaunch);
    RenderBatch rb;
    begin_batch(rb, *p, step);
    int64_t pix = 0;
    for (int i = 0; i < n_cams; ++i) {
        if ((rc = check_camera(cams[i], i))) return rc;
        if (!add_camera(rb, cams[i], out_rgba_dev + pix * 4)) return fail(MERF_E_INVALID, "cameras exceed one launch");
        pix += (int64_t)cams[i].width * cams[i].height;
    }
    rb.rec = rec_dev;
    rb.rec_count = count_dev;
    rb.rec_cap = cap;
    return render_launch(*ds, rb, p->tile_order, static_cast<hipStream_t>(hip_stream), order_dev);
}

int merf_render_timed(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                      float *out_rgba_dev, void *ev_start, void *ev_end, void *hip_stream) {
    clear_error();
    const DevScene *ds = scene_dev(s);
    if (!ds) return fail(MERF_E_INVALID, "merf_render_timed: invalid scene handle");
    float step = 0.0f;
    int rc = check_params(p, ds->res, &step);
    if (rc) return rc;
    if (!cams || !out_rgba_dev || !ev_start || !ev_end) return fail(MERF_E_INVALID, "NULL argument");
    if (n_cams < 1 || n_cams > kCamsPerLaunch)
        return fail(MERF_E_INVALID, "n_cams %d not in [1, %d]", n_cams, kCamsPerLaunch);
    RenderBatch rb;
    begin_batch(rb, *p, step);
    int64_t pix = 0;
    for (int i = 0; i < n_cams; ++i) {
        if ((rc = check_camera(cams[i], i))) return rc;
        if (!add_camera(rb, cams[i], out_rgba_dev + pix * 4)) return fail(MERF_E_INVALID, "cameras exceed one launch");
        pix += (int64_t)cams[i].width * cams[i].height;
    }
    return render_launch(*ds, rb, p->tile_order, static_cast<hipStream_t>(hip_stream), nullptr,
                         static_cast<hipEvent_t>(ev_start), static_cast<hipEvent_t>(ev_end));
}

int merf_render_phases(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                       float *out_rgba_dev, uint64_t *phases_dev, void *hip_stream) {
    clear_error();
    const DevScene *ds = scene_dev(s);
    if (!ds) return fail(MERF_E_INVALID, "merf_render_phases: invalid scene handle");
    float step = 0.0f;
    int rc = check_params(p, ds->res, &step);
    if (rc) return rc;
    if (!p->stats_dev) return fail(MERF_E_INVALID, "the phase profile needs stats_dev");
    if (!cams || !out_rgba_dev || !phases_dev) return fail(MERF_E_INVALID, "NULL buffer");
    if (n_cams < 1 || n_cams > kCamsPerLaunch)
        return fail(MERF_E_INVALID, "n_cams %d not in [1, %d]", n_cams, kCamsPerLaunch);
    RenderBatch rb;
    begin_batch(rb, *p, step);
    int64_t pix = 0;
    for (int i = 0; i < n_cams; ++i) {
        if ((rc = check_camera(cams[i], i))) return rc;
        if (!add_camera(rb, cams[i], out_rgba_dev + pix * 4)) return fail(MERF_E_INVALID, "cameras exceed one launch");
        pix += (int64_t)cams[i].width * cams[i].height;
    }
    rb.phases = reinterpret_cast<unsigned long long *>(phases_dev);
    return render_launch(*ds, rb, p->tile_order, static_cast<hipStream_t>(hip_stream));
}

int merf_replay_gathers(merf_scene_t s, const uint32_t *rec_dev, const int32_t *count_dev, int32_t cap,
                        const int32_t *order_dev, int32_t n_slots, float *out_dev, void *hip_stream) {
    clear_error();
    const DevScene *ds = scene_dev(s);
    if (!ds) return fail(MERF_E_INVALID, "merf_replay_gathers: invalid scene handle");
    if (n_slots < 64 || n_slots % 64 != 0) return fail(MERF_E_INVALID, "n_slots %d not a positive multiple of 64", n_slots);
    if (cap < 1) return fail(MERF_E_INVALID, "cap %d < 1", cap);
    if (!rec_dev || !count_dev || !order_dev || !out_dev) return fail(MERF_E_INVALID, "NULL buffer");
    hipError_t e = launch_gather_replay(*ds, rec_dev, count_dev, cap, order_dev, n_slots / 64, out_dev,
                                        static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "replay launch");
    return MERF_OK;
}

}  // extern "C"
