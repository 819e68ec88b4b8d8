// merf_api.hip -- host side of the C ABI declared in include/merf.h:
// argument validation, device residency and HBM budget of baked scenes,
// launch of the render kernels, thread-local error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "merf.h"
#include "merf_device.h"
#include "merf_internal.h"

using namespace merf;

struct merf_scene {
    uint32_t magic;
    void *dev_base;
    size_t dev_bytes;
    DevScene ds;
    int32_t nbricks;
    bool ordered;           // allocated stream-ordered (scene_upload_on)
};

namespace merf {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(MERF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_error.clear(); }

}  // namespace merf

namespace {

constexpr uint32_t kMagic = 0x4d455246u;  // "MERF"

std::mutex g_mutex;
std::unordered_set<merf_scene *> g_live;
size_t g_budget = SIZE_MAX;
size_t g_in_use = 0;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool live(merf_scene *s) {
    std::lock_guard<std::mutex> lk(g_mutex);
    return s && g_live.count(s) && s->magic == kMagic;
}

int validate_desc(const merf_scene_desc *d) {
    if (!d) return fail(MERF_E_INVALID, "scene descriptor is NULL");
    if (d->struct_size != sizeof(merf_scene_desc))
        return fail(MERF_E_INVALID, "struct_size %u != sizeof(merf_scene_desc) %zu", d->struct_size,
                    sizeof(merf_scene_desc));
    if (d->block_size != kBlock) return fail(MERF_E_INVALID, "block_size must be %d (got %d)", kBlock, d->block_size);
    if (d->channels != kChannels) return fail(MERF_E_INVALID, "channels must be %d (got %d)", kChannels, d->channels);
    // grid_res = 0: planes only (no 3D grid); plane_res = 0: sparse grid only
    if (d->grid_res != 0 && (d->grid_res < 2 * kBlock || d->grid_res % kBlock != 0 || d->grid_res > 4096))
        return fail(MERF_E_INVALID, "grid_res %d must be 0 or a multiple of 8 in [16, 4096]", d->grid_res);
    if (d->grid_res == 0 && d->plane_res == 0) return fail(MERF_E_INVALID, "scene has neither grid nor planes");
    // the kernels address every array with 32-bit byte offsets
    if (d->plane_res != 0 && (d->plane_res < 2 || d->plane_res > 8192))
        return fail(MERF_E_INVALID, "plane_res %d must be 0 or in [2, 8192]", d->plane_res);
    const int64_t nbl = d->grid_res / kBlock;
    if (d->num_blocks < 0 || d->num_blocks > nbl * nbl * nbl)
        return fail(MERF_E_INVALID, "num_blocks %d out of range", d->num_blocks);
    if (nbl > 0 && !d->block_index) return fail(MERF_E_INVALID, "block_index is NULL");
    if (d->num_blocks > 0 && !d->blocks) return fail(MERF_E_INVALID, "blocks is NULL");
    if (d->plane_res > 0 && !d->planes) return fail(MERF_E_INVALID, "planes is NULL");
    if (d->occ_levels < 1 || d->occ_levels > MERF_MAX_OCC_LEVELS)
        return fail(MERF_E_INVALID, "occ_levels %d must be in [1, %d]", d->occ_levels, MERF_MAX_OCC_LEVELS);
    for (int l = 0; l < d->occ_levels; ++l) {
        if (d->occ_res[l] < 1 || d->occ_res[l] > 1024)
            return fail(MERF_E_INVALID, "occ_res[%d] = %d must be in [1, 1024]", l, d->occ_res[l]);
        if (!d->occ[l]) return fail(MERF_E_INVALID, "occ[%d] is NULL", l);
        // coarse to fine, each level refining the previous one (a max-pool
        // pyramid), so every cell of the finest level lies in one cell of each
        if (l > 0 && d->occ_res[l] % d->occ_res[l - 1] != 0)
            return fail(MERF_E_INVALID, "occ_res[%d] = %d is not a multiple of occ_res[%d] = %d", l, d->occ_res[l],
                        l - 1, d->occ_res[l - 1]);
    }
    if (!(d->m_density > 0.0f) || !(d->m_feature > 0.0f) || !std::isfinite(d->m_density) ||
        !std::isfinite(d->m_feature))
        return fail(MERF_E_INVALID, "m_density / m_feature must be positive and finite");
    if (d->mlp_in != kMlpIn || d->mlp_hidden != kMlpHidden)
        return fail(MERF_E_INVALID, "MLP must be %d -> %d -> %d -> 3 (got in=%d hidden=%d)", kMlpIn, kMlpHidden,
                    kMlpHidden, d->mlp_in, d->mlp_hidden);
    if (!d->mlp_params) return fail(MERF_E_INVALID, "mlp_params is NULL");
    const int64_t nidx = nbl * nbl * nbl;
    std::vector<uint8_t> seen((size_t)std::max(d->num_blocks, 1), 0);
    for (int64_t i = 0; i < nidx; ++i) {
        int32_t b = d->block_index[i];
        if (b < -1 || b >= d->num_blocks)
            return fail(MERF_E_INVALID, "block_index[%lld] = %d out of [-1, %d)", (long long)i, b, d->num_blocks);
        if (b >= 0) {
            if (seen[(size_t)b]) return fail(MERF_E_INVALID, "block slot %d referenced twice", b);
            seen[(size_t)b] = 1;
        }
    }
    return MERF_OK;
}

// A brick is needed at block position b when any of the 8 blocks b + {0,1}^3
// is stored.
int64_t count_bricks(const merf_scene_desc *d) {
    const int nbl = d->grid_res / kBlock;
    auto stored = [&](int bx, int by, int bz) {
        return bx < nbl && by < nbl && bz < nbl && d->block_index[((size_t)bz * nbl + by) * nbl + bx] >= 0;
    };
    int64_t n = 0;
    for (int bz = 0; bz < nbl; ++bz)
        for (int by = 0; by < nbl; ++by)
            for (int bx = 0; bx < nbl; ++bx) {
                bool need = false;
                for (int dz = 0; dz < 2 && !need; ++dz)
                    for (int dy = 0; dy < 2 && !need; ++dy)
                        for (int dx = 0; dx < 2 && !need; ++dx) need = stored(bx + dx, by + dy, bz + dz);
                n += need ? 1 : 0;
            }
    return n;
}

// Offsets of the arrays inside a scene's single device allocation.
struct Layout {
    size_t bidx, bricks, planes, occ[kMaxLevels], dist, mlp, total;
};

// A scene without a grid gets a one-entry index (pointing at the zero brick);
// one without planes gets zero 2x2 stand-in planes.
Layout make_layout(const merf_scene_desc *d, int64_t nbricks) {
    const size_t nbl = (size_t)(d->grid_res / kBlock), R = d->plane_res > 0 ? (size_t)d->plane_res : 2;
    Layout o{};
    size_t off = 0;
    o.bidx = off; off = align_up(off + std::max<size_t>(nbl * nbl * nbl, 1) * sizeof(int32_t), 256);
    o.bricks = off; off = align_up(off + (size_t)(nbricks + 1) * kBrickBytes, 256);
    o.planes = off; off = align_up(off + 3 * R * R * kChannels, 256);
    for (int l = 0; l < d->occ_levels; ++l) {
        const size_t r = (size_t)d->occ_res[l];
        o.occ[l] = off;
        off = align_up(off + r * r * r, 256);
    }
    const size_t rf = (size_t)d->occ_res[d->occ_levels - 1];
    o.dist = off; off = align_up(off + (rf <= (size_t)kOctMaxRes ? 8 : 1) * rf * rf * rf, 256);
    o.mlp = off; off = align_up(off + kMlpParams * sizeof(float), 256);
    o.total = off;
    return o;
}

// Bricks with a one-voxel apron: brick (bx, by, bz) holds voxels 8b .. 8b+8 of
// each axis.  A brick is stored when any of the 8 blocks it touches is stored;
// all other index entries point at one shared all-zero brick (the last).
// The host only assigns the slots; the device packs the voxels.
void assign_bricks(const merf_scene_desc *d, std::vector<int32_t> &bidx, std::vector<int32_t> &pos) {
    const int nbl = d->grid_res / kBlock;
    auto stored = [&](int bx, int by, int bz) {
        return bx < nbl && by < nbl && bz < nbl && d->block_index[((size_t)bz * nbl + by) * nbl + bx] >= 0;
    };
    bidx.assign((size_t)nbl * nbl * nbl, -1);
    pos.clear();
    for (int bz = 0; bz < nbl; ++bz)
        for (int by = 0; by < nbl; ++by)
            for (int bx = 0; bx < nbl; ++bx) {
                bool need = false;
                for (int dz = 0; dz < 2 && !need; ++dz)
                    for (int dy = 0; dy < 2 && !need; ++dy)
                        for (int dx = 0; dx < 2 && !need; ++dx) need = stored(bx + dx, by + dy, bz + dz);
                if (need) {
                    bidx[((size_t)bz * nbl + by) * nbl + bx] = (int32_t)pos.size();
                    pos.push_back(bx | (by << 10) | (bz << 20));
                }
            }
    const int32_t zero = (int32_t)pos.size();
    for (int32_t &b : bidx)
        if (b < 0) b = zero;
    if (bidx.empty()) bidx.push_back(zero);   // stand-in grid of a planes-only scene
}

}  // namespace

namespace merf {

const DevScene *scene_dev(merf_scene_t s) { return live(s) ? &s->ds : nullptr; }

size_t scene_device_bytes(const merf_scene_desc *desc) {
    if (validate_desc(desc) != MERF_OK) return 0;
    return make_layout(desc, count_bricks(desc)).total;
}

namespace {

// Work buffers of the tile order (cost keys, their group counts and the
// order, for up to kOrderMaxTiles tiles).  The prepass runs on a stream of
// the library's own (one per device), since it reads only the resident scene
// and these buffers: it need not wait for the caller's earlier work, so it
// overlaps the previous frame's render.  The caller's stream waits for its
// event `ready`.  A buffer is free again once the event `done`, recorded
// after the render that read it, has completed; the host checks that, so no
// device queue ever waits on the caller's stream (a device-side wait there
// cost about 10 us per frame).  A device has at most kOrderBufs buffers; when
// all are in flight, the call waits on the host for the oldest.  Buffers and
// streams are held until the process ends.
struct OrderBuf {
    int device;
    uint8_t *keys;
    uint32_t *group_counts;
    int32_t *order;
    hipEvent_t ready, done;
    uint64_t last_use;                           // 0: not used yet
};
constexpr int kOrderBufs = 64;
// The events order device work only (the host merely asks whether a buffer
// is free), so they skip the system-scope cache flush of an event record.
constexpr unsigned kOrderEventFlags = hipEventDisableTiming | hipEventDisableSystemFence;
std::mutex g_order_mutex;
std::vector<OrderBuf> g_order_bufs;
std::vector<std::pair<int, hipStream_t>> g_order_streams;
uint64_t g_order_uses = 0;

// The library's prepass stream of a device, or null (caller holds g_order_mutex).
hipStream_t order_stream(int device) {
    for (auto &ds : g_order_streams)
        if (ds.first == device) return ds.second;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_order_streams.emplace_back(device, st);
    return st;
}

// Index of a free buffer of the device, or -1 (caller holds g_order_mutex).
int order_buffer(int device) {
    int n = 0;
    for (int i = 0; i < (int)g_order_bufs.size(); ++i) {
        const OrderBuf &b = g_order_bufs[i];
        if (b.device != device) continue;
        ++n;
        if (b.last_use == 0 || hipEventQuery(b.done) == hipSuccess) return i;
    }
    if (n < kOrderBufs) {
        OrderBuf b{device, nullptr, nullptr, nullptr, nullptr, nullptr, 0};
        if (hipMalloc(&b.keys, kOrderMaxTiles) == hipSuccess &&
            hipMalloc(&b.group_counts, sizeof(uint32_t) * (kOrderMaxTiles / 16)) == hipSuccess &&
            hipMalloc(&b.order, sizeof(int32_t) * kOrderMaxTiles) == hipSuccess &&
            hipEventCreateWithFlags(&b.ready, kOrderEventFlags) == hipSuccess &&
            hipEventCreateWithFlags(&b.done, kOrderEventFlags) == hipSuccess) {
            g_order_bufs.push_back(b);
            return (int)g_order_bufs.size() - 1;
        }
        if (b.keys) (void)hipFree(b.keys);
        if (b.group_counts) (void)hipFree(b.group_counts);
        if (b.order) (void)hipFree(b.order);
        if (b.ready) (void)hipEventDestroy(b.ready);
    }
    // every buffer of the device is in flight: the launch keeps the plain
    // order (the same image) rather than blocking the caller on the oldest
    return -1;
}

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

}  // namespace

int render_launch(const DevScene &ds, RenderBatch &rb, int tile_order, hipStream_t stream, int32_t *order_out,
                  hipEvent_t ev_start, hipEvent_t ev_end) {
    std::unique_lock<std::mutex> lock(g_order_mutex, std::defer_lock);
    int buf = -1;
    if (tile_order == 0 && rb.total_tiles >= kOrderMinTiles && rb.total_tiles <= kOrderMaxTiles &&
        !capturing(stream)) {
        lock.lock();
        // the work buffers are allocated on the current device: order only
        // when the stream belongs to it
        int device = -1;
        hipDevice_t sdev = -1;
        const bool same = hipGetDevice(&device) == hipSuccess &&
                          (!stream || (hipStreamGetDevice(stream, &sdev) == hipSuccess && sdev == device));
        hipStream_t ps = same ? order_stream(device) : nullptr;
        if (ps) buf = order_buffer(device);
        // a not-ready event query is no error (leave any other error alone)
        if (hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
        if (buf >= 0) {
            const OrderBuf &b = g_order_bufs[buf];
            hipError_t e = launch_tile_order(ds, rb, b.keys, b.group_counts, b.order, ps);
            if (e == hipSuccess) e = hipEventRecord(b.ready, ps);
            if (e == hipSuccess) e = hipStreamWaitEvent(stream, b.ready, 0);
            if (e != hipSuccess) return hip_fail(e, "tile order");
            rb.order = b.order;
        }
    }
    hipError_t e = ev_start ? hipEventRecord(ev_start, stream) : hipSuccess;
    if (e != hipSuccess) return hip_fail(e, "start event");
    e = launch_render(ds, rb, stream);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    const char *what = nullptr;
    if (ev_end && (e = hipEventRecord(ev_end, stream)) != hipSuccess) what = "end event";
    if (!what && order_out) {
        e = rb.order ? hipMemcpyAsync(order_out, rb.order, sizeof(int32_t) * (size_t)rb.total_tiles,
                                      hipMemcpyDeviceToDevice, stream)
                     : launch_identity_order(order_out, rb.total_tiles, stream);
        if (e != hipSuccess) what = "tile order copy";
    }
    if (buf >= 0) {
        // after everything that reads the buffer on this stream, errors or not
        OrderBuf &b = g_order_bufs[buf];
        const hipError_t ed = hipEventRecord(b.done, stream);
        if (ed == hipSuccess) {
            b.last_use = ++g_order_uses;
        } else {
            // without its event the buffer cannot be known free again
            b.device = -1;
            if (!what) {
                e = ed;
                what = "tile order event";
            }
        }
    }
    return what ? hip_fail(e, what) : MERF_OK;
}

int check_params(const merf_render_params *p, int res, float *step_out) {
    if (!p) return fail(MERF_E_INVALID, "render params are NULL");
    if (p->struct_size != sizeof(merf_render_params))
        return fail(MERF_E_INVALID, "params struct_size %u != %zu", p->struct_size, sizeof(merf_render_params));
    const float step = p->step > 0.0f ? p->step : 4.0f / (float)res;
    if (!std::isfinite(step) || step < 1e-6f) return fail(MERF_E_INVALID, "step %g out of range", (double)p->step);
    if (!(p->t_min >= 0.0f && p->t_min < 1.0f)) return fail(MERF_E_INVALID, "t_min %g not in [0, 1)", (double)p->t_min);
    if (p->delta_mode != 0 && p->delta_mode != 1) return fail(MERF_E_INVALID, "delta_mode %d", p->delta_mode);
    if (p->mlp_prec < 0 || p->mlp_prec > 2) return fail(MERF_E_INVALID, "mlp_prec %d not in {0, 1, 2}", p->mlp_prec);
    if (p->feat_prec < 0 || p->feat_prec > 2) return fail(MERF_E_INVALID, "feat_prec %d not in {0, 1, 2}", p->feat_prec);
    if (p->skip_mode != 0 && p->skip_mode != 1) return fail(MERF_E_INVALID, "skip_mode %d not in {0, 1}", p->skip_mode);
    if (p->tile_order != 0 && p->tile_order != 1)
        return fail(MERF_E_INVALID, "tile_order %d not in {0, 1}", p->tile_order);
    *step_out = step;
    return MERF_OK;
}

int check_camera(const merf_camera &c, int i) {
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
        return fail(MERF_E_INVALID, "camera %d: size %dx%d out of range", i, c.width, c.height);
    bool ok = std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy) &&
              c.fx != 0.0f && c.fy != 0.0f;
    for (int k = 0; k < 12; ++k) ok = ok && std::isfinite(c.c2w[k]);
    if (!ok) return fail(MERF_E_INVALID, "camera %d: non-finite or zero intrinsics / pose", i);
    return MERF_OK;
}

void begin_batch(RenderBatch &rb, const merf_render_params &p, float step) {
    std::memset(&rb, 0, sizeof rb);
    rb.step = step;
    rb.inv_step = 1.0f / step;
    rb.t_min = p.t_min;
    rb.delta_mode = p.delta_mode;
    rb.mlp_prec = p.mlp_prec;
    rb.feat_prec = p.feat_prec;
    rb.skip_mode = p.skip_mode;
    rb.stats = reinterpret_cast<unsigned long long *>(p.stats_dev);
}

bool add_camera(RenderBatch &rb, const merf_camera &c, float *out) {
    if (rb.n_cams >= kCamsPerLaunch) return false;
    const int tiles_x = (c.width + kTile - 1) / kTile;
    const int64_t tiles = (int64_t)rb.total_tiles + (int64_t)tiles_x * ((c.height + kTile - 1) / kTile);
    if (tiles > INT32_MAX) return false;
    DevCamera &dc = rb.cams[rb.n_cams++];
    std::memcpy(dc.c2w, c.c2w, sizeof dc.c2w);
    dc.fx = c.fx; dc.fy = c.fy; dc.cx = c.cx; dc.cy = c.cy;
    dc.inv_fx = 1.0f / c.fx;
    dc.inv_fy = 1.0f / c.fy;
    dc.width = c.width; dc.height = c.height;
    dc.tiles_x = tiles_x;
    dc.tile_start = rb.total_tiles;
    dc.out = out;
    rb.total_tiles = (int32_t)tiles;
    return true;
}

}  // namespace merf

extern "C" {

const char *merf_last_error(void) { return merf::g_error.c_str(); }

int merf_set_hbm_budget(size_t bytes) {
    std::lock_guard<std::mutex> lk(g_mutex);
    g_budget = bytes;
    return MERF_OK;
}

size_t merf_hbm_in_use(void) {
    std::lock_guard<std::mutex> lk(g_mutex);
    return g_in_use;
}

size_t merf_scene_bytes(merf_scene_t s) { return live(s) ? s->dev_bytes : 0; }

}  // extern "C"

namespace {

// Device allocation of an upload: plain (hipMalloc / hipFree, which waits for
// the device) or stream-ordered on `stream` (hipMallocAsync / hipFreeAsync,
// which wait for nothing but that stream's earlier work).
hipError_t dev_alloc(void **p, size_t n, bool ordered, hipStream_t stream) {
    return ordered ? hipMallocAsync(p, n, stream) : hipMalloc(p, n);
}
hipError_t dev_free(void *p, bool ordered, hipStream_t stream) {
    return ordered ? hipFreeAsync(p, stream) : hipFree(p);
}

// merf_scene_upload (ordered = false: null stream, plain allocation) and
// scene_upload_on (ordered = true: everything on stream).
int upload_impl(const merf_scene_desc *desc, merf_scene_t *out, bool ordered, hipStream_t stream) {
    clear_error();
    if (!out) return fail(MERF_E_INVALID, "output handle pointer is NULL");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (!ordered) stream = nullptr;

    const int64_t nbricks = count_bricks(desc);
    if ((nbricks + 1) * (int64_t)kBrickBytes >= (int64_t)1 << 31)
        return fail(MERF_E_INVALID, "%lld bricks exceed the 2 GiB addressed by 32-bit offsets", (long long)nbricks);
    std::vector<int32_t> bidx, bpos;
    assign_bricks(desc, bidx, bpos);
    const int L = desc->grid_res, R = desc->plane_res, nbl = L / kBlock;
    const Layout lay = make_layout(desc, nbricks);
    const size_t o_bidx = lay.bidx, o_bricks = lay.bricks, o_planes = lay.planes, o_mlp = lay.mlp, total = lay.total;
    const size_t *o_occ = lay.occ;

    {
        std::lock_guard<std::mutex> lk(g_mutex);
        if (g_in_use + total > g_budget)
            return fail(MERF_E_OOM, "scene needs %zu device bytes; %zu in use, budget %zu", total, g_in_use, g_budget);
        g_in_use += total;    // reserve; released below on failure
    }
    auto release = [&]() {
        std::lock_guard<std::mutex> lk(g_mutex);
        g_in_use -= total;
    };

    // resident allocation + staging for the raw blocks, their index and the
    // brick positions (freed once the bricks are packed)
    const size_t raw_blocks = (size_t)desc->num_blocks * kBlock * kBlock * kBlock * kChannels;
    const size_t s_blocks = 0, s_index = align_up(std::max<size_t>(raw_blocks, 8), 256),
                 s_pos = s_index + align_up((size_t)nbl * nbl * nbl * sizeof(int32_t), 256),
                 s_dist0 = s_pos + align_up(std::max<size_t>(bpos.size(), 1) * sizeof(int32_t), 256);
    const size_t rf = (size_t)desc->occ_res[desc->occ_levels - 1], nf = rf * rf * rf;
    const bool octants = rf <= (size_t)kOctMaxRes;
    // distance scratch: seed + second byte grid, or seed + int32 prefix sums
    const size_t s_dist1 = s_dist0 + align_up(nf, 256),
                 staging = s_dist1 + align_up(octants ? nf * sizeof(int32_t) : nf, 256);
    void *base = nullptr, *stage = nullptr;
    hipError_t e = dev_alloc(&base, total, ordered, stream);
    if (e == hipSuccess) e = dev_alloc(&stage, staging, ordered, stream);
    if (e == hipSuccess && ordered) e = hipStreamSynchronize(stream);   // allocation failures surface here
    if (e != hipSuccess || !base || !stage) {
        (void)hipGetLastError();
        if (base) (void)dev_free(base, ordered, stream);
        if (base && ordered) (void)hipStreamSynchronize(stream);
        release();
        return fail(MERF_E_OOM, "hipMalloc (%zu + %zu staging bytes) failed: %s", total, staging, hipGetErrorString(e));
    }
    auto dev = [&](size_t o) { return static_cast<uint8_t *>(base) + o; };
    auto stg = [&](size_t o) { return static_cast<uint8_t *>(stage) + o; };
    struct Copy { uint8_t *dst; const void *src; size_t n; };
    std::vector<Copy> copies = {
        {dev(o_bidx), bidx.data(), bidx.size() * sizeof(int32_t)},
        {dev(o_planes), desc->planes, (size_t)3 * R * R * kChannels},
        {dev(o_mlp), desc->mlp_params, kMlpParams * sizeof(float)},
        {stg(s_blocks), desc->blocks, raw_blocks},
        {stg(s_index), desc->block_index, (size_t)nbl * nbl * nbl * sizeof(int32_t)},
        {stg(s_pos), bpos.data(), bpos.size() * sizeof(int32_t)},
    };
    for (int l = 0; l < desc->occ_levels; ++l) {
        size_t r = (size_t)desc->occ_res[l];
        copies.push_back({dev(o_occ[l]), desc->occ[l], r * r * r});
    }
    for (const Copy &c : copies) {
        if (c.n == 0) continue;
        // hipMemcpyDefault: blocks, planes, occupancy levels and MLP may be
        // host or device memory (e.g. a pyramid built by merf_occupancy_pyramid)
        e = ordered ? hipMemcpyAsync(c.dst, c.src, c.n, hipMemcpyDefault, stream)
                    : hipMemcpy(c.dst, c.src, c.n, hipMemcpyDefault);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess && R == 0) e = hipMemsetAsync(dev(o_planes), 0, (size_t)3 * 2 * 2 * kChannels, stream);
    if (e == hipSuccess)
        e = launch_pack_bricks(stg(s_blocks), reinterpret_cast<const int32_t *>(stg(s_index)),
                               reinterpret_cast<const int32_t *>(stg(s_pos)), (int)nbricks, L, dev(o_bricks), stream);
    if (e == hipSuccess) {
        OccLevels lv{};
        lv.n = desc->occ_levels;
        for (int l = 0; l < lv.n; ++l) {
            lv.occ[l] = dev(o_occ[l]);
            lv.res[l] = desc->occ_res[l];
        }
        e = octants ? launch_octant_extents(lv, stg(s_dist0), reinterpret_cast<int32_t *>(stg(s_dist1)),
                                            dev(lay.dist), stream)
                    : launch_distance_grid(lv, stg(s_dist0), stg(s_dist1), dev(lay.dist), stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)dev_free(stage, ordered, stream);
    if (e != hipSuccess) {
        (void)dev_free(base, ordered, stream);
        if (ordered) (void)hipStreamSynchronize(stream);
        release();
        return hip_fail(e, "scene upload");
    }

    merf_scene *s = new merf_scene();
    s->magic = kMagic;
    s->dev_base = base;
    s->dev_bytes = total;
    s->nbricks = (int32_t)nbricks;
    s->ordered = ordered;
    DevScene &ds = s->ds;
    ds.brick_index = reinterpret_cast<const int32_t *>(dev(o_bidx));
    ds.bricks = dev(o_bricks);
    ds.planes = dev(o_planes);
    for (int l = 0; l < kMaxLevels; ++l) {
        ds.occ[l] = l < desc->occ_levels ? dev(o_occ[l]) : nullptr;
        ds.occ_res[l] = l < desc->occ_levels ? desc->occ_res[l] : 1;
        ds.occ_cell[l] = 4.0f / (float)ds.occ_res[l];
    }
    ds.dist = dev(lay.dist);
    ds.dist_res = (int32_t)rf;
    ds.dist_oct_stride = octants ? (uint32_t)nf : 0u;
    ds.dist_cell = 4.0f / (float)rf;
    ds.mlp = reinterpret_cast<const float *>(dev(o_mlp));
    ds.L = L > 0 ? L : kBlock;            // stand-ins, see DevScene
    ds.R = R > 0 ? R : 2;
    ds.nbl = L > 0 ? nbl : 1;
    ds.nsrc = (L > 0 ? 1.0f : 0.0f) + (R > 0 ? 3.0f : 0.0f);
    ds.res = std::max(L, R);
    ds.occ_levels = desc->occ_levels;
    ds.m_density = desc->m_density;
    ds.m_feature = desc->m_feature;
    // kernel constants (after every field they derive from)
    ds.p_scale = (float)ds.R * 0.25f;
    ds.p_off = 2.0f * ds.p_scale - 0.5f;
    ds.p_max = (float)(ds.R - 1);
    ds.g_scale = (float)ds.L * 0.25f;
    ds.g_off = 2.0f * ds.g_scale - 0.5f;
    ds.g_max = (float)(ds.L - 1);
    ds.d_scale = eq8_scale(ds.m_density);
    ds.d_off = -ds.nsrc * ds.m_density;
    ds.f_scale = eq8_scale(ds.m_feature);
    ds.f_off = -ds.nsrc * ds.m_feature;
    ds.d_scale24 = ds.d_scale * 16777216.0f;     // exact: a power of two
    ds.f_scale24 = ds.f_scale * 16777216.0f;
    ds.grid_w = L > 0 ? 1.0f : 0.0f;
    ds.planes_w = R > 0 ? 1.0f : 0.0f;
    ds.dist_scale = (float)ds.dist_res * 0.25f;
    ds.dist_off = 2.0f * ds.dist_scale;
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        g_live.insert(s);
    }
    *out = s;
    return MERF_OK;
}

// Forget a live scene and return its memory to the budget; false if s is
// not live.
bool unregister(merf_scene_t s) {
    std::lock_guard<std::mutex> lk(g_mutex);
    if (!s || !g_live.count(s)) return false;
    g_live.erase(s);
    g_in_use -= s->dev_bytes;
    return true;
}

}  // namespace

namespace merf {

int scene_upload_on(const merf_scene_desc *desc, hipStream_t stream, merf_scene_t *out) {
    return upload_impl(desc, out, true, stream);
}

int scene_image_on(merf_scene_t s, void *host, size_t host_bytes, hipStream_t stream, SceneImage *img) {
    clear_error();
    if (!live(s)) return fail(MERF_E_INVALID, "scene_image_on: invalid scene handle");
    if (!img || !host || host_bytes < s->dev_bytes)
        return fail(MERF_E_INVALID, "scene_image_on: the image needs %zu host bytes", s->dev_bytes);
    hipError_t e = hipMemcpyAsync(host, s->dev_base, s->dev_bytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "scene image");
    img->ds = s->ds;
    img->base = reinterpret_cast<uintptr_t>(s->dev_base);
    img->bytes = s->dev_bytes;
    img->nbricks = s->nbricks;
    return MERF_OK;
}

int scene_from_image_on(const SceneImage &img, const void *host, hipStream_t stream, merf_scene_t *out) {
    clear_error();
    if (!out) return fail(MERF_E_INVALID, "output handle pointer is NULL");
    *out = nullptr;
    if (!host || img.bytes == 0) return fail(MERF_E_INVALID, "scene_from_image_on: empty image");
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        if (g_in_use + img.bytes > g_budget)
            return fail(MERF_E_OOM, "scene needs %zu device bytes; %zu in use, budget %zu", img.bytes, g_in_use, g_budget);
        g_in_use += img.bytes;
    }
    void *base = nullptr;
    hipError_t e = hipMallocAsync(&base, img.bytes, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(base, host, img.bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess || !base) {
        (void)hipGetLastError();
        if (base) {
            (void)hipFreeAsync(base, stream);
            (void)hipStreamSynchronize(stream);
        }
        std::lock_guard<std::mutex> lk(g_mutex);
        g_in_use -= img.bytes;
        return fail(MERF_E_OOM, "scene image of %zu bytes: %s", img.bytes, hipGetErrorString(e));
    }
    // every array keeps its offset in the allocation
    auto at = [&](const void *p) -> const uint8_t * {
        return p ? static_cast<const uint8_t *>(base) + (reinterpret_cast<uintptr_t>(p) - img.base) : nullptr;
    };
    merf_scene *s = new merf_scene();
    s->magic = kMagic;
    s->dev_base = base;
    s->dev_bytes = img.bytes;
    s->nbricks = img.nbricks;
    s->ordered = true;
    DevScene &ds = s->ds;
    ds = img.ds;
    ds.brick_index = reinterpret_cast<const int32_t *>(at(img.ds.brick_index));
    ds.bricks = at(img.ds.bricks);
    ds.planes = at(img.ds.planes);
    for (int l = 0; l < kMaxLevels; ++l) ds.occ[l] = at(img.ds.occ[l]);
    ds.dist = at(img.ds.dist);
    ds.mlp = reinterpret_cast<const float *>(at(img.ds.mlp));
    {
        std::lock_guard<std::mutex> lk(g_mutex);
        g_live.insert(s);
    }
    *out = s;
    return MERF_OK;
}

int scene_release_on(merf_scene_t s, hipStream_t stream) {
    clear_error();
    if (!unregister(s)) return fail(MERF_E_INVALID, "scene_release_on: unknown or already freed scene handle");
    const hipError_t e = dev_free(s->dev_base, s->ordered, stream);
    s->magic = 0;
    delete s;
    if (e != hipSuccess) return hip_fail(e, "scene release");
    return MERF_OK;
}

}  // namespace merf

extern "C" {

int merf_scene_upload(const merf_scene_desc *desc, merf_scene_t *out) { return upload_impl(desc, out, false, nullptr); }

int merf_free(merf_scene_t s) {
    clear_error();
    if (!unregister(s)) return fail(MERF_E_INVALID, "merf_free: unknown or already freed scene handle");
    hipError_t e1 = hipDeviceSynchronize();
    hipError_t e2 = dev_free(s->dev_base, s->ordered, nullptr);
    if (e2 == hipSuccess && s->ordered) e2 = hipStreamSynchronize(nullptr);
    s->magic = 0;
    delete s;
    if (e1 != hipSuccess) return hip_fail(e1, "hipDeviceSynchronize (merf_free)");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFree (merf_free)");
    return MERF_OK;
}

int merf_render(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                float *out_rgba_dev, void *hip_stream) {
    clear_error();
    if (!live(s)) return fail(MERF_E_INVALID, "merf_render: invalid scene handle");
    float step = 0.0f;
    int rc = check_params(p, s->ds.res, &step);
    if (rc) return rc;
    if (n_cams < 0) return fail(MERF_E_INVALID, "n_cams %d < 0", n_cams);
    if (n_cams == 0) return MERF_OK;
    if (!cams) return fail(MERF_E_INVALID, "cams is NULL");
    if (!out_rgba_dev) return fail(MERF_E_INVALID, "output buffer is NULL");
    for (int i = 0; i < n_cams; ++i)
        if ((rc = check_camera(cams[i], i))) return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    int64_t pix = 0;
    for (int first = 0; first < n_cams;) {
        RenderBatch rb;
        begin_batch(rb, *p, step);
        while (first < n_cams && add_camera(rb, cams[first], out_rgba_dev + pix * 4)) {
            pix += (int64_t)cams[first].width * cams[first].height;
            ++first;
        }
        if (rb.n_cams == 0) return fail(MERF_E_INVALID, "camera %d alone exceeds one launch", first);
        if ((rc = render_launch(s->ds, rb, p->tile_order, stream))) return rc;
    }
    return MERF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Render without allocating (merf_render_noalloc).  The tile-order work
// buffers of merf_render are hipMalloc'd on first use; here they are one fixed
// device array of this file, and every kernel runs on the caller's stream
// (no stream, event or buffer of the library's own).  Each device holds its
// own copy of the array at its own address, looked up once per device.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kFixedKeys = kOrderMaxTiles;                               // uint8 cost keys
constexpr size_t kFixedCounts = sizeof(uint32_t) * (kOrderMaxTiles / 16);   // key counts per group of 16 tiles
constexpr size_t kFixedOrder = sizeof(int32_t) * kOrderMaxTiles;            // the order
constexpr size_t kFixedBytes = kFixedKeys + kFixedCounts + kFixedOrder;     // 672 KiB
static_assert(kFixedKeys % 256 == 0 && kFixedCounts % 256 == 0, "sub-buffer alignment");

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mutex;
uint8_t *g_fixed_ptr[kMaxDevices] = {};     // device address of `scratch` per device ordinal, once looked up

}  // namespace

static __device__ __align__(256) uint8_t scratch[kFixedBytes];

namespace {

// Device address of this device's `scratch`.  The array's name is a host-side
// stand-in; kernels get this address.  Called with the device current.
int fixed_scratch(int device, uint8_t **out) {
    if (device < 0 || device >= kMaxDevices) return fail(MERF_E_INVALID, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_fixed_mutex);
    if (!g_fixed_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_fixed_ptr[device] = static_cast<uint8_t *>(p);
    }
    *out = g_fixed_ptr[device];
    return MERF_OK;
}

// Tiles of the launch that starts at camera `first` (the same packing as
// add_camera: up to kCamsPerLaunch cameras); advances first.
int64_t next_launch_tiles(const merf_camera *cams, int32_t n_cams, int &first) {
    int64_t tiles = 0;
    for (int k = 0; k < kCamsPerLaunch && first < n_cams; ++k, ++first)
        tiles += (int64_t)((cams[first].width + kTile - 1) / kTile) * ((cams[first].height + kTile - 1) / kTile);
    return tiles;
}

}  // namespace

extern "C" {

int merf_render_noalloc(merf_scene_t s, const merf_camera *cams, int32_t n_cams, const merf_render_params *p,
                        float *out_rgba_dev, void *hip_stream) {
    clear_error();
    if (!live(s)) return fail(MERF_E_INVALID, "merf_render_noalloc: invalid scene handle");
    float step = 0.0f;
    int rc = check_params(p, s->ds.res, &step);
    if (rc) return rc;
    if (n_cams < 0) return fail(MERF_E_INVALID, "n_cams %d < 0", n_cams);
    if (n_cams == 0) return MERF_OK;
    if (!cams) return fail(MERF_E_INVALID, "cams is NULL");
    if (!out_rgba_dev) return fail(MERF_E_INVALID, "output buffer is NULL");
    for (int i = 0; i < n_cams; ++i)
        if ((rc = check_camera(cams[i], i))) return rc;
    // every launch that would run in tile order must fit the fixed buffers;
    // checked before anything is launched
    const bool ordered = p->tile_order == 0;
    if (ordered) {
        for (int first = 0; first < n_cams;) {
            const int at = first;
            const int64_t tiles = next_launch_tiles(cams, n_cams, first);
            if (tiles > kOrderMaxTiles)
                return fail(MERF_E_INVALID,
                            "merf_render_noalloc: the launch of cameras %d..%d has %lld tiles, more than the "
                            "%d its fixed tile-order buffers hold (use tile_order 1 or fewer cameras per call)",
                            at, first - 1, (long long)tiles, kOrderMaxTiles);
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    int device = -1;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDevice_t sdev = device;
    if (stream && (e = hipStreamGetDevice(stream, &sdev)) != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
    if (sdev != device)
        return fail(MERF_E_INVALID, "merf_render_noalloc: the stream belongs to device %d, the current device is %d",
                    (int)sdev, device);
    uint8_t *fixed = nullptr;
    if (ordered && (rc = fixed_scratch(device, &fixed))) return rc;
    int64_t pix = 0;
    for (int first = 0; first < n_cams;) {
        RenderBatch rb;
        begin_batch(rb, *p, step);
        while (first < n_cams && add_camera(rb, cams[first], out_rgba_dev + pix * 4)) {
            pix += (int64_t)cams[first].width * cams[first].height;
            ++first;
        }
        if (rb.n_cams == 0) return fail(MERF_E_INVALID, "camera %d alone exceeds one launch", first);
        if (ordered && rb.total_tiles >= kOrderMinTiles) {
            // the prepass writes every key, group count and order entry the
            // launch reads, so nothing left by an earlier call needs clearing
            uint8_t *keys = fixed;
            uint32_t *counts = reinterpret_cast<uint32_t *>(fixed + kFixedKeys);
            int32_t *order = reinterpret_cast<int32_t *>(fixed + kFixedKeys + kFixedCounts);
            if ((e = launch_tile_order(s->ds, rb, keys, counts, order, stream)) != hipSuccess)
                return hip_fail(e, "tile order");
            rb.order = order;
        }
        if ((e = launch_render(s->ds, rb, stream)) != hipSuccess) return hip_fail(e, "render launch");
    }
    return MERF_OK;
}

int merf_dequantize(const uint8_t *codes_dev, int64_t n, float m, int32_t prec, void *out_dev, void *hip_stream) {
    clear_error();
    if (n < 0) return fail(MERF_E_INVALID, "n %lld < 0", (long long)n);
    if (n == 0) return MERF_OK;
    if (!codes_dev || !out_dev) return fail(MERF_E_INVALID, "NULL buffer");
    if (!(m > 0.0f) || !std::isfinite(m)) return fail(MERF_E_INVALID, "m %g must be positive", (double)m);
    if (prec < 0 || prec > 2) return fail(MERF_E_INVALID, "prec %d not in {0, 1, 2}", prec);
    hipError_t e = launch_dequant(codes_dev, n, m, eq8_scale(m), prec, out_dev, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "dequant launch");
    return MERF_OK;
}

int merf_occupancy_pyramid(const uint8_t *mask_dev, int32_t res, const int32_t *factors, int32_t n_levels,
                           uint8_t *const *out_dev, void *hip_stream) {
    clear_error();
    if (res < 1 || res > 2048) return fail(MERF_E_INVALID, "res %d not in [1, 2048]", res);
    if (n_levels < 1 || n_levels > 8) return fail(MERF_E_INVALID, "n_levels %d not in [1, 8]", n_levels);
    if (!mask_dev || !factors || !out_dev) return fail(MERF_E_INVALID, "NULL buffer");
    for (int l = 0; l < n_levels; ++l) {
        if (factors[l] < 1 || res % factors[l] != 0)
            return fail(MERF_E_INVALID, "factor %d does not divide res %d", factors[l], res);
        if (!out_dev[l]) return fail(MERF_E_INVALID, "out_dev[%d] is NULL", l);
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    for (int l = 0; l < n_levels; ++l) {
        hipError_t e = launch_maxpool(mask_dev, res, factors[l], out_dev[l], stream);
        if (e != hipSuccess) return hip_fail(e, "max-pool launch");
    }
    return MERF_OK;
}

namespace {

// Checks and packs the occupancy levels of the distance-grid entry points.
int occ_levels_arg(const uint8_t *const *occ_dev, const int32_t *res, int32_t n_levels, const uint8_t *out_dev,
                   OccLevels &lv) {
    if (n_levels < 1 || n_levels > kMaxLevels)
        return fail(MERF_E_INVALID, "n_levels %d not in [1, %d]", n_levels, kMaxLevels);
    if (!occ_dev || !res || !out_dev) return fail(MERF_E_INVALID, "NULL buffer");
    lv = OccLevels{};
    lv.n = n_levels;
    for (int l = 0; l < n_levels; ++l) {
        if (res[l] < 1 || res[l] > kMaxDistRes) return fail(MERF_E_INVALID, "res[%d] = %d not in [1, %d]", l, res[l], kMaxDistRes);
        if (l > 0 && res[l] % res[l - 1] != 0)
            return fail(MERF_E_INVALID, "res[%d] = %d is not a multiple of res[%d] = %d", l, res[l], l - 1, res[l - 1]);
        if (!occ_dev[l]) return fail(MERF_E_INVALID, "occ_dev[%d] is NULL", l);
        lv.occ[l] = occ_dev[l];
        lv.res[l] = res[l];
    }
    return MERF_OK;
}

}  // namespace

int merf_distance_grid(const uint8_t *const *occ_dev, const int32_t *res, int32_t n_levels, uint8_t *out_dev,
                       void *hip_stream) {
    clear_error();
    OccLevels lv;
    int rc = occ_levels_arg(occ_dev, res, n_levels, out_dev, lv);
    if (rc) return rc;
    const size_t r = (size_t)res[n_levels - 1], n = r * r * r;
    void *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, 2 * align_up(n, 256));
    if (e != hipSuccess || !tmp) {
        (void)hipGetLastError();
        return fail(MERF_E_OOM, "hipMalloc of %zu scratch bytes failed", 2 * align_up(n, 256));
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    uint8_t *t0 = static_cast<uint8_t *>(tmp), *t1 = t0 + align_up(n, 256);
    e = launch_distance_grid(lv, t0, t1, out_dev, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "distance grid");
    return MERF_OK;
}

int merf_octant_extent_grid(const uint8_t *const *occ_dev, const int32_t *res, int32_t n_levels, uint8_t *out_dev,
                            void *hip_stream) {
    clear_error();
    OccLevels lv;
    int rc = occ_levels_arg(occ_dev, res, n_levels, out_dev, lv);
    if (rc) return rc;
    const size_t r = (size_t)res[n_levels - 1], n = r * r * r;
    const size_t bytes = align_up(n, 256) + align_up(n * sizeof(int32_t), 256);
    void *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, bytes);
    if (e != hipSuccess || !tmp) {
        (void)hipGetLastError();
        return fail(MERF_E_OOM, "hipMalloc of %zu scratch bytes failed", bytes);
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    uint8_t *seed = static_cast<uint8_t *>(tmp);
    int32_t *sat = reinterpret_cast<int32_t *>(seed + align_up(n, 256));
    e = launch_octant_extents(lv, seed, sat, out_dev, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "octant extent grid");
    return MERF_OK;
}

}  // extern "C"
