// merf_serve.hip -- serving runtime declared in include/merf_serve.h.
//
// Registered scenes (host copies owned by the server) become resident in
// device memory under a byte budget: at registration when they fit, otherwise
// when a request needs them, evicting the least requested scenes that no
// earlier request needs.  When scenes are evicted, a scene's host copy after
// its first upload is the device image that upload built, so a re-admission
// is one copy and runs no kernels beside the renders.  A worker thread continuously batches waiting
// requests of resident scenes -- any scenes, any image sizes -- into
// launches of the served render kernel on several HIP streams, with a grid
// from a fixed set of classes (persistent beyond the largest); a launch reads
// its work descriptors and the scene table from device memory, so each slot
// replays one captured graph per kernel variant and grid class without
// changing it.  A loader thread admits scenes as memory frees up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "merf_internal.h"
#include "merf_serve.h"

using namespace merf;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kMaxResident = 64;             // scene table slots of a server
constexpr int kVariants = 18;                // MLP fp32 / fp16 / bf16  x  features (feat_prec 0..2)  x  skip mode
// Grid classes: 64 << 2c workgroups for c = 0 .. 6 (64 to 262144, one tile
// each), and a persistent grid of 4096 workgroups (the device's wave slots at
// four waves per SIMD) for larger launches.
constexpr int kGridClasses = 8;
constexpr int kPersistentGrid = 4096;
// time constant (seconds) of the decayed request counts that order evictions
constexpr double kHeatTau = 2.0;

enum SceneState { kAbsent = 0, kLoading, kResident };

struct Request {
    int32_t scene = 0;
    merf_camera cam{};
    merf_render_params p{};
    float step = 0.0f;
    float *out = nullptr;
    Clock::time_point t_submit, t_start, t_done;
    int status = MERF_OK;
    bool done = false;
    std::shared_ptr<std::atomic<bool>> flag;  // set with done, read by waiters without the lock
};

// A registered scene: the server's host copy of the baked scene, and its
// residency.
struct SceneEntry {
    // one host buffer, pinned if possible: the registered arrays (desc points
    // into it) until the first upload, then the device image that upload built
    void *host = nullptr;
    bool pinned = false;
    bool imaged = false;                     // host holds img's bytes
    merf_scene_desc desc{};                  // points into host while !imaged
    SceneImage img{};
    size_t need = 0;                         // device bytes of a resident copy
    int res = 1;                             // max(L, R): default step 4/res
    SceneState state = kAbsent;
    merf_scene_t h = nullptr;
    int slot = -1;                           // scene table slot while resident
    uint64_t last_used = 0;
    // requests for the scene, each decaying with time constant kHeatTau since
    // its submission (value at heat_t): the eviction order, coldest first
    double heat = 0.0;
    Clock::time_point heat_t{};
    int queued = 0, running = 0;
    bool draining = false;                   // being emptied to make room (see loader_main)
};

struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> tickets;
    ServeLaunch *staging = nullptr;          // pinned host: the next launch's descriptors
    ServeLaunch *desc_dev = nullptr;         // device copy read by the kernel
    ServeCtl *ctl_dev = nullptr;             // control block of this slot's launches
    Graph graphs[kVariants][kGridClasses];
};

}  // namespace

struct merf_server {
    merf_server_config cfg{};
    size_t budget = SIZE_MAX;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_load, cv_done;
    std::deque<uint64_t> queue;              // waiting requests, oldest first
    std::unordered_map<uint64_t, Request> reqs;
    std::map<int32_t, SceneEntry> scenes;    // node-based: entries stay put
    std::vector<Slot> slots;
    DevScene *table_dev = nullptr;           // [kMaxResident]
    bool slot_used[kMaxResident] = {};
    std::mutex load_mu;                      // serialises uploads and releases on load_stream
    hipStream_t load_stream = nullptr;
    std::thread worker, loader;
    bool stop = false;
    uint64_t next_ticket = 1, tick = 0;
    uint64_t admit_ticket = 0;               // request the loader is making room for (0: none)
    int32_t next_scene = 1;
    size_t resident = 0;                     // device bytes of resident and loading scenes
    int inflight = 0;
    std::atomic<uint64_t> arrivals{0};       // submits, read by the worker without the lock
    uint64_t epoch = 0;                      // bumped (under mu) whenever new work may have become dispatchable
    merf_server_stats st{};
};

// The worker and waiters poll for up to this long before they block: a
// blocked thread takes tens of microseconds to wake, a frame is a few hundred.
constexpr auto kSpin = std::chrono::microseconds(300);

namespace {

std::mutex g_servers_mu;
std::unordered_set<merf_server *> g_servers;

bool server_live(merf_server *s) {
    std::lock_guard<std::mutex> lk(g_servers_mu);
    return s && g_servers.count(s);
}

int variant_of(const merf_render_params &p) { return p.mlp_prec + 3 * p.feat_prec + 9 * p.skip_mode; }

// Grid of a launch of n tiles: the smallest class with a workgroup for every
// tile, or the persistent class, whose workgroups loop, for larger launches.
int grid_class(int64_t n) {
    int c = 0;
    while (c + 1 < kGridClasses && n > (int64_t)64 << (2 * c)) ++c;
    return c;
}
int grid_of_class(int c) { return c == kGridClasses - 1 ? kPersistentGrid : 64 << (2 * c); }

// A queued request may be dispatched when its scene is resident, unless the
// scene is being emptied to admit an older request's scene.
bool dispatchable(const merf_server *S, uint64_t ticket, const Request &r) {
    auto it = S->scenes.find(r.scene);
    if (it == S->scenes.end() || it->second.state != kResident) return false;
    return !(it->second.draining && S->admit_ticket && ticket > S->admit_ticket);
}

// Enqueue the slot's launch: the descriptors are copied in by the first node
// of the slot's graph for this variant and grid (captured on first use), or
// by a plain copy before a plain launch.
hipError_t launch_slot(merf_server *S, Slot &sl, const merf_render_params &p, int gclass, bool *was_graph) {
    *was_graph = false;
    const int grid = grid_of_class(gclass);
    auto enqueue = [&]() {
        hipError_t e = hipMemcpyAsync(sl.desc_dev, sl.staging, sizeof(ServeLaunch), hipMemcpyHostToDevice, sl.stream);
        // only a launch of the persistent class takes positions from the counters
        if (e == hipSuccess && gclass == kGridClasses - 1) e = launch_zero_ctl(sl.ctl_dev, sl.stream);
        if (e == hipSuccess)
            e = launch_render_served(S->table_dev, sl.desc_dev, sl.ctl_dev, p.mlp_prec, p.feat_prec, p.skip_mode, grid,
                                     sl.stream);
        return e;
    };
    if (!S->cfg.use_graphs) return enqueue();
    Graph &g = sl.graphs[variant_of(p)][gclass];
    if (!g.exec) {
        hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        const hipError_t el = enqueue();
        e = hipStreamEndCapture(sl.stream, &g.graph);
        if (el != hipSuccess) return el;
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return e;
    }
    *was_graph = true;
    return hipGraphLaunch(g.exec, sl.stream);
}

void finish_slot(merf_server *S, Slot &sl, int status) {
    const auto now = Clock::now();
    for (uint64_t t : sl.tickets) {
        auto it = S->reqs.find(t);
        if (it == S->reqs.end()) continue;
        Request &r = it->second;
        r.t_done = now;
        r.done = true;
        r.status = status;
        r.flag->store(true, std::memory_order_release);
        auto sc = S->scenes.find(r.scene);
        if (sc != S->scenes.end()) --sc->second.running;
        ++S->st.completed;
    }
    S->inflight -= (int)sl.tickets.size();
    sl.tickets.clear();
    sl.busy = false;
}

// Fuse the oldest dispatchable request with later dispatchable requests of
// the same kernel variant (any scene, any size) into one launch on slot sl.
// Returns false when no request can be dispatched.
bool dispatch(merf_server *S, Slot &sl) {
    auto head = S->queue.end();
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
        if (dispatchable(S, *it, S->reqs[*it])) {
            head = it;
            break;
        }
    if (head == S->queue.end()) return false;
    const merf_render_params hp = S->reqs[*head].p;
    ServeLaunch &L = *sl.staging;
    L.n_work = 0;
    L.total_tiles = 0;
    std::vector<uint64_t> taken;
    bool mixed = false;
    for (auto it = head; it != S->queue.end() && (int)taken.size() < S->cfg.max_batch;) {
        const uint64_t t = *it;
        Request &r = S->reqs[t];
        if (!dispatchable(S, t, r) || variant_of(r.p) != variant_of(hp)) {
            ++it;
            continue;
        }
        const int64_t tiles = (int64_t)((r.cam.width + kTile - 1) / kTile) * ((r.cam.height + kTile - 1) / kTile);
        if ((int64_t)L.total_tiles + tiles > INT32_MAX / 2) break;
        SceneEntry &se = S->scenes[r.scene];
        ServeWork &w = L.work[L.n_work++];
        RenderBatch one;                      // camera set-up shared with merf_render
        begin_batch(one, r.p, r.step);
        add_camera(one, r.cam, r.out);
        w.cam = one.cams[0];
        w.cam.tile_start = L.total_tiles;
        w.scene = se.slot;
        w.step = one.step;
        w.inv_step = one.inv_step;
        w.t_min = one.t_min;
        w.delta_mode = one.delta_mode;
        L.total_tiles += (int32_t)tiles;
        mixed = mixed || r.scene != S->reqs[taken.empty() ? t : taken[0]].scene;
        --se.queued;
        ++se.running;
        se.last_used = ++S->tick;
        taken.push_back(t);
        it = S->queue.erase(it);
    }
    const auto now = Clock::now();
    for (uint64_t t : taken) S->reqs[t].t_start = now;
    sl.tickets = taken;
    sl.busy = true;
    S->inflight += (int)taken.size();
    S->st.max_inflight = std::max(S->st.max_inflight, S->inflight);
    bool was_graph = false;
    hipError_t e = launch_slot(S, sl, hp, grid_class(L.total_tiles), &was_graph);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        finish_slot(S, sl, MERF_E_DEVICE);
        S->cv_done.notify_all();
        S->cv_load.notify_all();
        return true;
    }
    ++S->st.launches;
    if (was_graph) ++S->st.graph_launches;
    if (mixed) ++S->st.mixed_launches;
    return true;
}

void worker_main(merf_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool busy = false, finished = false;
        for (Slot &sl : S->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) {
                busy = true;
                continue;
            }
            finish_slot(S, sl, q == hipSuccess ? MERF_OK : MERF_E_DEVICE);
            finished = true;
        }
        if (finished) {
            S->cv_done.notify_all();
            S->cv_load.notify_all();          // scenes may have become evictable
        }
        bool waiting = false;                 // queued requests nothing can dispatch now
        for (Slot &sl : S->slots) {
            if (sl.busy || S->queue.empty()) continue;
            if (!dispatch(S, sl)) {
                waiting = true;
                break;
            }
            busy = busy || sl.busy;
        }
        if (S->stop && S->queue.empty() && !busy) break;
        if (!busy && (S->queue.empty() || waiting)) {
            // idle: poll for new requests for a while, then block until
            // something that may be dispatchable happens
            const uint64_t epoch = S->epoch, seen = S->arrivals.load(std::memory_order_acquire);
            lk.unlock();
            const auto t0 = Clock::now();
            while (S->arrivals.load(std::memory_order_acquire) == seen && Clock::now() - t0 < kSpin)
                std::this_thread::yield();
            lk.lock();
            S->cv_work.wait(lk, [&] { return S->epoch != epoch || S->stop; });
        } else {
            // poll completions without holding the lock
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

// Copy a scene's device view into its table slot (caller holds load_mu).
int write_table(merf_server *S, int slot, merf_scene_t h) {
    const DevScene *ds = scene_dev(h);
    if (!ds) return fail(MERF_E_INVALID, "scene table: invalid handle");
    hipError_t e = hipMemcpyAsync(S->table_dev + slot, ds, sizeof(DevScene), hipMemcpyHostToDevice, S->load_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->load_stream);
    return e == hipSuccess ? MERF_OK : hip_fail(e, "scene table");
}

int free_table_slot(merf_server *S) {
    for (int i = 0; i < kMaxResident; ++i)
        if (!S->slot_used[i]) return i;
    return -1;
}

void free_host(SceneEntry &e);

// After a scene's first upload, the server's host copy of its arrays is
// replaced by the device image that upload built.  Later admissions are then
// one host-to-device copy, which runs on a copy engine: the build kernels
// (brick packing, empty-space grids) would otherwise run again on every
// re-admission, beside the renders of the resident scenes, and slow them.
// Only a server that evicts idle scenes re-admits them, so only such a server
// keeps images.  Best effort: without host memory for the image, the arrays
// stay and every admission builds the scene again.
void keep_image(merf_server *S, SceneEntry &e, merf_scene_t h) {
    const size_t n = e.need;
    void *buf = nullptr;
    const bool pinned = hipHostMalloc(&buf, n, hipHostMallocDefault) == hipSuccess && buf;
    if (!pinned) {
        (void)hipGetLastError();
        buf = std::malloc(n);
        if (!buf) return;
    }
    SceneImage img;
    if (scene_image_on(h, buf, n, S->load_stream, &img) != MERF_OK) {
        if (pinned) (void)hipHostFree(buf);
        else std::free(buf);
        clear_error();
        return;
    }
    free_host(e);
    e.host = buf;
    e.pinned = pinned;
    e.imaged = true;
    e.img = img;
    e.desc = merf_scene_desc{};
}

// Make scene se resident: upload it (from its device image once there is
// one) and fill its table slot (caller holds load_mu, not mu; se->state is
// kLoading and its bytes are reserved).
int admit(merf_server *S, SceneEntry *se, int slot) {
    const auto t0 = Clock::now();
    merf_scene_t h = nullptr;
    const bool from_image = se->imaged;
    int rc = from_image ? scene_from_image_on(se->img, se->host, S->load_stream, &h)
                        : scene_upload_on(&se->desc, S->load_stream, &h);
    if (rc == MERF_OK && !se->imaged && S->cfg.evict_idle) keep_image(S, *se, h);   // only evictions re-admit
    if (rc == MERF_OK) rc = write_table(S, slot, h);
    const auto us = std::chrono::duration_cast<std::chrono::microseconds>(Clock::now() - t0).count();
    std::lock_guard<std::mutex> lk(S->mu);
    S->st.admission_us += (uint64_t)us;
    if (rc != MERF_OK) {
        if (h) (void)scene_release_on(h, S->load_stream);
        S->resident -= se->need;
        S->slot_used[slot] = false;
        se->state = kAbsent;
        return rc;
    }
    se->h = h;
    se->slot = slot;
    se->state = kResident;
    se->last_used = ++S->tick;
    ++S->st.admissions;
    if (from_image) ++S->st.image_admissions;
    return MERF_OK;
}

// Evict a resident scene that nothing running reads (caller holds mu; the
// device memory is released later, under load_mu, by release_evicted).
merf_scene_t evict(merf_server *S, SceneEntry &se) {
    merf_scene_t h = se.h;
    S->resident -= se.need;
    S->slot_used[se.slot] = false;
    se.h = nullptr;
    se.slot = -1;
    se.state = kAbsent;
    se.draining = false;
    ++S->st.evictions;
    return h;
}

int release_evicted(merf_server *S, const std::vector<merf_scene_t> &hs) {
    int rc = MERF_OK;
    for (merf_scene_t h : hs)
        if (scene_release_on(h, S->load_stream) != MERF_OK) rc = MERF_E_DEVICE;
    if (!hs.empty() && hipStreamSynchronize(S->load_stream) != hipSuccess) rc = MERF_E_DEVICE;
    return rc;
}

// Fail every queued request of scene id (its admission failed).
void fail_queued(merf_server *S, int32_t id, int status) {
    const auto now = Clock::now();
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        Request &r = S->reqs[*it];
        if (r.scene != id) {
            ++it;
            continue;
        }
        r.t_start = r.t_done = now;
        r.done = true;
        r.status = status;
        r.flag->store(true, std::memory_order_release);
        --S->scenes[id].queued;
        ++S->st.completed;
        it = S->queue.erase(it);
    }
}

double heat_at(const SceneEntry &e, Clock::time_point now) {
    const double dt = std::chrono::duration<double>(now - e.heat_t).count();
    return e.heat * std::exp(-std::max(dt, 0.0) / kHeatTau);
}

// Admission by memory.  The oldest waiting request whose scene is absent
// gets its scene loaded as soon as the budget allows.  Room is made by
// evicting resident scenes that no request older than it needs, least
// requested first (request counts decayed over kHeatTau seconds, then least
// recently used): with a skewed popularity, the tail of rarely requested
// scenes takes turns in the memory left over while the popular ones stay.
// Victims still running are first drained: they take no newer requests until
// they are evicted.  Requests older than the waiting one keep being served,
// so every request is eventually admitted.
void loader_main(merf_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        // the oldest waiting request of an absent scene
        uint64_t want = 0;
        SceneEntry *se = nullptr;
        int32_t want_id = 0;
        for (uint64_t t : S->queue) {
            const Request &r = S->reqs[t];
            auto it = S->scenes.find(r.scene);
            if (it != S->scenes.end() && it->second.state == kAbsent) {
                want = t;
                se = &it->second;
                want_id = r.scene;
                break;
            }
        }
        if (!se) {
            bool freed = S->admit_ticket != 0;
            S->admit_ticket = 0;
            for (auto &kv : S->scenes) {
                freed = freed || kv.second.draining;
                kv.second.draining = false;
            }
            if (freed) {                               // drained scenes take requests again
                ++S->epoch;
                S->cv_work.notify_all();
            }
            if (S->stop) break;
            S->cv_load.wait(lk);
            continue;
        }
        S->admit_ticket = want;
        const int slot = free_table_slot(S);
        std::vector<merf_scene_t> evicted;
        if (S->resident + se->need > S->budget || slot < 0) {
            if (!S->cfg.evict_idle) {                 // only removals free memory
                if (S->stop) {                        // none will come: fail the scene's requests
                    fail_queued(S, want_id, fail(MERF_E_OOM, "scene %d does not fit the budget", want_id));
                    S->cv_done.notify_all();
                    continue;
                }
                S->cv_load.wait(lk);
                continue;
            }
            // candidates: resident scenes no request older than `want` needs
            // (the queue is in ticket order, so a scene's first waiting
            // request decides), least requested first
            std::unordered_map<int32_t, uint64_t> first_wait;
            for (uint64_t t : S->queue) first_wait.emplace(S->reqs[t].scene, t);
            struct Cand {
                double heat;
                uint64_t last_used;
                SceneEntry *e;
            };
            const auto now = Clock::now();
            std::vector<Cand> order;
            for (auto &kv : S->scenes) {
                SceneEntry &e = kv.second;
                if (e.state != kResident) continue;
                auto fw = first_wait.find(kv.first);
                if (fw == first_wait.end() || fw->second > want) order.push_back({heat_at(e, now), e.last_used, &e});
            }
            std::sort(order.begin(), order.end(), [](const Cand &a, const Cand &b) {
                return a.heat != b.heat ? a.heat < b.heat : a.last_used < b.last_used;
            });
            std::vector<SceneEntry *> cand;
            for (const Cand &c : order) cand.push_back(c.e);
            size_t room = S->budget - std::min(S->budget, S->resident);
            bool slot_ok = slot >= 0;
            std::vector<SceneEntry *> victims;
            for (SceneEntry *e : cand) {
                if (room >= se->need && slot_ok) break;
                victims.push_back(e);
                room += e->need;
                slot_ok = true;
            }
            bool ready = room >= se->need && slot_ok;
            for (SceneEntry *e : victims) ready = ready && e->running == 0;
            if (!ready) {
                for (SceneEntry *e : victims) e->draining = true;
                S->cv_load.wait(lk);
                continue;
            }
            for (SceneEntry *e : victims) evicted.push_back(evict(S, *e));
        }
        const int use = slot >= 0 ? slot : free_table_slot(S);
        S->slot_used[use] = true;
        S->resident += se->need;
        se->state = kLoading;
        lk.unlock();
        int rc;
        {
            std::lock_guard<std::mutex> ll(S->load_mu);
            rc = release_evicted(S, evicted);
            if (rc == MERF_OK) rc = admit(S, se, use);
        }
        lk.lock();
        if (rc != MERF_OK) {
            fail_queued(S, want_id, rc);
            S->cv_done.notify_all();
        }
        S->admit_ticket = 0;
        for (auto &kv : S->scenes) kv.second.draining = false;
        ++S->epoch;
        S->cv_work.notify_all();
    }
}

void free_host(SceneEntry &e) {
    if (!e.host) return;
    if (e.pinned) (void)hipHostFree(e.host);
    else std::free(e.host);
    e.host = nullptr;
    e.imaged = false;
}

// The server's host copy of a scene descriptor's arrays, in one buffer:
// pinned memory when it can be had (uploads are then plain DMA), else
// pageable.  The arrays may be host or device memory, except block_index
// (host).  Returns false if no memory could be had or a copy failed.
bool copy_scene(const merf_scene_desc *d, SceneEntry &e) {
    const size_t nbl = (size_t)(d->grid_res / 8);
    const size_t n_idx = nbl * nbl * nbl * sizeof(int32_t);
    const size_t n_blk = (size_t)d->num_blocks * 8 * 8 * 8 * (size_t)d->channels;
    const size_t n_pl = (size_t)3 * d->plane_res * d->plane_res * (size_t)d->channels;
    size_t n_occ[MERF_MAX_OCC_LEVELS] = {};
    for (int l = 0; l < d->occ_levels; ++l) n_occ[l] = (size_t)d->occ_res[l] * d->occ_res[l] * d->occ_res[l];
    const size_t n_mlp = ((size_t)d->mlp_in * d->mlp_hidden + d->mlp_hidden + (size_t)d->mlp_hidden * d->mlp_hidden +
                          d->mlp_hidden + (size_t)d->mlp_hidden * 3 + 3) * sizeof(float);
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t total = up(n_idx) + up(n_blk) + up(n_pl) + up(n_mlp);
    for (int l = 0; l < d->occ_levels; ++l) total += up(n_occ[l]);
    e.pinned = hipHostMalloc(&e.host, total, hipHostMallocDefault) == hipSuccess && e.host;
    if (!e.pinned) {
        (void)hipGetLastError();
        e.host = std::malloc(total);
        if (!e.host) return false;
    }
    uint8_t *at = static_cast<uint8_t *>(e.host);
    bool ok = true;
    auto put = [&](const void *src, size_t n) -> uint8_t * {   // src: host or device memory
        uint8_t *dst = at;
        if (n) ok = ok && hipMemcpy(dst, src, n, hipMemcpyDefault) == hipSuccess;
        at += up(n);
        return dst;
    };
    e.desc = *d;
    e.desc.block_index = reinterpret_cast<const int32_t *>(put(d->block_index, n_idx));
    e.desc.blocks = n_blk ? put(d->blocks, n_blk) : nullptr;
    e.desc.planes = n_pl ? put(d->planes, n_pl) : nullptr;
    for (int l = 0; l < MERF_MAX_OCC_LEVELS; ++l) e.desc.occ[l] = l < d->occ_levels ? put(d->occ[l], n_occ[l]) : nullptr;
    e.desc.mlp_params = reinterpret_cast<const float *>(put(d->mlp_params, n_mlp));
    e.res = std::max(std::max(d->grid_res, d->plane_res), 1);
    if (!ok) {
        (void)hipGetLastError();
        free_host(e);
    }
    return ok;
}

void destroy_slots(merf_server *S) {
    for (Slot &sl : S->slots) {
        for (auto &row : sl.graphs)
            for (Graph &g : row) {
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
                if (g.graph) (void)hipGraphDestroy(g.graph);
            }
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.desc_dev) (void)hipFree(sl.desc_dev);
        if (sl.ctl_dev) (void)hipFree(sl.ctl_dev);
    }
    if (S->table_dev) (void)hipFree(S->table_dev);
    if (S->load_stream) (void)hipStreamDestroy(S->load_stream);
}

}  // namespace

extern "C" {

int merf_server_create(const merf_server_config *cfg, merf_server_t *out) {
    clear_error();
    if (!out) return fail(MERF_E_INVALID, "output handle pointer is NULL");
    *out = nullptr;
    if (!cfg || cfg->struct_size != sizeof(merf_server_config))
        return fail(MERF_E_INVALID, "server config missing or struct_size != %zu", sizeof(merf_server_config));
    if (cfg->slots < 1 || cfg->slots > 8) return fail(MERF_E_INVALID, "slots %d not in [1, 8]", cfg->slots);
    if (cfg->max_batch < 1 || cfg->max_batch > kCamsPerLaunch)
        return fail(MERF_E_INVALID, "max_batch %d not in [1, %d]", cfg->max_batch, kCamsPerLaunch);
    merf_server *S = new merf_server();
    S->cfg = *cfg;
    S->budget = cfg->hbm_budget ? cfg->hbm_budget : SIZE_MAX;
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess) e = hipMalloc(&S->table_dev, sizeof(DevScene) * kMaxResident);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->load_stream, hipStreamNonBlocking);
    S->slots.resize((size_t)cfg->slots);
    for (Slot &sl : S->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&sl.staging), sizeof(ServeLaunch));
        if (e == hipSuccess) e = hipMalloc(&sl.desc_dev, sizeof(ServeLaunch));
        if (e == hipSuccess) e = hipMalloc(&sl.ctl_dev, sizeof(ServeCtl));
        if (e == hipSuccess) e = hipMemset(sl.ctl_dev, 0, sizeof(ServeCtl));
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        destroy_slots(S);
        delete S;
        return hip_fail(e, "merf_server_create");
    }
    S->worker = std::thread(worker_main, S);
    S->loader = std::thread(loader_main, S);
    {
        std::lock_guard<std::mutex> lk(g_servers_mu);
        g_servers.insert(S);
    }
    *out = S;
    return MERF_OK;
}

int merf_server_destroy(merf_server_t S) {
    clear_error();
    {
        std::lock_guard<std::mutex> lk(g_servers_mu);
        if (!S || !g_servers.count(S)) return fail(MERF_E_INVALID, "unknown server");
        g_servers.erase(S);
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    S->cv_load.notify_all();
    S->worker.join();
    S->loader.join();
    int rc = MERF_OK;
    for (auto &kv : S->scenes) {
        if (kv.second.h && scene_release_on(kv.second.h, S->load_stream) != MERF_OK) rc = MERF_E_DEVICE;
        free_host(kv.second);
    }
    if (hipStreamSynchronize(S->load_stream) != hipSuccess) rc = MERF_E_DEVICE;
    destroy_slots(S);
    delete S;
    return rc;
}

int merf_server_add_scene(merf_server_t S, const merf_scene_desc *desc, int32_t *scene_id) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    if (!scene_id) return fail(MERF_E_INVALID, "scene_id is NULL");
    const size_t need = scene_device_bytes(desc);
    if (need == 0) {
        merf_scene_t tmp = nullptr;                 // reports the descriptor error
        return merf_scene_upload(desc, &tmp);
    }
    if (need > S->budget) return fail(MERF_E_OOM, "scene needs %zu device bytes, the budget is %zu", need, S->budget);
    SceneEntry fresh;
    if (!copy_scene(desc, fresh)) return fail(MERF_E_OOM, "no host memory for (or no copy into) the server's copy of the scene");
    fresh.need = need;
    SceneEntry *se = nullptr;
    int32_t id = 0;
    int slot = -1;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        id = S->next_scene++;
        se = &S->scenes[id];
        *se = fresh;
        // resident now if it fits; otherwise when a request needs it
        slot = free_table_slot(S);
        if (slot >= 0 && S->resident + need <= S->budget) {
            S->slot_used[slot] = true;
            S->resident += need;
            se->state = kLoading;
        } else {
            slot = -1;
        }
        ++S->st.registered;
    }
    int rc = MERF_OK;
    if (slot >= 0) {
        std::lock_guard<std::mutex> ll(S->load_mu);
        rc = admit(S, se, slot);
    }
    if (rc != MERF_OK) {
        std::lock_guard<std::mutex> lk(S->mu);
        free_host(S->scenes[id]);
        S->scenes.erase(id);
        --S->st.registered;
        return rc;
    }
    *scene_id = id;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        ++S->epoch;
    }
    S->cv_work.notify_all();
    return MERF_OK;
}

int merf_server_remove_scene(merf_server_t S, int32_t scene_id) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    merf_scene_t h = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->scenes.find(scene_id);
        if (it == S->scenes.end()) return fail(MERF_E_INVALID, "unknown scene %d", scene_id);
        SceneEntry &se = it->second;
        if (se.queued + se.running > 0 || se.state == kLoading)
            return fail(MERF_E_INVALID, "scene %d has %d requests queued or running", scene_id, se.queued + se.running);
        if (se.state == kResident) {
            h = se.h;
            S->resident -= se.need;
            S->slot_used[se.slot] = false;
        }
        free_host(se);
        S->scenes.erase(it);
        --S->st.registered;
    }
    S->cv_load.notify_all();                          // memory may have freed up
    if (!h) return MERF_OK;
    std::lock_guard<std::mutex> ll(S->load_mu);
    int rc = scene_release_on(h, S->load_stream);
    if (rc == MERF_OK && hipStreamSynchronize(S->load_stream) != hipSuccess) rc = hip_fail(hipGetLastError(), "release");
    return rc;
}

int merf_server_submit(merf_server_t S, int32_t scene_id, const merf_camera *cam, const merf_render_params *p,
                       float *out_rgba_dev, uint64_t *ticket) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    if (!cam || !ticket || !out_rgba_dev) return fail(MERF_E_INVALID, "NULL camera, ticket or output");
    int rc = check_camera(*cam, 0);
    if (rc) return rc;
    if (p && p->stats_dev) return fail(MERF_E_INVALID, "statistics counters are not available through the server");
    bool absent = false;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->scenes.find(scene_id);
        if (it == S->scenes.end()) return fail(MERF_E_INVALID, "unknown scene %d", scene_id);
        Request r;
        if ((rc = check_params(p, it->second.res, &r.step))) return rc;
        r.scene = scene_id;
        r.cam = *cam;
        r.p = *p;
        r.out = out_rgba_dev;
        r.flag = std::make_shared<std::atomic<bool>>(false);
        r.t_submit = Clock::now();
        const uint64_t t = S->next_ticket++;
        S->reqs.emplace(t, r);
        S->queue.push_back(t);
        ++it->second.queued;
        it->second.heat = heat_at(it->second, r.t_submit) + 1.0;
        it->second.heat_t = r.t_submit;
        ++S->st.submitted;
        absent = it->second.state == kAbsent;
        ++S->epoch;
        *ticket = t;
    }
    S->arrivals.fetch_add(1, std::memory_order_release);
    S->cv_work.notify_one();
    if (absent) S->cv_load.notify_one();
    return MERF_OK;
}

int merf_server_poll(merf_server_t S, uint64_t ticket) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(MERF_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    return it->second.done ? 1 : 0;
}

int merf_server_wait(merf_server_t S, uint64_t ticket, double *latency_ms, double *queue_ms) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(MERF_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done) {
        // poll the request's flag for a while without the lock, then block
        const std::shared_ptr<std::atomic<bool>> flag = it->second.flag;
        lk.unlock();
        const auto t0 = Clock::now();
        while (!flag->load(std::memory_order_acquire) && Clock::now() - t0 < kSpin) std::this_thread::yield();
        lk.lock();
        it = S->reqs.find(ticket);
        if (it == S->reqs.end()) return fail(MERF_E_INVALID, "ticket %llu was waited for twice", (unsigned long long)ticket);
    }
    S->cv_done.wait(lk, [&] { return it->second.done; });
    const Request &r = it->second;
    using ms = std::chrono::duration<double, std::milli>;
    if (latency_ms) *latency_ms = ms(r.t_done - r.t_submit).count();
    if (queue_ms) *queue_ms = ms(r.t_start - r.t_submit).count();
    const int status = r.status;
    S->reqs.erase(it);
    if (status != MERF_OK) return fail(status, "request %llu failed", (unsigned long long)ticket);
    return MERF_OK;
}

int merf_server_drain(merf_server_t S) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->queue.empty() && S->inflight == 0; });
    return MERF_OK;
}

int merf_server_get_stats(merf_server_t S, merf_server_stats *out) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    if (!out) return fail(MERF_E_INVALID, "stats pointer is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    size_t bytes = 0;
    int n = 0;
    for (const auto &kv : S->scenes)
        if (kv.second.state == kResident) {
            bytes += kv.second.need;
            ++n;
        }
    out->resident_bytes = bytes;
    out->resident_scenes = n;
    return MERF_OK;
}

}  // extern "C"
