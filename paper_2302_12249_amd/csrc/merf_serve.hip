// merf_serve.hip -- serving runtime declared in include/merf_serve.h:
// resident scenes under a device-memory budget, a host request queue, and a
// worker thread that continuously batches waiting requests into render
// launches on several HIP streams (optionally replaying captured hipGraphs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
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

struct Request {
    int32_t scene = 0;
    merf_camera cam{};
    merf_render_params p{};
    float step = 0.0f;
    float *out = nullptr;
    Clock::time_point t_submit, t_start, t_done;
    int status = MERF_OK;
    bool done = false;
};

struct SceneEntry {
    merf_scene_t h = nullptr;
    size_t bytes = 0;
    uint64_t last_used = 0;
    int active = 0;                          // queued + running requests
};

constexpr int kVariants = 12;                // MLP fp32 / fp16 / bf16  x  features fp32 / fp16  x  skip mode

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> tickets;
    hipGraph_t graph[kVariants] = {};
    hipGraphExec_t exec[kVariants] = {};
    hipGraphNode_t node[kVariants] = {};
};

}  // namespace

struct merf_server {
    merf_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::map<int32_t, SceneEntry> scenes;
    std::vector<Slot> slots;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1, tick = 0;
    int32_t next_scene = 1;
    size_t resident = 0;
    int inflight = 0;
    merf_server_stats st{};
};

namespace {

std::mutex g_servers_mu;
std::unordered_set<merf_server *> g_servers;

bool server_live(merf_server *s) {
    std::lock_guard<std::mutex> lk(g_servers_mu);
    return s && g_servers.count(s);
}

// Same scene and same parameters: the requests can share one launch.
bool same_batch_key(const Request &a, const Request &b) {
    return a.scene == b.scene && a.step == b.step && a.p.t_min == b.p.t_min && a.p.delta_mode == b.p.delta_mode &&
           a.p.mlp_prec == b.p.mlp_prec && a.p.feat_prec == b.p.feat_prec && a.p.skip_mode == b.p.skip_mode;
}

// Launch rb on the slot: a plain launch, or the slot's graph for this kernel
// variant (captured on first use, afterwards updated with the new arguments).
hipError_t launch_on_slot(Slot &sl, const DevScene &sc, const RenderBatch &rb, bool graphs, bool *was_graph) {
    *was_graph = false;
    if (!graphs) return launch_render(sc, rb, sl.stream);
    const int v = rb.mlp_prec + 3 * rb.feat_prec + 6 * rb.skip_mode;
    void *args[] = {const_cast<DevScene *>(&sc), const_cast<RenderBatch *>(&rb)};
    hipError_t e = hipSuccess;
    if (!sl.exec[v]) {
        e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t el = hipLaunchKernel(render_kernel(rb), render_grid(rb), dim3(kRenderBlock), args, 0, sl.stream);
        e = hipStreamEndCapture(sl.stream, &sl.graph[v]);
        if (el != hipSuccess) return el;
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&sl.exec[v], sl.graph[v], nullptr, nullptr, 0);
        if (e != hipSuccess) return e;
        size_t n = 1;
        e = hipGraphGetNodes(sl.graph[v], &sl.node[v], &n);
        if (e != hipSuccess) return e;
        if (n != 1) return hipErrorInvalidValue;
    } else {
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(render_kernel(rb));
        kp.gridDim = render_grid(rb);
        kp.blockDim = dim3(kRenderBlock);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        e = hipGraphExecKernelNodeSetParams(sl.exec[v], sl.node[v], &kp);
        if (e != hipSuccess) return e;
    }
    *was_graph = true;
    return hipGraphLaunch(sl.exec[v], sl.stream);
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
        auto sc = S->scenes.find(r.scene);
        if (sc != S->scenes.end()) --sc->second.active;
        ++S->st.completed;
    }
    S->inflight -= (int)sl.tickets.size();
    sl.tickets.clear();
    sl.busy = false;
}

// Fuse the oldest waiting request with later waiting requests of the same
// scene and parameters into one launch on slot sl.
void dispatch(merf_server *S, Slot &sl) {
    const uint64_t head = S->queue.front();
    const Request &hr = S->reqs[head];
    auto sit = S->scenes.find(hr.scene);
    const DevScene *sc = sit == S->scenes.end() ? nullptr : scene_dev(sit->second.h);
    RenderBatch rb;
    begin_batch(rb, hr.p, hr.step);
    std::vector<uint64_t> taken;
    for (auto it = S->queue.begin(); it != S->queue.end() && (int)taken.size() < S->cfg.max_batch;) {
        Request &r = S->reqs[*it];
        if (same_batch_key(hr, r) && add_camera(rb, r.cam, r.out)) {
            taken.push_back(*it);
            it = S->queue.erase(it);
        } else {
            ++it;
        }
    }
    const auto now = Clock::now();
    for (uint64_t t : taken) S->reqs[t].t_start = now;
    sl.tickets = taken;
    sl.busy = true;
    S->inflight += (int)taken.size();
    S->st.max_inflight = std::max(S->st.max_inflight, S->inflight);
    if (sit != S->scenes.end()) sit->second.last_used = ++S->tick;
    bool was_graph = false;
    hipError_t e = sc ? launch_on_slot(sl, *sc, rb, S->cfg.use_graphs != 0, &was_graph) : hipErrorInvalidValue;
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        finish_slot(S, sl, MERF_E_DEVICE);
        S->cv_done.notify_all();
        return;
    }
    ++S->st.launches;
    if (was_graph) ++S->st.graph_launches;
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
        if (finished) S->cv_done.notify_all();
        for (Slot &sl : S->slots) {
            if (sl.busy || S->queue.empty()) continue;
            dispatch(S, sl);
            busy = busy || sl.busy;
        }
        if (S->stop && S->queue.empty() && !busy) break;
        if (!busy && S->queue.empty()) {
            S->cv_work.wait(lk);
        } else {
            // poll completions without holding the lock
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(5));
            lk.lock();
        }
    }
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
    hipError_t e = hipGetDevice(&S->device);
    S->slots.resize((size_t)cfg->slots);
    for (Slot &sl : S->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        for (Slot &sl : S->slots) {
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        delete S;
        return hip_fail(e, "merf_server_create");
    }
    S->worker = std::thread(worker_main, S);
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
    S->worker.join();
    int rc = MERF_OK;
    for (auto &kv : S->scenes)
        if (merf_free(kv.second.h) != MERF_OK) rc = MERF_E_DEVICE;
    for (Slot &sl : S->slots) {
        for (int v = 0; v < kVariants; ++v) {
            if (sl.exec[v]) (void)hipGraphExecDestroy(sl.exec[v]);
            if (sl.graph[v]) (void)hipGraphDestroy(sl.graph[v]);
        }
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
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
    std::vector<merf_scene_t> evicted;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        const size_t budget = S->cfg.hbm_budget ? S->cfg.hbm_budget : SIZE_MAX;
        if (need > budget) return fail(MERF_E_OOM, "scene needs %zu bytes, budget is %zu", need, budget);
        while (S->resident + need > budget) {
            // least recently used idle scene
            auto victim = S->scenes.end();
            for (auto it = S->scenes.begin(); it != S->scenes.end(); ++it)
                if (it->second.active == 0 && it->second.h &&
                    (victim == S->scenes.end() || it->second.last_used < victim->second.last_used))
                    victim = it;
            if (!S->cfg.evict_idle || victim == S->scenes.end())
                return fail(MERF_E_OOM, "scene needs %zu bytes; %zu of %zu resident and none can be evicted", need,
                            S->resident, budget);
            evicted.push_back(victim->second.h);
            S->resident -= victim->second.bytes;
            S->scenes.erase(victim);
            ++S->st.evictions;
        }
        S->resident += need;                         // reserve while uploading
    }
    int rc = MERF_OK;
    for (merf_scene_t h : evicted)
        if (merf_free(h) != MERF_OK) rc = MERF_E_DEVICE;
    merf_scene_t h = nullptr;
    if (rc == MERF_OK) rc = merf_scene_upload(desc, &h);
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc != MERF_OK) {
        S->resident -= need;
        return rc;
    }
    const size_t got = merf_scene_bytes(h);
    S->resident = S->resident - need + got;
    const int32_t id = S->next_scene++;
    SceneEntry &e = S->scenes[id];
    e.h = h;
    e.bytes = got;
    e.last_used = ++S->tick;
    *scene_id = id;
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
        if (it->second.active > 0)
            return fail(MERF_E_INVALID, "scene %d has %d requests in flight", scene_id, it->second.active);
        h = it->second.h;
        S->resident -= it->second.bytes;
        S->scenes.erase(it);
    }
    return merf_free(h);
}

int merf_server_submit(merf_server_t S, int32_t scene_id, const merf_camera *cam, const merf_render_params *p,
                       float *out_rgba_dev, uint64_t *ticket) {
    clear_error();
    if (!server_live(S)) return fail(MERF_E_INVALID, "unknown server");
    if (!cam || !ticket || !out_rgba_dev) return fail(MERF_E_INVALID, "NULL camera, ticket or output");
    int rc = check_camera(*cam, 0);
    if (rc) return rc;
    if (p && p->stats_dev) return fail(MERF_E_INVALID, "statistics counters are not available through the server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->scenes.find(scene_id);
        if (it == S->scenes.end()) return fail(MERF_E_INVALID, "unknown scene %d", scene_id);
        const DevScene *ds = scene_dev(it->second.h);
        Request r;
        if ((rc = check_params(p, ds ? ds->res : 1, &r.step))) return rc;
        r.scene = scene_id;
        r.cam = *cam;
        r.p = *p;
        r.out = out_rgba_dev;
        r.t_submit = Clock::now();
        const uint64_t t = S->next_ticket++;
        S->reqs.emplace(t, r);
        S->queue.push_back(t);
        ++it->second.active;
        ++S->st.submitted;
        *ticket = t;
    }
    S->cv_work.notify_one();
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
    S->cv_done.wait(lk, [&] { return it->second.done; });
    const Request &r = it->second;
    using ms = std::chrono::duration<double, std::milli>;
    if (latency_ms) *latency_ms = ms(r.t_done - r.t_submit).count();
    if (queue_ms) *queue_ms = ms(r.t_start - r.t_submit).count();
    const int status = r.status;
    S->reqs.erase(it);
    if (status != MERF_OK) return fail(status, "request %llu failed on the device", (unsigned long long)ticket);
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
    out->resident_bytes = S->resident;
    out->resident_scenes = (int32_t)S->scenes.size();
    return MERF_OK;
}

}  // extern "C"
