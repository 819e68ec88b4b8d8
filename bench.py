#!/usr/bin/env python
"""Benchmark of the MERF deferred renderer on one MI355X.

Workload: the full-size plain FP32 scene (512^3 sparse grid of 8^3 blocks at
~5% occupancy, three 2048^2 uint8 planes with 8 channels, 3-level occupancy
pyramid, content to ||x||_inf = 100 before contraction) rendered from one
1920x1080 camera inside the unit cube.  A step is one merf_render call of that
frame (ray generation, contraction, skipping, gathers, compositing and the
deferred MLP -- the whole hot path in one render kernel, after a small
prepass that orders the tiles heaviest first).  Steps run back to back on
one stream; inputs are resident in device memory before timing starts.

Prints ONE JSON line.  Besides throughput it reports:
  roofline      algorithmic gather bytes per launch / average render-kernel
                time (HIP events recorded around that kernel on its stream,
                on every fifth timed step), against HBM peak;
  latency_ms    p50 / p99 of frames rendered alone (host wall time from the
                call until the frame is done, prepass included);
  cpu_baseline  the FP64 oracle on a bounded row sample of the same frame;
  served        the serving mix through the server (1 GiB budget, and every
                scene resident) beside plain calls, p50 / p99 latency;
  serving_load  p50 / p99 latency at fractions of the served capacity;
  stress        32 resident scenes, 4K and 512^2 requests, served vs plain.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "rays/sec (Mrays/s) at 1080p, % HBM roofline; p50/p99 frame latency served vs plain"
# algorithmic bytes (density first): per evaluated sample 20 density codes +
# 4 B brick index; per sample with alpha != 0 another 20 x 7 appearance codes;
# 1 B per occupancy lookup; 16 B of output per ray.
B_EVAL, B_CONTRIB, B_OCC, B_RAY = 24, 140, 1, 16
# algorithmic vector-ALU FLOPs (the method's arithmetic as the oracle states
# it, counting a multiply-add as 2 and a transcendental as 1):
#   evaluated sample: interpolation weights (grid 8 triple products + 3
#     complements = 19; planes 3 x (4 products + 2 complements) = 18), the
#     density sum over 20 texels (40), Eq. 8 affine (2), exp (1), alpha and
#     transmittance update (5)                                     = 85
#   sample with alpha != 0: 7 channels x 20 texels (280), Eq. 8 affine (14),
#     7 sigmoids (21), compositing 7 multiply-adds (14)              = 329
#   ray: pinhole direction and normalisation (20), direction encoding (36),
#     RGB = C_d + h (3)                                              = 59
# The deferred MLP (1696 FLOP per pixel) runs on the matrix cores and is
# reported separately (mlp_mfma).
F_EVAL, F_CONTRIB, F_RAY = 85, 329, 59
# vector FP32 peak without packed-FP32 instructions, derived from the unit
# counts: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# everything that decides what the render kernel reads and how (kernel, scene
# layout, brick packing); counters taken on other sources are stale
KERNEL_SOURCES = ["paper_2302_12249_amd/csrc/merf_render.hip", "paper_2302_12249_amd/csrc/merf_device.h",
                  "paper_2302_12249_amd/csrc/merf_api.hip", "paper_2302_12249_amd/csrc/merf_ingest.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_full_1080p_traffic.json")
MFMA_FILE = os.path.join(ROOT, "profiles", "render_full_1080p_mfma.json")
# the deferred MLP per pixel: 34 x 16 + 16 x 16 + 16 x 3 multiply-adds (App. B)
MLP_FLOP_PER_PIXEL = 2 * (34 * 16 + 16 * 16 + 16 * 3)
MFMA_F32_PEAK_TFLOPS = 157.3


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_mfma():
    """MFMA counters of the render kernel from the committed rocprofv3 run, if
    taken on the current kernel source; otherwise None."""
    try:
        t = json.load(open(MFMA_FILE))
    except (OSError, ValueError):
        return None
    return t if t.get("kernel_sha") == kernel_hash() else None


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source; otherwise None."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def phase_profile(merf, r, cams, out):
    """Shader-clock cycles per wave by phase, and loop counts per wave, of one
    frame (merf_render_phases: the counting kernel with clock reads at points
    all 64 lanes pass together; same image)."""
    ph = merf.render_phases(r.handle, cams, out)
    waves = max(ph["waves"], 1)
    names = ["setup", "march", "open", "shade", "composite", "mlp"]
    cyc = {n: ph[n + "_cycles"] / waves for n in names}
    total = sum(cyc.values())
    return {"cycles_per_wave": cyc, "total_cycles_per_wave": total,
            "fraction": {n: cyc[n] / total for n in names},
            "per_wave": {"march_passes": ph["march_passes"] / waves, "open_passes": ph["open_passes"] / waves,
                         "shade_passes": ph["shade_passes"] / waves, "rounds": ph["rounds"] / waves},
            "shade_lane_util": ph["shade_lanes"] / max(64 * ph["shade_passes"], 1),
            "opens_per_ray": ph["open_lanes"] / max(ph["stats"]["rays"], 1),
            "waves": ph["waves"]}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, cams, seconds: float):
    """The FP64 oracle on the host: a bounded sample of rows of the frame on all
    host threads, plus a small sample on one thread."""
    import oracle
    os_ = oracle.OracleScene(scene)
    W, H = int(cams.size[0, 0]), int(cams.size[0, 1])
    t0 = time.perf_counter()
    pilot_stride = 135                      # 8 rows
    oracle.render(os_, cams, rows_stride=pilot_stride, row_offset=0, fragile=False, stats=False)
    t_pilot = time.perf_counter() - t0
    per_row = t_pilot / len(range(0, H, pilot_stride))
    rows = max(8, min(H, int(seconds / max(per_row, 1e-9))))
    stride = max(1, H // rows)
    t0 = time.perf_counter()
    out, _ = oracle.render(os_, cams, rows_stride=stride, row_offset=stride // 2, fragile=False, stats=False)
    dt = time.perf_counter() - t0
    n = out.shape[0]
    # one thread, 8 rows spread over the frame
    t1 = time.perf_counter()
    one, _ = oracle.render(os_, cams, rows_stride=135, row_offset=67, fragile=False, stats=False, nthreads=1)
    dt1 = time.perf_counter() - t1
    import numpy as np
    rows = np.arange(stride // 2, H, stride)
    sel = (rows[:, None] * W + np.arange(W)[None, :]).reshape(-1)
    threads = oracle.max_threads()
    return ({"value": n / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
             "sample": (f"one row in {stride} of" if stride > 1 else "all rows of") +
                       f" the {W}x{H} frame ({n} rays, {dt:.1f} s on {threads} threads, FP64 C, OpenMP)",
             "one_thread_Mrays/s": one.shape[0] / dt1 / 1e6,
             "one_thread_sample": f"every 135th row ({one.shape[0]} rays, {dt1:.1f} s)",
             "cpu_model": cpu_model()},
            (out, sel))


def _serving_mix(n_requests: int, seed: int):
    """The serving mix's requests: 8 scenes, resolutions uniform over four
    sizes, scenes drawn from a Zipf(1.5) popularity.  Returns the scenes, the
    four sizes, each request's size, the cameras, each request's scene and the
    generator (for the arrival times drawn after it)."""
    import numpy as np
    import synth

    scenes = synth.serving_scenes()
    sizes_all = [(256, 256), (512, 512), (1280, 720), (1920, 1080)]
    rng = np.random.default_rng(seed)
    sizes = [sizes_all[i] for i in rng.integers(0, len(sizes_all), n_requests)]
    cams = synth.random_cameras(n_requests, seed=seed + 1, sizes=sizes)
    pop = 1.0 / np.arange(1, len(scenes) + 1) ** 1.5
    scene_of = rng.choice(len(scenes), n_requests, p=pop / pop.sum())
    return scenes, sizes_all, sizes, cams, scene_of, rng


def _open_loop_served(srv, ids, scene_of, arr, outs, params, arrive):
    """Submit request i to the server at arrive[i] seconds after the start,
    then wait for all.  Returns each request's (latency ms, queue ms) and the
    seconds from the start to the last completion.  The latency counts from
    the scheduled arrival: the server's own figure (from its submit to the
    completion) plus how late the submit call returned, so that a client
    loop that falls behind its schedule cannot hide waiting."""
    import numpy as np

    tk, late = [], np.zeros(len(arrive))
    t0 = time.perf_counter()
    for i in range(len(arrive)):
        while time.perf_counter() - t0 < arrive[i]:
            pass
        tk.append(srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), params))
        late[i] = time.perf_counter() - t0 - arrive[i]
    waited = [srv.wait(t) for t in tk]
    span = time.perf_counter() - t0
    return [(w[0] + 1e3 * d, w[1]) for w, d in zip(waited, late)], span


def _open_loop_plain(renderers, arr, scene_of, sizes, arrive, params):
    """The plain path on a request stream: each request is one merf_render
    call on one stream, issued at its arrival time, followed by a timing
    event.  Completion times come from the events, relative to one recorded
    on the idle device at the start.  Returns per-request latency in ms."""
    import numpy as np
    import torch
    from paper_2302_12249_amd import merf

    n = len(arrive)
    outs = [torch.empty((w * h, 4), dtype=torch.float32, device="cuda") for (w, h) in sizes]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    one = [_one(arr, i) for i in range(n)]
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(n):
        while time.perf_counter() - t0 < arrive[i]:
            pass
        merf.merf_render(renderers[scene_of[i]].handle, one[i], 1, params, outs[i].data_ptr(), stream.cuda_stream)
        evs[i].record(stream)
    torch.cuda.synchronize()
    done = np.array([start.elapsed_time(e) for e in evs])          # ms after t0
    return done - np.asarray(arrive) * 1e3


def _one(arr, i):
    """merf_camera[1] holding arr[i]."""
    import ctypes as C
    from paper_2302_12249_amd import merf
    one = (merf.merf_camera * 1)()
    C.memmove(C.addressof(one), C.addressof(arr[i]), C.sizeof(merf.merf_camera))
    return one


def serving_leg(n_requests: int, seed: int = 200, budget: int = 1 << 30):
    """Serving mix: 8 scenes (seeds 100-107, occupancy 2-15%, 256^3/1024^2 or
    512^3/2048^2, 1.74 GB together) registered with a server whose device
    budget is 1 GiB, so scenes are evicted and re-admitted; single views of
    resolution uniform over {256^2, 512^2, 1280x720, 1920x1080}, scene drawn
    from a Zipf(1.5) popularity; served with the fp16 deferred MLP by
    continuous batching on 4 slots (persistent launches, graph replay).
    Closed loop (all queued at once) gives the capacity; then a Poisson
    stream at 0.7x that capacity gives the latency, and the same stream
    (same arrival times) goes through the plain fp32 merf_render, one call per
    request on one stream, with every scene resident.  Sampled rows of
    served requests are checked against the FP64 oracle."""
    import numpy as np
    import torch
    import oracle
    from paper_2302_12249_amd import merf

    scenes, sizes_all, sizes, cams, scene_of, rng = _serving_mix(n_requests, seed)
    arr = merf.camera_array(cams)
    p16 = merf.render_params(mlp_prec="f16")
    rays = sum(w * h for (w, h) in sizes)
    res = {"scenes": len(scenes), "scene_bytes_total": None, "hbm_budget": budget, "requests": n_requests,
           "mlp": "f16", "popularity": "zipf 1.5"}
    srv = merf.Server(slots=4, max_batch=16, use_graphs=True, evict_idle=True, hbm_budget=budget)
    try:
        t0 = time.perf_counter()
        ids = [srv.add_scene(s) for s in scenes]
        res["register_s"] = time.perf_counter() - t0
        st0 = srv.stats()
        res["resident_after_register"] = int(st0["resident_scenes"])
        outs = [torch.empty((w * h, 4), dtype=torch.float32, device="cuda") for (w, h) in sizes]
        torch.cuda.synchronize()
        # closed loop: everything queued at once -> capacity (the last of
        # three passes, so that admissions have settled into the popular set)
        for _ in range(3):
            t0 = time.perf_counter()
            tk = [srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), p16) for i in range(n_requests)]
            for t in tk:
                srv.wait(t)
            cap_s = time.perf_counter() - t0
        capacity = n_requests / cap_s
        # open loop: Poisson arrivals at 0.7x capacity
        lam = 0.7 * capacity
        arrive = np.cumsum(rng.exponential(1.0 / lam, n_requests))
        st1 = srv.stats()
        waited, span = _open_loop_served(srv, ids, scene_of, arr, outs, p16, arrive)
        lat = np.array([w[0] for w in waited])
        st = srv.stats()
    finally:
        srv.close()
    # accuracy of served images (fp16 MLP) against the FP64 oracle: every
    # 16th row of 8 requests, two of each resolution
    picks = []
    for wh in sizes_all:
        picks += [i for i in range(n_requests) if sizes[i] == wh][:2]
    worst, se, npx, frag = 0.0, 0.0, 0, 0
    for i in picks:
        w, h = sizes[i]
        ref, fl = oracle.render(scenes[scene_of[i]], cams.subset(i), rows_stride=16, row_offset=5, fragile=True)
        rows = np.arange(5, h, 16)
        sel = (rows[:, None] * w + np.arange(w)[None, :]).reshape(-1)
        d = outs[i].cpu().numpy()[sel].astype(np.float64) - ref
        ok = fl["fragile"] == 0
        worst = max(worst, float(np.abs(d[ok]).max()))
        se += float(np.sum(d[:, :3] ** 2))
        npx += d.shape[0] * 3
        frag += int((~ok).sum())
    psnr = 10.0 * np.log10(1.0 / max(se / max(npx, 1), 1e-30))
    res.update({"capacity_req_per_s": capacity, "capacity_Mrays/s": rays / cap_s / 1e6,
                "arrival_rate_per_s": lam, "offered_Mrays/s": rays / span / 1e6,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()),
                "queue_p50_ms": float(np.percentile([w[1] for w in waited], 50)),
                "launches": int(st["launches"] - st1["launches"]),
                "mixed_scene_launches": int(st["mixed_launches"] - st1["mixed_launches"]),
                "graph_launches": int(st["graph_launches"] - st1["graph_launches"]),
                "admissions": int(st["admissions"]), "evictions": int(st["evictions"]),
                "admission_ms_mean": st["admission_us"] / max(st["admissions"], 1) / 1e3,
                "admissions_in_stream": int(st["admissions"] - st1["admissions"]),
                "max_inflight": int(st["max_inflight"]),
                "resident_bytes": int(st["resident_bytes"]),
                "oracle_check": {"requests": len(picks), "rows": "every 16th", "psnr_db": psnr,
                                 "max_abs_nonfragile": worst, "fragile_pixels": frag}})
    # the same stream served with every scene resident (no budget): what the
    # admissions above cost, beside the plain path below
    srv = merf.Server(slots=4, max_batch=16, use_graphs=True)
    try:
        ids = [srv.add_scene(s) for s in scenes]
        outs = [torch.empty((w * h, 4), dtype=torch.float32, device="cuda") for (w, h) in sizes]
        torch.cuda.synchronize()
        for t in [srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), p16) for i in range(min(32, n_requests))]:
            srv.wait(t)
        waited, _ = _open_loop_served(srv, ids, scene_of, arr, outs, p16, arrive)
        lat_all = np.array([w[0] for w in waited])
    finally:
        srv.close()
    res["served_all_resident_same_stream"] = {"p50_ms": float(np.percentile(lat_all, 50)),
                                              "p99_ms": float(np.percentile(lat_all, 99)),
                                              "mean_ms": float(lat_all.mean())}
    # the plain fp32 path on the same request stream (every scene resident)
    rends = [merf.Renderer(s) for s in scenes]
    try:
        res["scene_bytes_total"] = int(sum(merf.scene_bytes(r.handle) for r in rends))
        pf = merf.render_params(order="plain")
        for i in range(min(8, n_requests)):               # warm up
            rends[scene_of[i]].render(cams.subset(i), order="plain")
        torch.cuda.synchronize()
        plat = _open_loop_plain(rends, arr, scene_of, sizes, arrive, pf)
    finally:
        for r in rends:
            r.close()
    res["plain_fp32_same_stream"] = {"p50_ms": float(np.percentile(plat, 50)),
                                     "p99_ms": float(np.percentile(plat, 99)), "mean_ms": float(plat.mean())}
    return res


def serving_load_workload(n_requests: int, seed: int = 200, budget: int = 1 << 30,
                          loads=(0.3, 0.5, 0.7, 0.85, 0.95, 1.1)):
    """Latency against offered load on the serving mix (its scenes, sizes and
    popularity).  The reference rate is the capacity of the server with every
    scene resident (fp16 MLP, closed loop: all requests queued at once).
    Poisson streams at each fraction of it go through that server, through a
    server whose device budget is 1 GiB (scenes evicted and re-admitted), and
    through the plain fp32 merf_render on one stream.  Every stream has the
    same requests in the same order, with the arrival times of one unit-rate
    Poisson stream scaled to its rate.  The closed-loop capacities of the
    budgeted server and of the plain path are reported too."""
    import numpy as np
    import torch
    from paper_2302_12249_amd import merf

    scenes, _, sizes, cams, scene_of, rng = _serving_mix(n_requests, seed)
    arr = merf.camera_array(cams)
    p16 = merf.render_params(mlp_prec="f16")
    rays = sum(w * h for (w, h) in sizes)
    unit = np.cumsum(rng.exponential(1.0, n_requests))
    outs = [torch.empty((w * h, 4), dtype=torch.float32, device="cuda") for (w, h) in sizes]

    def point(f, lat, last_s):
        return {"load": f, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "completed_Mrays/s": rays / last_s / 1e6}

    def served_curve(srv, ref):
        """Closed-loop capacity (the last of three passes, so that admissions
        have settled), then the open-loop streams at fractions of ref (of
        this capacity if ref is None)."""
        ids = [srv.add_scene(s) for s in scenes]
        torch.cuda.synchronize()
        for _ in range(3):
            t0 = time.perf_counter()
            for t in [srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), p16) for i in range(n_requests)]:
                srv.wait(t)
            cap = n_requests / (time.perf_counter() - t0)
        ref = ref or cap
        st0 = srv.stats()
        pts = []
        for f in loads:
            waited, last_s = _open_loop_served(srv, ids, scene_of, arr, outs, p16, unit / (f * ref))
            pts.append(point(f, np.array([w[0] for w in waited]), last_s))
        st = srv.stats()
        return ref, cap, {"capacity_req_per_s": cap, "points": pts,
                          "admissions": int(st["admissions"] - st0["admissions"]),
                          "evictions": int(st["evictions"] - st0["evictions"])}

    res = {"requests_per_point": n_requests, "hbm_budget": budget, "loads": list(loads)}
    srv = merf.Server(slots=4, max_batch=16, use_graphs=True)
    try:
        ref, _, res["served_all_resident"] = served_curve(srv, None)
    finally:
        srv.close()
    res["reference_req_per_s"] = ref
    res["reference_Mrays/s"] = rays * ref / n_requests / 1e6
    srv = merf.Server(slots=4, max_batch=16, use_graphs=True, evict_idle=True, hbm_budget=budget)
    try:
        _, _, res["served_budget"] = served_curve(srv, ref)
    finally:
        srv.close()
    rends = [merf.Renderer(s) for s in scenes]
    try:
        pf = merf.render_params(order="plain")
        for i in range(min(8, n_requests)):               # warm up
            rends[scene_of[i]].render(cams.subset(i), order="plain")
        torch.cuda.synchronize()
        back_to_back = _open_loop_plain(rends, arr, scene_of, sizes, np.zeros(n_requests), pf)
        pts = []
        for f in loads:
            arrive = unit / (f * ref)
            lat = _open_loop_plain(rends, arr, scene_of, sizes, arrive, pf)
            pts.append(point(f, lat, float((lat + arrive * 1e3).max()) / 1e3))
    finally:
        for r in rends:
            r.close()
    res["plain_fp32"] = {"capacity_req_per_s": n_requests / (float(back_to_back.max()) / 1e3), "points": pts}
    at = {p["load"]: p for p in res["served_budget"]["points"]}
    return {"metric": "p50/p99 frame latency against offered load, served vs plain (serving mix)",
            "value": at[0.7]["p99_ms"] if 0.7 in at else None,
            "unit": "ms (p99 of the budgeted server at 0.7 of the resident capacity)",
            "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": "serving mix: 8 scenes (256^3/1024^2 to 512^3/2048^2, 2-15% occupancy, "
                                   "1.74 GB), Zipf(1.5) popularity, views of 256^2/512^2/1280x720/1920x1080, "
                                   "Poisson arrivals at fractions of the served capacity",
                       "slots": 4, "max_batch": 16, "mlp": "f16 served, f32 plain"},
            "load_sweep": res}


def precision_config(steps: int, scene=None):
    """Precision config: the full-size scene as 16 seeded 1920x1080 orbit views in
    one batched render call; fp32 / fp16 / bf16 MLP and both fp16 feature
    modes (every code dequantised to fp16; appearance interpolated from fp16
    operands), each
    timed (CUDA events around `steps` calls) and compared with the FP64 oracle
    on every 64th row of every view (PSNR over all sampled pixels, max error
    over the pixels the oracle does not flag as fragile)."""
    import numpy as np
    import torch
    import oracle
    import synth
    from paper_2302_12249_amd import merf

    scene = scene if scene is not None else synth.preset_scene("full")
    cams = synth.orbit_cameras(16)
    rays = cams.num_pixels()
    r = merf.Renderer(scene)
    stream = torch.cuda.current_stream()
    out = torch.empty((rays, 4), dtype=torch.float32, device="cuda")
    W, H = 1920, 1080
    t0 = time.perf_counter()
    ref, st = oracle.render(scene, cams, rows_stride=64, row_offset=31, fragile=True)
    t_oracle = time.perf_counter() - t0
    rows = np.arange(31, H, 64)
    sel = np.concatenate([(c * W * H + rows[:, None] * W + np.arange(W)[None, :]).reshape(-1) for c in range(16)])
    ok = st["fragile"] == 0
    res = {}
    for name, mlp, feat in (("f32", "f32", "f32"), ("mlp_f16", "f16", "f32"), ("mlp_bf16", "bf16", "f32"),
                            ("feat_f16_mlp_f16", "f16", "f16"), ("feat_f16_mlp_bf16", "bf16", "f16"),
                            ("feat_f16i_mlp_f32", "f32", "f16_interp"), ("feat_f16i_mlp_f16", "f16", "f16_interp"),
                            ("feat_f16i_mlp_bf16", "bf16", "f16_interp")):
        for _ in range(2):
            r.render(cams, out=out, mlp_prec=mlp, feat_prec=feat)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            r.render(cams, out=out, mlp_prec=mlp, feat_prec=feat)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        d = out.cpu().numpy()[sel].astype(np.float64) - ref
        res[name] = {"mlp": mlp, "features": feat, "ms_per_call": ms, "Mrays/s": rays / (ms * 1e-3) / 1e6,
                     "psnr_db": 10 * np.log10(1 / max(float(np.mean(d[:, :3] ** 2)), 1e-30)),
                     "psnr_db_nonfragile": 10 * np.log10(1 / max(float(np.mean(d[ok, :3] ** 2)), 1e-30)),
                     "max_abs_nonfragile": float(np.abs(d[ok]).max()), "max_abs": float(np.abs(d).max()),
                     "mean_abs": float(np.abs(d).mean())}
    r.close()
    return {"workload": "full-size scene, 16 orbit views at 1920x1080 in one merf_render call", "rays_per_call": rays,
            "calls_timed": steps, "oracle_rows": "every 64th row of every view", "oracle_pixels": int(len(sel)),
            "oracle_s": t_oracle, "fragile_frac": float((~ok).mean()), "modes": res}


def precision_workload(steps: int):
    pc = precision_config(steps)
    return {"metric": "Mrays/s, 16 x 1080p views (precision config)", "value": pc["modes"]["f32"]["Mrays/s"],
            "unit": "Mrays/s", "n_gpus": 1, "steps": steps, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": pc["workload"], "rays_per_step": pc["rays_per_call"]}, "precision": pc}


def stress_workload(n_scenes: int, n_requests: int):
    """Stress config: n_scenes resident 512^3/2048^2 scenes at up to 25% block
    occupancy, half step (2/R), 3840x2160 requests mixed with 512^2 requests,
    bf16 MLP through the server; beside the plain fp32 renderer (one request
    per merf_render call) on the same requests."""
    import numpy as np
    import torch
    import synth
    from paper_2302_12249_amd import merf

    rng = np.random.default_rng(300)
    srv = merf.Server(slots=4, max_batch=16, use_graphs=True)
    ids, gen_s = [], 0.0
    scenes = []
    try:
        for k in range(n_scenes):
            t0 = time.perf_counter()
            sc = synth.make_scene(512, 2048, float(rng.uniform(0.05, 0.25)), 1.99, 0.05, 0.25, pools=(8, 2, 1),
                                  seed=300 + k, mlp_seed=5300 + k, name=f"stress{k}")
            gen_s += time.perf_counter() - t0
            ids.append(srv.add_scene(sc))
            scenes.append(sc if k < 2 else None)          # keep two for the plain comparison
            del sc
        sizes = [(3840, 2160) if rng.random() < 0.25 else (512, 512) for _ in range(n_requests)]
        cams = synth.random_cameras(n_requests, seed=301, sizes=sizes)
        scene_of = rng.integers(0, n_scenes, n_requests)
        arr = merf.camera_array(cams)
        step = 2.0 / 2048
        p16 = merf.render_params(step=step, mlp_prec="bf16")
        outs = [torch.empty((w * h, 4), dtype=torch.float32, device="cuda") for (w, h) in sizes]
        rays = sum(w * h for (w, h) in sizes)
        for _ in range(2):
            tk = [srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), p16) for i in range(n_requests)]
            lat = np.array([srv.wait(t)[0] for t in tk])
        t0 = time.perf_counter()
        tk = [srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), p16) for i in range(n_requests)]
        lat = np.array([srv.wait(t)[0] for t in tk])
        span = time.perf_counter() - t0
        st = srv.stats()
        # plain fp32 renderer on the requests of the two kept scenes
        plain = []
        for k in (0, 1):
            rr = merf.Renderer(scenes[k])
            idx = [i for i in range(n_requests) if scene_of[i] == k][:8]
            for i in idx:
                for _ in range(2):
                    rr.render(cams.subset(i), out=outs[i], step=step)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                rr.render(cams.subset(i), out=outs[i], step=step)
                torch.cuda.synchronize()
                plain.append((sizes[i][0] * sizes[i][1], time.perf_counter() - t1))
            rr.close()
    finally:
        srv.close()
    prays = sum(n for n, _ in plain)
    ptime = sum(t for _, t in plain)
    return {"metric": "served Mrays/s and p50/p99 latency (stress config)", "value": rays / span / 1e6,
            "unit": "Mrays/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"{n_scenes} resident 512^3/2048^2 scenes (5-25% occupancy), step 2/R, "
                                   f"{n_requests} requests 3840x2160 or 512^2, bf16 MLP",
                       "resident_bytes": int(st["resident_bytes"]), "scene_generation_s": gen_s},
            "served": {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                       "launches": int(st["launches"]), "max_inflight": int(st["max_inflight"])},
            "plain_fp32_Mrays/s": prays / ptime / 1e6 if ptime > 0 else None}


def variants_workload(steps: int):
    """Representation variants on the full-size camera: MERF (512^3 grid +
    2048^2 planes), the same scene without its grid (planes only, the paper's
    Sec. 7 ablation) and block-sparse grids without planes (512^3 and 1024^3,
    in the spirit of the SNeRG++ comparison): device bytes against Mrays/s."""
    import numpy as np
    import torch
    import synth
    from paper_2302_12249_amd import merf

    full = synth.preset_scene("full")
    cams = synth.full_camera()
    rays = cams.num_pixels()
    variants = [("merf_L512_R2048", full), ("planes_only_R2048", synth.planes_only(full)),
                ("grid_only_L512", synth.grid_only_scene(512, 0.05, seed=2)),
                ("grid_only_L1024", synth.grid_only_scene(1024, 0.05, seed=2))]
    out = torch.empty((rays, 4), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    for name, sc in variants:
        r = merf.Renderer(sc)
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        r.render(cams, out=out, stats=st)
        for _ in range(3):
            r.render(cams, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            r.render(cams, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        cnt = st.cpu().numpy()
        res[name] = {"device_bytes": merf.scene_bytes(r.handle), "ms_per_frame": ms,
                     "Mrays/s": rays / (ms * 1e-3) / 1e6, "evaluated_per_ray": float(cnt[3]) / rays,
                     "step": sc.step}
        r.close()
    return {"metric": "Mrays/s at 1080p and device bytes per representation", "value": res["merf_L512_R2048"]["Mrays/s"],
            "unit": "Mrays/s", "n_gpus": 1, "steps": steps, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": "full-size camera, four representations of the same kind of scene"},
            "variants": res}


def resolutions_workload(steps: int):
    """The Full scene from the full-size camera at several resolutions, frames
    back to back on one stream, with the tiles heaviest first and in plain
    order: where the tile order starts to pay (launches of 8192 tiles or more)."""
    import torch
    import synth
    from paper_2302_12249_amd import merf

    full = synth.preset_scene("full")
    pose = synth.full_camera().c2w[0].astype("float64")
    r = merf.Renderer(full)
    res = {}
    for w, h in ((256, 256), (512, 512), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)):
        cams = synth.make_cameras([pose], [(w, h)])
        rays = cams.num_pixels()
        out = torch.empty((rays, 4), dtype=torch.float32, device="cuda")
        row = {"tiles": ((w + 7) // 8) * ((h + 7) // 8)}
        for order in ("heavy_first", "plain"):
            for _ in range(5):
                r.render(cams, out=out, order=order)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                r.render(cams, out=out, order=order)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            row[order] = {"ms_per_frame": ms, "Mrays/s": rays / (ms * 1e-3) / 1e6}
        res[f"{w}x{h}"] = row
        del out
    r.close()
    return {"metric": "Mrays/s by resolution, frames back to back", "value": res["1920x1080"]["heavy_first"]["Mrays/s"],
            "unit": "Mrays/s", "n_gpus": 1, "steps": steps, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": "full-size scene and camera pose at six resolutions, both tile orders"},
            "resolutions": res}


class KernelTimer:
    """Pairs of HIP timing events created without the system-scope cache
    flush that an ordinary event record performs (hipEventDisableSystemFence):
    the flush would slow the kernel being timed and the one after it."""

    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self, n):
        import ctypes as C
        import torch
        torch.cuda.init()
        self.C = C
        self.hip = C.CDLL("libamdhip64.so.7")       # the runtime torch already loaded
        self.hip.hipEventCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]
        self.ev = []
        for _ in range(2 * n):
            e = C.c_void_p()
            assert self.hip.hipEventCreateWithFlags(C.byref(e), self.DISABLE_SYSTEM_FENCE) == 0
            self.ev.append(e)

    def pair(self, i):
        return self.ev[2 * i], self.ev[2 * i + 1]

    def ms(self, a, b):
        t = self.C.c_float()
        assert self.hip.hipEventElapsedTime(self.C.byref(t), a, b) == 0
        return t.value

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)


def timed_frames(merf, r, cams, img, n, **kw):
    """Mean render-kernel and whole-frame GPU times (ms) of n frames rendered
    back to back into img with render parameters kw."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(3):
        r.render(cams, out=img, **kw)
    tm = KernelTimer(n)
    torch.cuda.synchronize()
    for i in range(n):
        merf.render_timed(r.handle, cams, img, *tm.pair(i), **kw)
    torch.cuda.synchronize()
    kern = [tm.ms(*tm.pair(i)) for i in range(n)]
    frame = [tm.ms(tm.pair(i - 1)[1], tm.pair(i)[1]) for i in range(1, n)]
    tm.close()
    return float(np.mean(kern)), float(np.mean(frame))


def isolated_latency(r, cams, img, n, **kw):
    """Host wall time (ms) of n frames each rendered alone: render, then wait
    for it, so nothing overlaps (the tile-order prepass included)."""
    import numpy as np
    import torch
    for _ in range(3):
        r.render(cams, out=img, **kw)
    torch.cuda.synchronize()
    lat = []
    for _ in range(n):
        t0 = time.perf_counter()
        r.render(cams, out=img, **kw)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "mean": float(np.mean(lat))}


def two_in_flight(r, cams, out, steps):
    """Frames rendered on two alternating streams, so consecutive frames overlap."""
    import torch
    s2 = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs2 = [out, torch.empty_like(out)]
    for i in range(4):
        r.render(cams, out=outs2[i % 2], stream=s2[i % 2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        r.render(cams, out=outs2[i % 2], stream=s2[i % 2])
    torch.cuda.synchronize()
    ms2 = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_frame": ms2, "Mrays/s": cams.num_pixels() / (ms2 * 1e-3) / 1e6}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=150)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["full", "precision", "stress", "variants", "resolutions", "serving_load"],
                    default="full",
                    help="full (default, the headline line), precision (16 x 1080p views), stress, "
                         "variants (representations: memory against speed), resolutions (tile order by frame "
                         "size) or serving_load (latency against offered load on the serving mix)")
    ap.add_argument("--stress-scenes", type=int, default=32,
                    help="resident scenes of the Stress config (in the default line and --workload stress; 0: skip)")
    ap.add_argument("--precision-steps", type=int, default=5,
                    help="timed calls per mode of the 16 x 1080p precision config in the default line (0 skips it)")
    ap.add_argument("--serve-requests", type=int, default=240,
                    help="requests in the serving-mix leg (0 skips it)")
    ap.add_argument("--serve-load", type=int, default=1,
                    help="1: the default line includes latency against offered load on the serving mix "
                         "(--serve-requests requests a point); 0 skips it")
    ap.add_argument("--no-overlap", action="store_true",
                    help="skip the two-frames-in-flight leg (its concurrent launches would blur per-kernel profiles)")
    ap.add_argument("--event-every", type=int, default=5,
                    help="record the render kernel's timing events on every n-th timed step")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline frames (for profiling: the other legs launch the same render "
                         "kernel with other settings, which would mix into its per-kernel averages)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, run a plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this renderer runs on one GPU; --gpus {args.gpus} is not supported "
              "(every pixel is independent, so more GPUs would split cameras or tiles; not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2302_12249_amd import merf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "precision":
        print(json.dumps(precision_workload(args.steps)), flush=True)
        return
    if args.workload == "variants":
        print(json.dumps(variants_workload(args.steps)), flush=True)
        return
    if args.workload == "resolutions":
        print(json.dumps(resolutions_workload(args.steps)), flush=True)
        return
    if args.workload == "stress":
        print(json.dumps(stress_workload(args.stress_scenes, args.serve_requests)), flush=True)
        return
    if args.workload == "serving_load":
        print(json.dumps(serving_load_workload(max(args.serve_requests, 1))), flush=True)
        return
    scene = synth.preset_scene("full")
    cams = synth.full_camera()
    rays = cams.num_pixels()
    r = merf.Renderer(scene)
    stream = torch.cuda.current_stream()
    out = torch.empty((rays, 4), dtype=torch.float32, device="cuda")

    # untimed: counters of the work one frame does
    st = torch.zeros(8, dtype=torch.int64, device="cuda")
    r.render(cams, out=out, stats=st)
    torch.cuda.synchronize()
    cnt = st.cpu().numpy()
    n_rays, occ_lookups, visited, evaluated, contributing = [int(v) for v in cnt[:5]]
    alg_bytes = evaluated * B_EVAL + contributing * B_CONTRIB + occ_lookups * B_OCC + n_rays * B_RAY
    alg_flops = evaluated * F_EVAL + contributing * F_CONTRIB + n_rays * F_RAY
    # untimed: where a wave's time goes (phase-profiled variant of the kernel)
    phases = phase_profile(merf, r, cams, out)

    for _ in range(args.warmup):
        r.render(cams, out=out)
    torch.cuda.synchronize()

    # per step, the library records a pair of events right around the render
    # kernel on its stream (the frame's tile-order prepass runs before, on
    # the library's own stream, overlapping the previous frame)
    # every event_every-th step records its events (an event record between
    # two kernels costs a few microseconds, so timing every step would slow
    # the very frames being measured)
    ev_steps = list(range(0, args.steps, max(1, args.event_every)))
    tm = KernelTimer(len(ev_steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    j = 0
    for i in range(args.steps):
        if j < len(ev_steps) and i == ev_steps[j]:
            merf.render_timed(r.handle, cams, out, *tm.pair(j))
            j += 1
        else:
            r.render(cams, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([tm.ms(*tm.pair(j)) for j in range(len(ev_steps))])        # ms, render kernel
    # GPU time per frame: from one timed frame's end to the next one's, over
    # the frames between them
    frame = np.array([tm.ms(tm.pair(j)[1], tm.pair(j + 1)[1]) / (ev_steps[j + 1] - ev_steps[j])
                      for j in range(len(ev_steps) - 1)] or [float("nan")])
    tm.close()

    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = float(per.mean())
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    res = {
        "metric": METRIC,
        "value": rays / (ms_per_step * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "full-size plain FP32: 512^3 sparse grid of 8^3 blocks (~5% occupied), three "
                               "2048^2 uint8 planes x 8 channels, 3-level occupancy (16^3/64^3/128^3), "
                               "one 1920x1080 view from inside the unit cube",
                   "scene_seed": scene.seed, "camera_seed": 22, "rays_per_step": rays, "step": scene.step},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
        "kernel_ms": kernel_ms,
        "frame_gpu_ms": float(frame.mean()),
        "latency_ms": None if args.headline_only else isolated_latency(r, cams, out, 100),
        "per_ray": {"evaluated": evaluated / n_rays, "contributing": contributing / n_rays,
                    "visited": visited / n_rays, "occ_lookups": occ_lookups / n_rays},
        "alg_bytes_per_launch": alg_bytes,
        "alg_valu_flops_per_launch": alg_flops,
        "valu_roof": {"achieved_TFLOP/s": alg_flops / (kernel_ms * 1e-3) / 1e12, "peak_TFLOP/s": VALU_F32_PEAK_TFLOPS,
                      "frac": alg_flops / (kernel_ms * 1e-3) / 1e12 / VALU_F32_PEAK_TFLOPS},
        "phases": phases,
    }
    # the deferred MLP, the path's only dense contraction, on the matrix cores
    mf = measured_mfma()
    mlp_flop = n_rays * MLP_FLOP_PER_PIXEL
    res["mlp_mfma"] = {"flop_per_launch": mlp_flop,
                       "TFLOP/s_over_kernel": mlp_flop / (kernel_ms * 1e-3) / 1e12,
                       "peak_TFLOP/s": MFMA_F32_PEAK_TFLOPS,
                       "issued_flop_per_launch": mf["mfma_flop_per_launch"] if mf else None,
                       "mfma_busy_pct": mf["mfma_util_pct"] if mf else None}
    # the same frames with two in flight (alternating streams, as a renderer
    # double-buffers): the tail of one frame overlaps the start of the next
    if not args.no_overlap:
        res["two_in_flight"] = two_in_flight(r, cams, out, args.steps)
    prec = {}
    if not args.headline_only:
        # the same frame with the tiles in plain order (no cost prepass)
        pl_img = torch.empty_like(out)
        pl_kernel, pl_frame = timed_frames(merf, r, cams, pl_img, 20, order="plain")
        res["plain_order"] = {"kernel_ms": pl_kernel, "frame_gpu_ms": pl_frame,
                              "Mrays/s": rays / (pl_frame * 1e-3) / 1e6,
                              "latency_ms": isolated_latency(r, cams, pl_img, 100, order="plain"),
                              "same_image": bool(torch.equal(pl_img, out))}
        del pl_img
        # the paper's level-by-level skipping (skip_mode 1) on the same frame:
        # same image, more march steps
        lv_img = torch.empty_like(out)
        st_lv = torch.zeros(8, dtype=torch.int64, device="cuda")
        r.render(cams, out=lv_img, stats=st_lv, skip="levels")
        lv_kernel, lv_ms = timed_frames(merf, r, cams, lv_img, 20, skip="levels")
        c_lv = st_lv.cpu().numpy()
        res["skip_levels"] = {"kernel_ms": lv_kernel, "frame_gpu_ms": lv_ms, "Mrays/s": rays / (lv_ms * 1e-3) / 1e6,
                              "visited_per_ray": float(c_lv[2]) / n_rays, "occ_lookups_per_ray": float(c_lv[1]) / n_rays,
                              "same_image": bool(torch.equal(lv_img, out))}
        del lv_img
        # gather bound: replay the frame's recorded texel loads with no arithmetic
        rec = merf.GatherRecord(r.handle, cams, cap=96)
        torch.cuda.synchronize()
        counts = rec.count.cpu().numpy()
        for _ in range(3):
            rec.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            rec.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        rp_ms = e0.elapsed_time(e1) / 20
        gather_bytes = evaluated * B_EVAL + contributing * B_CONTRIB + n_rays * B_RAY
        res["gather_replay"] = {"kernel_ms": rp_ms, "gather_bytes": gather_bytes,
                                "replay_GB/s": gather_bytes / (rp_ms * 1e-3) / 1e9,
                                "render_GB/s": gather_bytes / (kernel_ms * 1e-3) / 1e9,
                                "render_frac_of_replay": rp_ms / kernel_ms,
                                "frame_frac_of_replay": rp_ms / float(frame.mean()),
                                "max_samples_per_ray": int(counts.max()),
                                "unrecorded_samples": int(np.maximum(counts - rec.cap, 0).sum()),
                                "same_image": bool(torch.equal(rec.image, out))}
        del rec
        # precision variants of the deferred MLP (fp16 / bf16 inputs on MFMA,
        # fp32 accumulation); compositing and transmittance stay fp32
        for name, mlp, feat in (("mlp_f16", "f16", "f32"), ("mlp_bf16", "bf16", "f32"),
                                ("feat_f16_mlp_f16", "f16", "f16"), ("feat_f16_mlp_bf16", "bf16", "f16"),
                                ("feat_f16i_mlp_f32", "f32", "f16_interp"), ("feat_f16i_mlp_f16", "f16", "f16_interp"),
                                ("feat_f16i_mlp_bf16", "bf16", "f16_interp")):
            img = torch.empty_like(out)
            k_ms, ms = timed_frames(merf, r, cams, img, 20, mlp_prec=mlp, feat_prec=feat)
            prec[name] = {"mlp": mlp, "features": feat, "kernel_ms": k_ms, "frame_gpu_ms": ms,
                          "Mrays/s": rays / (ms * 1e-3) / 1e6, "_img": img}
        res["precision"] = prec
    if not args.headline_only and args.precision_steps > 0:
        # the Precision config (16 x 1080p orbit views in one call)
        res["precision_config"] = precision_config(args.precision_steps, scene)
    if args.copy_probe_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters read
        # exactly copy_probe_mb MiB each when the counters are exact
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = src.numel() * 4
        del src, dst
    if args.serve_requests > 0:
        res["served"] = serving_leg(args.serve_requests)
    if args.serve_requests > 0 and args.stress_scenes > 0 and not args.headline_only:
        # the Stress config: many resident scenes, 4K and 512^2 requests, bf16
        # MLP through the server, beside plain fp32 calls
        st = stress_workload(args.stress_scenes, args.serve_requests)
        res["stress"] = {"workload": st["config"]["workload"], "resident_bytes": st["config"]["resident_bytes"],
                         "served_Mrays/s": st["value"], "served": st["served"],
                         "plain_fp32_Mrays/s": st["plain_fp32_Mrays/s"]}
    if args.serve_requests > 0 and args.serve_load and not args.headline_only:
        # latency against offered load on the serving mix (p50 / p99 ms from
        # the scheduled arrival at fractions of the all-resident capacity)
        sl = serving_load_workload(args.serve_requests, loads=(0.3, 0.5, 0.7, 0.95))["load_sweep"]
        curve = lambda k: {f'{p["load"]:.2f}': [round(p["p50_ms"], 3), round(p["p99_ms"], 2)]
                           for p in sl[k]["points"]}
        res["serving_load"] = {"requests_per_point": sl["requests_per_point"],
                               "reference_req_per_s": sl["reference_req_per_s"],
                               "reference_Mrays/s": sl["reference_Mrays/s"],
                               "p50_p99_ms": {k: curve(k) for k in ("served_all_resident", "served_budget",
                                                                    "plain_fp32")},
                               "capacity_req_per_s": {"served_budget": sl["served_budget"]["capacity_req_per_s"],
                                                      "plain_fp32": sl["plain_fp32"]["capacity_req_per_s"]}}
    images = {"f32": out.cpu().numpy()}
    for name, v in prec.items():
        images[name] = v.pop("_img").cpu().numpy()
    r.close()
    if not args.no_cpu_baseline:
        res["cpu_baseline"], _ = cpu_baseline(scene, cams, args.cpu_seconds)
        # accuracy of each path against the FP64 oracle on every 8th row, with
        # the oracle's fragility flags (pixels with a sample on an occupancy
        # face, where FP32 and FP64 may legitimately decide differently)
        import oracle
        W, H = int(cams.size[0, 0]), int(cams.size[0, 1])
        ref, st = oracle.render(scene, cams, rows_stride=8, row_offset=3, fragile=True)
        rows = np.arange(3, H, 8)
        sel = (rows[:, None] * W + np.arange(W)[None, :]).reshape(-1)
        ok = st["fragile"] == 0
        for name, img in images.items():
            d = img[sel].astype(np.float64) - ref
            mse = float(np.mean(d[:, :3] ** 2))
            mse_ok = float(np.mean(d[ok, :3] ** 2))
            acc = {"psnr_db": 10.0 * np.log10(1.0 / max(mse, 1e-30)),
                   "psnr_db_nonfragile": 10.0 * np.log10(1.0 / max(mse_ok, 1e-30)),
                   "max_abs_nonfragile": float(np.abs(d[ok]).max()), "max_abs": float(np.abs(d).max()),
                   "mean_abs": float(np.abs(d).mean()), "pixels": int(len(sel)),
                   "fragile_frac": float((~ok).mean())}
            if name == "f32":
                res["accuracy_f32"] = acc
            else:
                res["precision"][name].update(acc)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
