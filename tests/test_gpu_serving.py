"""GPU tests of the serving runtime (include/merf_serve.h): continuous
batching of uneven requests over several scenes, fused into persistent
launches across scenes, must give every request exactly the image
merf_render gives it alone; scenes are admitted by the device-memory budget,
evicted least requested first and re-admitted on demand."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import MIN_PSNR_DB, check

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def merf():
    from paper_2302_12249_amd import merf as m
    m.load()
    return m


@pytest.fixture(scope="module")
def scenes():
    return [synth.preset_scene("tiny", seed=s) for s in (1, 2, 3)]


def request_mix(n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(64, 64), (96, 40), (13, 7), (128, 128), (33, 65)]
    cams = synth.random_cameras(n, seed=seed, sizes=[sizes[i] for i in rng.integers(0, len(sizes), n)],
                                inside=2.5)
    scene_of = rng.integers(0, 3, n)
    prec = [("f32", "f16", "bf16")[i] for i in rng.integers(0, 3, n)]
    return cams, scene_of, prec


def render_alone(torch, merf, scene, cams, i, prec):
    r = merf.Renderer(scene)
    try:
        out = r.render(cams.subset(i), mlp_prec=prec)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        r.close()


@pytest.mark.parametrize("use_graphs", [True, False])
def test_mix_equals_alone(torch, merf, scenes, use_graphs):
    say(f"serving: 24 uneven requests over 3 scenes, graphs={use_graphs}")
    cams, scene_of, prec = request_mix(24, seed=7)
    arr = merf.camera_array(cams)
    srv = merf.Server(slots=3, max_batch=8, use_graphs=use_graphs)
    try:
        ids = [srv.add_scene(s) for s in scenes]
        # NaN-filled outputs, filled before any submit: the server's streams
        # are not ordered after torch's, so a pending fill could land after
        # the render
        outs = [torch.full((int(w) * int(h), 4), float("nan"), device="cuda") for w, h in cams.size]
        torch.cuda.synchronize()
        tickets = []
        steps = [0.0 if i % 4 else 1.0 / 48 for i in range(len(cams))]   # default step 4/R, or a coarser one
        feats = ["f16_interp" if i % 6 == 5 else "f32" for i in range(len(cams))]
        for i in range(len(cams)):
            p = merf.render_params(mlp_prec=prec[i], step=steps[i], feat_prec=feats[i])
            tickets.append(srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), p))
        lats = [srv.wait(t)[0] for t in tickets]
        st = srv.stats()
        say(f"  launches {st['launches']} (graph {st['graph_launches']}, mixed-scene {st['mixed_launches']}), "
            f"max in flight {st['max_inflight']}, latency p50 {np.percentile(lats, 50):.3f} ms")
        assert st["completed"] == len(cams)
        assert st["launches"] < len(cams)            # requests were fused
        assert st["mixed_launches"] >= 1             # ... across scenes
        if use_graphs:
            assert st["graph_launches"] == st["launches"]
        for i in range(len(cams)):
            r = merf.Renderer(scenes[scene_of[i]])
            try:
                alone = r.render(cams.subset(i), mlp_prec=prec[i], step=steps[i], feat_prec=feats[i])
                torch.cuda.synchronize()
                alone = alone.cpu().numpy()
            finally:
                r.close()
            assert np.array_equal(outs[i].cpu().numpy(), alone), i
    finally:
        srv.close()


def test_served_outputs_match_oracle(torch, merf, scenes):
    say("serving: 24 uneven requests over 3 scenes (fp32 / fp16 / bf16 MLP, fp32 or fp16-interpolated "
        "features) against the FP64 oracle")
    cams, scene_of, prec = request_mix(24, seed=13)
    feats = ["f16_interp" if i % 3 == 1 else "f32" for i in range(len(cams))]
    arr = merf.camera_array(cams)
    srv = merf.Server(slots=3, max_batch=8, use_graphs=True)
    try:
        ids = [srv.add_scene(s) for s in scenes]
        outs = [torch.full((int(w) * int(h), 4), float("nan"), device="cuda") for w, h in cams.size]
        torch.cuda.synchronize()
        tickets = [srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(),
                              merf.render_params(mlp_prec=prec[i], feat_prec=feats[i]))
                   for i in range(len(cams))]
        for t in tickets:
            srv.wait(t)
        for k in range(3):
            idx = [i for i in range(len(cams)) if scene_of[i] == k]
            sub = cams.subset(idx)
            ref, st = oracle.render(scenes[k], sub)
            gpu = np.concatenate([outs[i].cpu().numpy().astype(np.float64) for i in idx])
            check(gpu, ref, st["fragile"], f"served scene {k}: {len(idx)} requests", max_fragile=0.01,
                  min_psnr=MIN_PSNR_DB)
    finally:
        srv.close()


def test_arrivals_while_running_are_admitted(torch, merf, scenes):
    say("serving: requests arriving from another thread while launches run")
    cams, scene_of, prec = request_mix(40, seed=11)
    arr = merf.camera_array(cams)
    srv = merf.Server(slots=4, max_batch=4, use_graphs=True)
    try:
        ids = [srv.add_scene(s) for s in scenes]
        outs = [torch.empty((int(w) * int(h), 4), device="cuda") for w, h in cams.size]
        tickets = [None] * len(cams)

        def producer():
            for i in range(len(cams)):
                tickets[i] = srv.submit(ids[scene_of[i]], arr, i, outs[i].data_ptr(), merf.render_params())
                time.sleep(0.0002)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        srv.drain()
        st = srv.stats()
        say(f"  launches {st['launches']}, max in flight {st['max_inflight']}")
        assert st["completed"] == len(cams)
        for i in (0, 17, 39):
            alone = render_alone(torch, merf, scenes[scene_of[i]], cams, i, "f32")
            assert np.array_equal(outs[i].cpu().numpy(), alone)
        for t in tickets:
            lat, q = srv.wait(t)
            assert lat >= q >= 0.0
    finally:
        srv.close()


def test_admission_by_budget_and_eviction(torch, merf, scenes):
    say("serving: scene admission under an HBM budget")
    probe = merf.Server(slots=1)
    probe.add_scene(scenes[0])
    one = probe.stats()["resident_bytes"]
    probe.close()
    budget = 2 * one + one // 2                        # room for two scenes
    big = synth.preset_scene("tiny", seed=9)
    with pytest.raises(merf.MerfError) as e:           # a scene alone above the budget
        merf.Server(slots=1, hbm_budget=one // 2).add_scene(big)
    assert e.value.code == merf.MERF_E_OOM
    cams = synth.random_cameras(1, seed=3, sizes=[(48, 40)], inside=2.5)
    arr = merf.camera_array(cams)
    # without eviction: the third scene registers but stays absent; its
    # request waits until a removal frees memory
    srv = merf.Server(slots=2, hbm_budget=budget)
    try:
        a, b, c = [srv.add_scene(s) for s in scenes]
        st = srv.stats()
        assert st["registered"] == 3 and st["resident_scenes"] == 2 and st["resident_bytes"] <= budget
        out = torch.full((48 * 40, 4), float("nan"), device="cuda")
        torch.cuda.synchronize()
        t = srv.submit(c, arr, 0, out.data_ptr(), merf.render_params())
        time.sleep(0.2)
        assert not srv.poll(t)                          # no memory for scene c yet
        srv.remove_scene(a)
        srv.wait(t)
        st = srv.stats()
        assert st["resident_scenes"] == 2 and st["admissions"] == 3 and st["evictions"] == 0
        assert st["image_admissions"] == 0                 # every scene's first upload builds it
        alone = render_alone(torch, merf, scenes[2], cams, 0, "f32")
        assert np.array_equal(out.cpu().numpy(), alone)
    finally:
        srv.close()
    # with eviction: requests cycling over three scenes that do not fit
    # together; scenes are evicted and re-admitted
    srv = merf.Server(slots=2, max_batch=4, hbm_budget=budget, evict_idle=True)
    try:
        ids = [srv.add_scene(s) for s in scenes]
        assert srv.stats()["resident_scenes"] == 2
        n = 30
        order = [i % 3 for i in range(n)]
        cams = synth.random_cameras(n, seed=5, sizes=[(40, 24), (64, 64), (17, 9)] * 10, inside=2.5)
        arr = merf.camera_array(cams)
        outs = [torch.full((int(w) * int(h), 4), float("nan"), device="cuda") for w, h in cams.size]
        torch.cuda.synchronize()
        ts = [srv.submit(ids[order[i]], arr, i, outs[i].data_ptr(), merf.render_params()) for i in range(n)]
        for t in ts:
            srv.wait(t)
        st = srv.stats()
        say(f"  launches {st['launches']}, admissions {st['admissions']} ({st['image_admissions']} from "
            f"device images), evictions {st['evictions']}")
        assert st["completed"] == n and st["evictions"] >= 1 and st["admissions"] == 2 + st["evictions"]
        # the first admission of each scene builds it; every later one copies
        # the device image kept from that build
        assert st["image_admissions"] == st["admissions"] - 3
        assert st["resident_bytes"] <= budget and st["resident_scenes"] <= 2
        for i in range(n):
            alone = render_alone(torch, merf, scenes[order[i]], cams, i, "f32")
            assert np.array_equal(outs[i].cpu().numpy(), alone), i
    finally:
        srv.close()


def test_eviction_keeps_the_most_requested_scene(torch, merf, scenes):
    """Of two resident scenes, the one with more recent requests stays when a
    third needs room, even if the other was used last."""
    say("serving: eviction order by request counts")
    probe = merf.Server(slots=1)
    probe.add_scene(scenes[0])
    one = probe.stats()["resident_bytes"]
    probe.close()
    srv = merf.Server(slots=2, max_batch=4, hbm_budget=2 * one + one // 2, evict_idle=True)
    try:
        a, b, c = [srv.add_scene(s) for s in scenes]
        assert srv.stats()["resident_scenes"] == 2             # a and b
        order = [a] * 8 + [b] + [c] + [a]
        cams = synth.random_cameras(len(order), seed=23, sizes=[(40, 32)] * len(order), inside=2.5)
        arr = merf.camera_array(cams)
        outs = [torch.full((40 * 32, 4), float("nan"), device="cuda") for _ in order]
        torch.cuda.synchronize()
        for i, sid in enumerate(order):                       # one at a time: b is used after a
            srv.wait(srv.submit(sid, arr, i, outs[i].data_ptr(), merf.render_params()))
            if i == 9:
                st = srv.stats()
                assert st["admissions"] == 3 and st["evictions"] == 1
        st = srv.stats()
        say(f"  admissions {st['admissions']}, evictions {st['evictions']}")
        assert st["admissions"] == 3 and st["evictions"] == 1     # a stayed: b made room for c
        for i, sid in enumerate(order):
            alone = render_alone(torch, merf, scenes[[a, b, c].index(sid)], cams, i, "f32")
            assert np.array_equal(outs[i].cpu().numpy(), alone), i
    finally:
        srv.close()


def test_readmission_from_device_image_full_size(torch, merf):
    """Two 256^3 / 1024^2 scenes (three occupancy levels, the empty-space
    grids of the full-size layout) under a budget that holds one: every
    re-admission copies the device image kept from the first upload, and
    every request still gets merf_render's image bit for bit."""
    say("serving: re-admission from device images, 256^3 / 1024^2 scenes")
    two = synth.serving_scenes(seeds=(100, 103))
    sizes = []
    for sc in two:
        probe = merf.Server(slots=1)
        probe.add_scene(sc)
        sizes.append(probe.stats()["resident_bytes"])
        probe.close()
    srv = merf.Server(slots=2, max_batch=2, hbm_budget=max(sizes) + min(sizes) // 2, evict_idle=True)
    try:
        ids = [srv.add_scene(sc) for sc in two]
        order = [0, 1, 0, 1, 1, 0]
        cams = synth.random_cameras(len(order), seed=29, sizes=[(96, 64), (61, 37)] * 3, inside=1.5)
        arr = merf.camera_array(cams)
        outs = [torch.full((int(w) * int(h), 4), float("nan"), device="cuda") for w, h in cams.size]
        torch.cuda.synchronize()
        for i, k in enumerate(order):                 # one at a time: each switch evicts the other scene
            srv.wait(srv.submit(ids[k], arr, i, outs[i].data_ptr(), merf.render_params()))
        st = srv.stats()
        say(f"  admissions {st['admissions']} ({st['image_admissions']} from device images), "
            f"evictions {st['evictions']}")
        assert st["evictions"] >= 3 and st["image_admissions"] == st["admissions"] - 2
        for i, k in enumerate(order):
            alone = render_alone(torch, merf, two[k], cams, i, "f32")
            assert np.array_equal(outs[i].cpu().numpy(), alone), i
    finally:
        srv.close()


def test_admission_while_serving_from_threads(torch, merf, scenes):
    """Two client threads keep requesting four scenes, of which two fit: the
    loader must drain and evict scenes that are in use, and every request
    still gets its image."""
    say("serving: admission by memory under load from two threads")
    probe = merf.Server(slots=1)
    probe.add_scene(scenes[0])
    one = probe.stats()["resident_bytes"]
    probe.close()
    four = scenes + [synth.preset_scene("tiny", seed=4)]
    srv = merf.Server(slots=3, max_batch=6, hbm_budget=2 * one + one // 2, evict_idle=True)
    try:
        ids = [srv.add_scene(s) for s in four]
        n = 48
        rng = np.random.default_rng(17)
        which = rng.integers(0, 4, n)
        cams = synth.random_cameras(n, seed=19, sizes=[(32, 32), (56, 24)] * (n // 2), inside=2.5)
        arr = merf.camera_array(cams)
        outs = [torch.full((int(w) * int(h), 4), float("nan"), device="cuda") for w, h in cams.size]
        torch.cuda.synchronize()
        tickets = [None] * n

        def client(k):
            for i in range(k, n, 2):
                tickets[i] = srv.submit(ids[which[i]], arr, i, outs[i].data_ptr(), merf.render_params())
                time.sleep(0.0005)

        ths = [threading.Thread(target=client, args=(k,)) for k in (0, 1)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        srv.drain()
        st = srv.stats()
        say(f"  launches {st['launches']} (mixed-scene {st['mixed_launches']}), admissions {st['admissions']}, "
            f"evictions {st['evictions']}")
        assert st["completed"] == n and st["evictions"] >= 1
        assert st["image_admissions"] == st["admissions"] - 4
        for i in range(n):
            alone = render_alone(torch, merf, four[which[i]], cams, i, "f32")
            assert np.array_equal(outs[i].cpu().numpy(), alone), i
    finally:
        srv.close()


def test_launch_beyond_largest_class_is_persistent(torch, merf):
    """A launch of more tiles than the largest one-workgroup-per-tile class
    (262144) runs on the persistent grid, whose workgroups take tiles from
    per-XCD counters that a kernel node zeroes before each launch: two such
    launches in a row, then a small one, each request bitwise as rendered
    alone."""
    say("serving: two launches of one 8192x2176 request (278528 tiles each, persistent grid), then a small one")
    scene = synth.preset_scene("tiny", seed=5)
    sizes = [(8192, 2176)] * 2 + [(96, 64)]
    cams = synth.random_cameras(len(sizes), seed=29, sizes=sizes, inside=2.5)
    arr = merf.camera_array(cams)
    srv = merf.Server(slots=1, max_batch=1, use_graphs=True)
    try:
        sid = srv.add_scene(scene)
        outs = [torch.full((w * h, 4), float("nan"), device="cuda") for w, h in sizes]
        torch.cuda.synchronize()
        tickets = [srv.submit(sid, arr, i, outs[i].data_ptr(), merf.render_params()) for i in range(len(sizes))]
        for t in tickets:
            srv.wait(t)
        st = srv.stats()
        say(f"  launches {st['launches']} (graph {st['graph_launches']})")
        assert st["completed"] == len(sizes) and st["launches"] == 3
        r = merf.Renderer(scene)
        try:
            for i in range(len(sizes)):
                alone = r.render(cams.subset(i))
                torch.cuda.synchronize()
                assert torch.equal(outs[i], alone), i
        finally:
            r.close()
    finally:
        srv.close()


def test_launch_class_boundary(torch, merf):
    """262144 tiles (4096x4096) is the largest launch with a workgroup per
    tile; 262656 tiles (4096x4104) takes the persistent grid.  Each request
    bitwise as rendered alone."""
    say("serving: launches of 262144 tiles (one workgroup per tile) and 262656 tiles (persistent grid)")
    scene = synth.preset_scene("tiny", seed=6)
    sizes = [(4096, 4096), (4096, 4104)]
    cams = synth.random_cameras(len(sizes), seed=31, sizes=sizes, inside=2.5)
    arr = merf.camera_array(cams)
    srv = merf.Server(slots=1, max_batch=1, use_graphs=True)
    try:
        sid = srv.add_scene(scene)
        outs = [torch.full((w * h, 4), float("nan"), device="cuda") for w, h in sizes]
        torch.cuda.synchronize()
        tickets = [srv.submit(sid, arr, i, outs[i].data_ptr(), merf.render_params()) for i in range(len(sizes))]
        for t in tickets:
            srv.wait(t)
        assert srv.stats()["launches"] == 2
        r = merf.Renderer(scene)
        try:
            for i in range(len(sizes)):
                alone = r.render(cams.subset(i))
                torch.cuda.synchronize()
                assert torch.equal(outs[i], alone), i
        finally:
            r.close()
    finally:
        srv.close()


def test_busy_scene_cannot_be_removed(torch, merf, scenes):
    say("serving: removing a scene with queued work is refused")
    srv = merf.Server(slots=1, max_batch=1)
    try:
        sid = srv.add_scene(scenes[0])
        cams = synth.tiny_camera(w=128, h=128)
        arr = merf.camera_array(cams)
        outs = [torch.empty((128 * 128, 4), device="cuda") for _ in range(8)]
        ts = [srv.submit(sid, arr, 0, o.data_ptr(), merf.render_params()) for o in outs]
        busy = not srv.poll(ts[-1])
        if busy:
            with pytest.raises(merf.MerfError):
                srv.remove_scene(sid)
        srv.drain()
        srv.remove_scene(sid)
        assert srv.stats()["resident_scenes"] == 0
    finally:
        srv.close()
