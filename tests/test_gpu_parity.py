"""GPU parity: the HIP renderer (through the C ABI) against the FP64 oracle.

Bar (gpu_helpers): RGB and alpha within 2/255 max abs on pixels the oracle
does not flag as fragile, and within 1e-3 mean abs over all pixels; the
fp16 / bf16 MLP and fp16-feature paths meet the same per-pixel bound and
45 dB PSNR; dequantisation bit exact; renders bitwise deterministic.
"""
import numpy as np
import pytest

import oracle
import synth
from exact_round import dequant_table, to_bits
from gpu_helpers import MAX_ABS, MIN_PSNR_DB, check, gpu_render, psnr, rows_of, say
from scene_builders import dense_scene

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("fmt,prec", [("f32", 0), ("f16", 1), ("bf16", 2)])
def test_dequant_bit_exact(torch, merf, fmt, prec):
    """f16 runs the fp16-feature render path's own routine (deq_f16) with the
    scale the upload computes; f32 / bf16 the correctly rounded values."""
    say(f"dequant bit-exact {fmt}")
    codes = torch.arange(256, dtype=torch.uint8, device="cuda")
    dt = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}[prec]
    for m in (7, 14):
        out = torch.empty(256, dtype=dt, device="cuda")
        merf.merf_dequantize(codes.data_ptr(), 256, float(m), prec, out.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        if prec == 0:
            got = out.cpu().numpy().view(np.uint32)
        elif prec == 1:
            got = out.cpu().numpy().view(np.uint16).astype(np.uint32)
        else:
            got = out.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.uint32)
        want = to_bits(dequant_table(m, fmt), fmt)
        assert np.array_equal(got, want), (fmt, m, np.nonzero(got != want)[0][:10])


def test_tiny_parity(torch, merf, tiny_scene, tiny_cams):
    say("tiny 128x128 parity")
    gpu = gpu_render(torch, merf, tiny_scene, tiny_cams)
    ref, st = oracle.render(tiny_scene, tiny_cams)
    check(gpu, ref, st["fragile"], "tiny")


def test_tiny_parity_world_delta(torch, merf, tiny_scene, tiny_cams):
    say("tiny world-delta parity")
    gpu = gpu_render(torch, merf, tiny_scene, tiny_cams, delta_mode=1)
    ref, st = oracle.render(tiny_scene, tiny_cams, delta_mode=1)
    check(gpu, ref, st["fragile"], "tiny world delta")


def test_tiny_no_termination_and_coarse_step(torch, merf, tiny_scene, tiny_cams):
    say("tiny t_min=0, step 1/32")
    gpu = gpu_render(torch, merf, tiny_scene, tiny_cams, t_min=0.0, step=1.0 / 32)
    ref, st = oracle.render(tiny_scene, tiny_cams, t_min=0.0, step=1.0 / 32)
    check(gpu, ref, st["fragile"], "tiny t_min=0 step=1/32")


def test_stats_counters_match_oracle(torch, merf, tiny_scene, tiny_cams):
    say("tiny stats counters")
    gpu, cnt = gpu_render(torch, merf, tiny_scene, tiny_cams, stats=True)
    ref, st = oracle.render(tiny_scene, tiny_cams)
    rays, lookups, visited, evaluated, contributing, terminated = cnt[:6]
    assert rays == tiny_cams.num_pixels()
    fr = st["fragile"] > 0
    slack = st["evaluated"][fr].sum() + 2 * fr.sum() + 2
    assert abs(int(evaluated) - st["evaluated"].sum()) <= slack
    # alpha != 0 is decided in each side's own precision: FP32 rounds
    # 1 - exp(-tau delta) to 0 below ~3e-8, FP64 does not, so the kernel skips
    # the appearance read of more samples (their weight is below 1e-7)
    assert int(contributing) <= st["contributing"].sum() + slack
    assert int(contributing) <= int(evaluated)
    assert abs(int(terminated) - (st["T"] < 2e-4).sum()) <= fr.sum() + 2
    # skipping visits at most the lattice samples the oracle visits
    assert visited <= st["visited"].sum()
    # each visited sample reads each level at most once (cells already known
    # to be occupied are not read again)
    assert 0 < lookups <= visited * len(tiny_scene.occ)


@pytest.mark.parametrize("kw", [{}, {"t_min": 0.0, "step": 1.0 / 32}, {"delta_mode": 1}])
def test_skip_modes_render_the_same_image(torch, merf, tiny_scene, tiny_cams, kw):
    say(f"tiny: distance-grid skipping vs level-by-level skipping {kw}")
    a, ca = gpu_render(torch, merf, tiny_scene, tiny_cams, stats=True, skip="distance", **kw)
    b, cb = gpu_render(torch, merf, tiny_scene, tiny_cams, stats=True, skip="levels", **kw)
    say(f"  visited {ca[2]} vs {cb[2]}, lookups {ca[1]} vs {cb[1]}, evaluated {ca[3]} vs {cb[3]}")
    # both skip only samples in empty cells, so they evaluate the same samples
    assert np.array_equal(a, b)
    assert ca[3] == cb[3] and ca[4] == cb[4] and ca[5] == cb[5]
    assert ca[2] <= cb[2]


def test_fine_occupancy_uses_chebyshev_grid(torch, merf, tiny_scene, tiny_cams):
    say("tiny scene with a 512^3 finest occupancy level (one shared Chebyshev grid instead of octant grids)")
    import dataclasses
    r0, fine = tiny_scene.occ[-1]
    up = np.repeat(np.repeat(np.repeat(fine, 512 // r0, 0), 512 // r0, 1), 512 // r0, 2)
    sc = dataclasses.replace(tiny_scene, occ=list(tiny_scene.occ) + [(512, np.ascontiguousarray(up))])
    a = gpu_render(torch, merf, sc, tiny_cams)
    b = gpu_render(torch, merf, sc, tiny_cams, skip="levels")
    base = gpu_render(torch, merf, tiny_scene, tiny_cams)
    # the added level refines the finest one without changing any decision
    assert np.array_equal(a, b)
    assert np.array_equal(a, base)


def test_ragged_batch_and_offsets(torch, merf, tiny_scene):
    say("ragged multi-camera batch")
    base = synth.tiny_camera()
    sizes = [(13, 7), (1, 1), (64, 33), (9, 16)]
    cams = synth.make_cameras([base.c2w[0].astype(np.float64)] * 4, sizes)
    cams.intr[1] = [0.5, 0.5, 0.5, 0.5]
    gpu = gpu_render(torch, merf, tiny_scene, cams)
    ref, st = oracle.render(tiny_scene, cams)
    check(gpu, ref, st["fragile"], "ragged batch")
    # each camera alone gives the same bits as inside the batch
    off = 0
    for i in range(len(cams)):
        n = sizes[i][0] * sizes[i][1]
        alone = gpu_render(torch, merf, tiny_scene, cams.subset(i))
        assert np.array_equal(alone, gpu[off:off + n])
        off += n


def test_more_cameras_than_one_launch(torch, merf, tiny_scene):
    say("20 cameras (two launches)")
    cams = synth.random_cameras(20, seed=5, sizes=[(24 + i, 17 + 2 * i) for i in range(20)], inside=2.5)
    gpu = gpu_render(torch, merf, tiny_scene, cams)
    ref, st = oracle.render(tiny_scene, cams)
    check(gpu, ref, st["fragile"], "20 cameras")


def test_deterministic(torch, merf, tiny_scene, tiny_cams):
    say("determinism")
    a = gpu_render(torch, merf, tiny_scene, tiny_cams)
    b = gpu_render(torch, merf, tiny_scene, tiny_cams)
    assert np.array_equal(a, b)


def test_empty_scene(torch, merf):
    say("empty occupancy")
    sc = dense_scene(L=16, R=16, occ_fine=np.zeros((4, 4, 4), np.uint8))
    cams = synth.tiny_camera(w=16, h=12)
    gpu = gpu_render(torch, merf, sc, cams)
    ref, st = oracle.render(sc, cams)
    assert np.all(gpu[:, 3] == 0)
    check(gpu, ref, st["fragile"], "empty scene")


def test_constant_box_closed_form(torch, merf):
    say("constant-density box")
    from test_oracle_render import box_scene, const_field
    lo, hi = np.array([0.0, -0.5, -0.5]), np.array([1.0, 0.5, 0.5])
    sc = box_scene(lo, hi)
    cams = synth.make_cameras([np.array([[0, 0, 1, -0.3], [1, 0, 0, 0.0], [0, 1, 0, 0.0]], float)], [(32, 32)],
                              hfov_deg=30.0)
    gpu = gpu_render(torch, merf, sc, cams)
    ref, st = oracle.render(sc, cams)
    # an axis-aligned camera puts whole pixel rows on cell faces: many fragile
    check(gpu, ref, st["fragile"], "box", max_fragile=None)
    # alpha = 1 - exp(-tau * sum of evaluated deltas) holds on the GPU too
    ok = (st["fragile"] == 0) & (st["evaluated"] > 0)
    assert np.allclose(gpu[ok, 3], ref[ok, 3], atol=2e-6)


def test_upload_free_accounting(torch, merf, tiny_scene):
    say("upload / free accounting")
    before = merf.hbm_in_use()
    h = merf.scene_upload(tiny_scene)
    nb = merf.scene_bytes(h)
    assert nb >= tiny_scene.planes.nbytes and merf.hbm_in_use() == before + nb
    merf.merf_free(h)
    assert merf.hbm_in_use() == before
    with pytest.raises(merf.MerfError):
        merf.merf_free(h)
    merf.set_hbm_budget(before + nb - 1)
    try:
        with pytest.raises(merf.MerfError) as e:
            merf.scene_upload(tiny_scene)
        assert e.value.code == merf.MERF_E_OOM
    finally:
        merf.set_hbm_budget(2 ** 63)


@pytest.fixture(scope="module")
def full_scene():
    return synth.preset_scene("full")


def test_full_1080p_parity_sampled_rows(torch, merf, full_scene):
    say("full 1920x1080 parity (every 27th row checked by the oracle)")
    cams = synth.full_camera()
    gpu = gpu_render(torch, merf, full_scene, cams)
    stride, off = 27, 13
    ref, st = oracle.render(full_scene, cams, rows_stride=stride, row_offset=off)
    check(gpu[rows_of(cams, stride, off)], ref, st["fragile"], "full 1080p sampled rows")
    assert gpu[:, 3].max() > 0.5      # the view sees content
    # the paper's level-by-level skipping gives the same image
    lv = gpu_render(torch, merf, full_scene, cams, skip="levels")
    assert np.array_equal(gpu, lv)
    # so does the plain tile order (the default runs the 32400 tiles
    # estimated heaviest first)
    pl = gpu_render(torch, merf, full_scene, cams, order="plain")
    assert np.array_equal(gpu, pl)


def test_tile_order_multi_camera_same_image(torch, merf, full_scene):
    say("full scene, 3 orbit views at 1280x720 in one launch (43200 tiles): heavy-first vs plain order")
    cams = synth.orbit_cameras(3, w=1280, h=720)
    a = gpu_render(torch, merf, full_scene, cams)
    b = gpu_render(torch, merf, full_scene, cams, order="plain")
    assert np.array_equal(a, b)
    # one camera alone (14400 tiles, ordered on its own) gives the same bits
    one = gpu_render(torch, merf, full_scene, cams.subset(1))
    n = 1280 * 720
    assert np.array_equal(one, a[n:2 * n])


def test_tile_order_ragged_batch(torch, merf, full_scene):
    say("full scene, ragged batch 1920x1080 + 640x480 + 333x217 + 1x1 in one launch: heavy-first vs plain order")
    base = synth.full_camera().c2w[0].astype(np.float64)
    orbit = synth.orbit_cameras(3, w=8, h=8).c2w
    poses = [base] + [orbit[i].astype(np.float64) for i in range(3)]
    cams = synth.make_cameras(poses, [(1920, 1080), (640, 480), (333, 217), (1, 1)])
    a = gpu_render(torch, merf, full_scene, cams)
    b = gpu_render(torch, merf, full_scene, cams, order="plain")
    assert np.array_equal(a, b)
    # the odd-sized camera alone (below the ordered size range) gives the same bits
    off = 1920 * 1080 + 640 * 480
    alone = gpu_render(torch, merf, full_scene, cams.subset(2))
    assert np.array_equal(alone, a[off:off + 333 * 217])


def test_tile_order_concurrent_streams(torch, merf, full_scene):
    say("full 1080p view rendered 12 times on 3 streams at once (tile-order work buffers shared and reused)")
    cams = synth.full_camera()
    r = merf.Renderer(full_scene)
    try:
        ref = r.render(cams, order="plain")
        streams = [torch.cuda.Stream() for _ in range(3)]
        outs = [torch.empty_like(ref) for _ in range(12)]
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            r.render(cams, out=o, stream=streams[i % 3])
        torch.cuda.synchronize()
        for o in outs:
            assert torch.equal(o, ref)
    finally:
        r.close()


def test_tile_order_many_frames_in_flight(torch, merf, full_scene):
    say("full 1080p view rendered 80 times back to back without waiting (more frames in flight than "
        "tile-order work buffers: buffers are reused, and calls that find all of them in flight keep the "
        "plain order)")
    cams = synth.full_camera()
    r = merf.Renderer(full_scene)
    try:
        ref = r.render(cams, order="plain")
        outs = [torch.empty_like(ref) for _ in range(80)]
        torch.cuda.synchronize()
        for o in outs:
            r.render(cams, out=o)
        torch.cuda.synchronize()
        for o in outs:
            assert torch.equal(o, ref)
    finally:
        r.close()


def test_tile_order_effort_key_boundary(torch, merf, full_scene):
    say("full scene at 2048x2048 (65536 tiles: probe rays evaluate samples) and 2048x2056 (65792 tiles: "
        "probe rays stop at the first occupied sample), both against the plain order")
    pose = synth.full_camera().c2w[0].astype(np.float64)
    for w, h in ((2048, 2048), (2048, 2056)):
        cams = synth.make_cameras([pose], [(w, h)])
        a = gpu_render(torch, merf, full_scene, cams)
        b = gpu_render(torch, merf, full_scene, cams, order="plain")
        assert np.array_equal(a, b), (w, h)
        assert a[:, 3].max() > 0.5


def test_tile_order_4k_frame(torch, merf, full_scene):
    say("full scene, one 3840x2160 view (129600 tiles, the largest ordered launch size range)")
    cams = synth.make_cameras([synth.full_camera().c2w[0].astype(np.float64)], [(3840, 2160)])
    a = gpu_render(torch, merf, full_scene, cams)
    b = gpu_render(torch, merf, full_scene, cams, order="plain")
    assert np.array_equal(a, b)
    assert a[:, 3].max() > 0.5


def test_tile_order_rejects_unknown_value(torch, merf, tiny_scene, tiny_cams):
    r = merf.Renderer(tiny_scene)
    try:
        with pytest.raises(merf.MerfError) as e:
            r.render(tiny_cams, order=2)
        assert e.value.code == merf.MERF_E_INVALID
    finally:
        r.close()


def test_full_scene_orbit_views_sampled(torch, merf, full_scene):
    say("full scene, 4 orbit views at 480x270 (outer regions)")
    cams = synth.orbit_cameras(4, w=480, h=270)
    gpu = gpu_render(torch, merf, full_scene, cams)
    ref, st = oracle.render(full_scene, cams, rows_stride=9, row_offset=4)
    check(gpu[rows_of(cams, 9, 4)], ref, st["fragile"], "orbit views")


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_precision_mlp_tiny(torch, merf, tiny_scene, tiny_cams, prec):
    say(f"tiny, deferred MLP in {prec} on MFMA")
    gpu = gpu_render(torch, merf, tiny_scene, tiny_cams, mlp_prec=prec)
    ref, st = oracle.render(tiny_scene, tiny_cams)
    check(gpu, ref, st["fragile"], f"tiny mlp {prec}", min_psnr=MIN_PSNR_DB)
    # alpha is untouched by the MLP precision
    f32 = gpu_render(torch, merf, tiny_scene, tiny_cams)
    assert np.array_equal(gpu[:, 3], f32[:, 3])


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_precision_mlp_full_sampled(torch, merf, full_scene, prec):
    say(f"full 1080p, deferred MLP in {prec} (every 54th row checked)")
    cams = synth.full_camera()
    gpu = gpu_render(torch, merf, full_scene, cams, mlp_prec=prec)
    ref, st = oracle.render(full_scene, cams, rows_stride=54, row_offset=7)
    check(gpu[rows_of(cams, 54, 7)], ref, st["fragile"], f"full mlp {prec}", min_psnr=MIN_PSNR_DB)


@pytest.mark.parametrize("feat", ["f16", "f16_interp"])
@pytest.mark.parametrize("mlp", ["f32", "f16", "bf16"])
def test_fp16_features_tiny(torch, merf, tiny_scene, tiny_cams, mlp, feat):
    say(f"tiny, features {feat}, MLP {mlp}")
    gpu = gpu_render(torch, merf, tiny_scene, tiny_cams, feat_prec=feat, mlp_prec=mlp)
    ref, st = oracle.render(tiny_scene, tiny_cams)
    check(gpu, ref, st["fragile"], f"tiny feat {feat} mlp {mlp}", min_psnr=MIN_PSNR_DB)
    if feat == "f16_interp":
        # density is summed in fp32 as in the fp32 path: the same alpha bit for bit
        f32 = gpu_render(torch, merf, tiny_scene, tiny_cams, mlp_prec=mlp)
        assert np.array_equal(gpu[:, 3], f32[:, 3])


@pytest.mark.parametrize("feat", ["f16", "f16_interp"])
def test_fp16_features_full_sampled(torch, merf, full_scene, feat):
    say(f"full 1080p, features {feat} + MLP fp16 (every 54th row checked)")
    cams = synth.full_camera()
    gpu = gpu_render(torch, merf, full_scene, cams, feat_prec=feat, mlp_prec="f16")
    ref, st = oracle.render(full_scene, cams, rows_stride=54, row_offset=7)
    check(gpu[rows_of(cams, 54, 7)], ref, st["fragile"], f"full feat {feat} mlp f16", min_psnr=MIN_PSNR_DB)
    if feat == "f16_interp":
        # density is summed in fp32 as in the fp32 path: the same alpha bit for bit
        f32 = gpu_render(torch, merf, full_scene, cams, mlp_prec="f16")
        assert np.array_equal(gpu[:, 3], f32[:, 3])


def test_precision_orbit_views_sampled(torch, merf, full_scene):
    say("full scene, 16 orbit views at 480x270, every precision combination against the oracle")
    cams = synth.orbit_cameras(16, w=480, h=270)
    ref, st = oracle.render(full_scene, cams, rows_stride=9, row_offset=4)
    sel = rows_of(cams, 9, 4)
    for mlp, feat in (("f32", "f32"), ("f16", "f32"), ("bf16", "f32"), ("f16", "f16"), ("bf16", "f16"),
                      ("f32", "f16_interp"), ("f16", "f16_interp"), ("bf16", "f16_interp")):
        gpu = gpu_render(torch, merf, full_scene, cams, mlp_prec=mlp, feat_prec=feat)
        check(gpu[sel], ref, st["fragile"], f"orbit mlp {mlp} feat {feat}", min_psnr=MIN_PSNR_DB)


@pytest.mark.parametrize("feat", ["f32", "f16", "f16_interp"])
def test_planes_only_variant(torch, merf, tiny_scene, tiny_cams, feat):
    say(f"tiny scene without its 3D grid (planes only), features {feat}")
    po = synth.planes_only(tiny_scene)
    gpu = gpu_render(torch, merf, po, tiny_cams, feat_prec=feat)
    ref, st = oracle.render(po, tiny_cams)
    check(gpu, ref, st["fragile"], f"planes only, features {feat}")


@pytest.mark.parametrize("feat", ["f32", "f16", "f16_interp"])
def test_grid_only_variant(torch, merf, tiny_cams, feat):
    say(f"grid-only scene (L = 128, no planes), features {feat}")
    go = synth.grid_only_scene(128, 0.08, seed=4)
    gpu = gpu_render(torch, merf, go, tiny_cams, feat_prec=feat)
    ref, st = oracle.render(go, tiny_cams)
    check(gpu, ref, st["fragile"], f"grid only, features {feat}")
