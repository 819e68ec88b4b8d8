"""GPU tests of the measurement entry points (include/merf_measure.h): the
gather record renders the same image as merf_render, records one entry per
evaluated sample with in-range offsets, and the replay re-issues them; the
phase profile renders the same image and fills its slots consistently."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def merf():
    from paper_2302_12249_amd import merf as m
    m.load()
    return m


@pytest.mark.parametrize("cap", [64, 2])
def test_record_and_replay(torch, merf, tiny_scene, cap):
    print(f"gather record / replay, tiny view, cap {cap}", flush=True)
    cams = synth.tiny_camera(w=100, h=60)          # ragged: 13 x 8 tiles
    r = merf.Renderer(tiny_scene)
    try:
        plain = r.render(cams)
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        r.render(cams, stats=st)
        rec = merf.GatherRecord(r.handle, cams, cap=cap)
        out = rec.replay()
        torch.cuda.synchronize()
        assert rec.n_slots == 13 * 8 * 64
        assert torch.equal(rec.image, plain)
        count = rec.count.cpu().numpy()
        assert count.sum() == int(st[3]) == int(rec.stats[3])
        assert np.array_equal(out[:, 0].cpu().numpy(), np.minimum(count, cap).astype(np.float32))
        # every recorded offset lies inside its array
        R = tiny_scene.R
        nbl = tiny_scene.L // 8
        recs = rec.rec.cpu().numpy().view(np.uint32)
        k = np.arange(cap)[:, None]
        valid = k < count[None, :]
        planes = recs[..., :3][valid]
        assert planes.max() + R * 8 + 16 <= 3 * R * R * 8
        grid = recs[..., 3][valid]
        assert (grid >> 13).max() < nbl ** 3 and (grid & 8191).max() < 9 * 9 * 9 * 8
    finally:
        r.close()


def test_record_full_view_heavy_first_order(torch, merf):
    print("gather record, full 1080p view: tile order is a permutation, heavy tiles first, replay in that order",
          flush=True)
    scene = synth.preset_scene("full")
    cams = synth.full_camera()
    r = merf.Renderer(scene)
    try:
        plain = r.render(cams, order="plain")
        rec = merf.GatherRecord(r.handle, cams, cap=1)
        out = rec.replay()
        torch.cuda.synchronize()
        assert torch.equal(rec.image, plain)
        tiles = rec.n_slots // 64
        order = rec.order.cpu().numpy()
        assert np.array_equal(np.sort(order), np.arange(tiles))
        work = rec.count.cpu().numpy().reshape(tiles, 64).sum(1)[order]
        # the tiles run first carry far more samples than those run last
        head, tail = work[: tiles // 10].mean(), work[tiles // 2:].mean()
        print(f"  evaluated samples per tile: first 10% {head:.1f}, last 50% {tail:.1f}", flush=True)
        assert head > 4 * tail
        count = rec.count.cpu().numpy()
        assert np.array_equal(out[:, 0].cpu().numpy(), np.minimum(count, 1).astype(np.float32))
        # the plain order records the identity
        rec2 = merf.GatherRecord(r.handle, cams, cap=1, order="plain")
        torch.cuda.synchronize()
        assert np.array_equal(rec2.order.cpu().numpy(), np.arange(tiles))
        assert torch.equal(rec2.count, rec.count)
    finally:
        r.close()


def test_phase_profile_fields(torch, merf, tiny_scene):
    """merf_render_phases: same image as merf_render; one wave per tile; the
    loop counters in their slots agree with the statistics counters."""
    print("phase profile, tiny view", flush=True)
    cams = synth.tiny_camera(w=100, h=60)          # 13 x 8 tiles
    r = merf.Renderer(tiny_scene)
    try:
        plain = r.render(cams)
        out = torch.empty_like(plain)
        ph = merf.render_phases(r.handle, cams, out)
        torch.cuda.synchronize()
        assert torch.equal(out, plain)
        st = ph["stats"]
        assert ph["waves"] == 13 * 8
        assert st["rays"] == 100 * 60
        # every evaluated sample is shaded once; samples parked past a ray's
        # termination are shaded and dropped
        assert ph["shade_lanes"] >= st["evaluated"]
        assert ph["shade_lanes"] <= 64 * ph["shade_passes"]
        assert ph["rounds"] >= ph["shade_passes"] >= 1
        assert ph["march_passes"] >= ph["open_passes"]
        for k in ("setup_cycles", "march_cycles", "shade_cycles", "composite_cycles", "mlp_cycles"):
            assert ph[k] > 0, k
    finally:
        r.close()
