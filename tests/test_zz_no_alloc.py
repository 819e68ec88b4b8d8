"""merf_render_noalloc, the render entry point that allocates nothing,
against merf_render through the C ABI: the same image bit for bit on two
calls in a row (the second smaller), both in tile order, with the oracle
checking sampled rows of the first; launches beyond its fixed buffers are
rejected before anything runs."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import check, rows_of, say

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


def _both(torch, merf, handle, cams, **kw):
    """The image of merf_render and of merf_render_noalloc (each output
    filled with NaN first, so an unwritten pixel shows)."""
    n = cams.num_pixels()
    st = torch.cuda.current_stream().cuda_stream
    arr = merf.camera_array(cams)
    p = merf.render_params(**kw)
    ref = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
    got = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
    merf.merf_render(handle, arr, len(cams), p, ref.data_ptr(), st)
    merf.merf_render_noalloc(handle, arr, len(cams), p, got.data_ptr(), st)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_matches_render_on_two_calls(torch, merf):
    scene = synth.preset_scene("full")
    handle = merf.scene_upload(scene)
    try:
        # call 1: one 1920x1080 view (32400 tiles, heaviest-first order)
        cams = synth.full_camera()
        say("noalloc call 1: full scene, 1920x1080, tile order")
        ref, got = _both(torch, merf, handle, cams)
        assert np.all(np.isfinite(got))
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))
        stride, off = 27, 13
        want, st = oracle.render(scene, cams, rows_stride=stride, row_offset=off)
        check(got[rows_of(cams, stride, off)].astype(np.float64), want, st["fragile"], "noalloc 1080p sampled rows")
        # call 2, smaller: a 1024x576 view (9216 tiles, still ordered) and a
        # 333x217 one in the same launch; the fixed buffers hold call 1's
        # larger order, which this launch must not read
        small = synth.concat_cameras([synth.full_camera(w=1024, h=576), synth.full_camera(seed=5, w=333, h=217)])
        say("noalloc call 2: 1024x576 + 333x217, tile order")
        ref2, got2 = _both(torch, merf, handle, small)
        assert np.all(np.isfinite(got2))
        assert np.array_equal(ref2.view(np.uint32), got2.view(np.uint32))
        # a launch below the ordered range, and the plain order
        say("noalloc: tiny launch and plain order")
        tiny = synth.full_camera(w=96, h=64)
        r3, g3 = _both(torch, merf, handle, tiny)
        assert np.array_equal(r3.view(np.uint32), g3.view(np.uint32))
        r4, g4 = _both(torch, merf, handle, small, order="plain")
        assert np.array_equal(r4.view(np.uint32), g4.view(np.uint32))
        assert np.array_equal(r4.view(np.uint32), got2.view(np.uint32))
        # the reduced-precision kernel variants take the same path
        say("noalloc: fp16 interpolation with the bf16 MLP, tile order")
        r5, g5 = _both(torch, merf, handle, cams, feat_prec="f16_interp", mlp_prec="bf16")
        assert np.array_equal(r5.view(np.uint32), g5.view(np.uint32))
    finally:
        merf.merf_free(handle)


def test_noalloc_rejects_launch_beyond_fixed_buffers(torch, merf, tiny_scene):
    handle = merf.scene_upload(tiny_scene)
    try:
        # five 1080p views in one launch: 162000 tiles > 131072
        cams = synth.concat_cameras([synth.full_camera(seed=s) for s in range(5)])
        n = cams.num_pixels()
        out = torch.full((n, 4), -7.0, dtype=torch.float32, device="cuda")
        arr = merf.camera_array(cams)
        st = torch.cuda.current_stream().cuda_stream
        say("noalloc: oversize launch rejected")
        with pytest.raises(merf.MerfError) as ei:
            merf.merf_render_noalloc(handle, arr, len(cams), merf.render_params(), out.data_ptr(), st)
        assert ei.value.code == merf.MERF_E_INVALID
        assert "131072" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((out == -7.0).all())              # nothing ran
        # the plain order needs no fixed buffer
        merf.merf_render_noalloc(handle, arr, len(cams), merf.render_params(order="plain"), out.data_ptr(), st)
        ref = torch.empty_like(out)
        merf.merf_render(handle, arr, len(cams), merf.render_params(order="plain"), ref.data_ptr(), st)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32))
    finally:
        merf.merf_free(handle)
