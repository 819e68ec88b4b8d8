"""GPU tests of device-side ingest: the occupancy max-pool entry point
matches a numpy max-pool bit for bit, and the pyramid it builds is uploaded
from device memory and drives the renderer to the oracle's image."""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("res,factors", [(64, (16, 8, 2, 1)), (128, (32, 8, 4)), (48, (3, 16, 48))])
def test_maxpool_matches_numpy(torch, merf, res, factors):
    print(f"max-pool {res}^3 by {factors}", flush=True)
    rng = np.random.default_rng(res)
    mask = (rng.random((res, res, res)) < 0.01).astype(np.uint8) * rng.integers(1, 255, (res, res, res), dtype=np.uint8)
    outs = merf.occupancy_pyramid(torch.from_numpy(mask).cuda(), factors)
    torch.cuda.synchronize()
    for f, o in zip(factors, outs):
        want = synth.maxpool((mask > 0).astype(np.uint8), f) if f > 1 else (mask > 0).astype(np.uint8)
        assert np.array_equal(o.cpu().numpy(), want), f


def test_device_pyramid_renders_like_host_pyramid(torch, merf, tiny_scene, tiny_cams):
    """The pyramid built on the device (merf_occupancy_pyramid) is uploaded
    straight from device memory -- by merf_scene_upload and by the server --
    and renders the oracle's image."""
    print("tiny scene with a device-built occupancy pyramid, uploaded from device memory", flush=True)
    import dataclasses
    fine = tiny_scene.occ[-1][1]
    outs = merf.occupancy_pyramid(torch.from_numpy(np.ascontiguousarray(fine)).cuda(), (2, 1))
    torch.cuda.synchronize()
    assert all(np.array_equal(o.cpu().numpy(), h[1]) for o, h in zip(outs, tiny_scene.occ))
    # levels, planes and blocks as device tensors (block_index stays on the host)
    sc = dataclasses.replace(tiny_scene, occ=[(o.shape[0], o) for o in outs],
                             planes=torch.from_numpy(np.ascontiguousarray(tiny_scene.planes)).cuda(),
                             blocks=torch.from_numpy(np.ascontiguousarray(tiny_scene.blocks)).cuda())
    r = merf.Renderer(sc)
    try:
        gpu = r.render(tiny_cams)
        torch.cuda.synchronize()
        gpu = gpu.cpu().numpy()
    finally:
        r.close()
    ref, st = oracle.render(tiny_scene, tiny_cams)
    ok = st["fragile"] == 0
    assert np.abs(gpu.astype(np.float64) - ref)[ok].max() <= 2.0 / 255.0
    assert np.abs(gpu.astype(np.float64) - ref).mean() <= 1e-3
    # the same image as the host-built pyramid, bit for bit
    r = merf.Renderer(tiny_scene)
    try:
        host = r.render(tiny_cams)
        torch.cuda.synchronize()
        assert np.array_equal(host.cpu().numpy(), gpu)
    finally:
        r.close()
    # the server registers the scene from the same device arrays
    srv = merf.Server(slots=1)
    try:
        sid = srv.add_scene(sc)
        out = torch.full((tiny_cams.num_pixels(), 4), float("nan"), device="cuda")
        torch.cuda.synchronize()
        srv.wait(srv.submit(sid, merf.camera_array(tiny_cams), 0, out.data_ptr(), merf.render_params()))
        assert np.array_equal(out.cpu().numpy(), gpu)
    finally:
        srv.close()


def chebyshev_brute(levels):
    """Distance grid by definition: for each finest cell, the L-infinity
    distance in cells to the nearest cell occupied at every level (capped at
    255; 255 when there is none)."""
    rf = levels[-1].shape[0]
    comb = np.ones((rf,) * 3, bool)
    for o in levels:
        k = rf // o.shape[0]
        comb &= np.repeat(np.repeat(np.repeat(o > 0, k, 0), k, 1), k, 2)
    occ = np.argwhere(comb).astype(np.int32)
    if len(occ) == 0:
        return np.full((rf,) * 3, 255, np.uint8)
    cells = np.indices((rf,) * 3).reshape(3, -1).T.astype(np.int32)
    best = np.full(len(cells), 255, np.int32)
    for i in range(0, len(occ), 64):
        d = np.abs(cells[:, None, :] - occ[None, i:i + 64, :]).max(axis=2).min(axis=1)
        best = np.minimum(best, d)
    return np.minimum(best, 255).astype(np.uint8).reshape((rf,) * 3)


@pytest.mark.parametrize("case", ["pyramid", "and_of_levels", "empty", "cap"])
def test_distance_grid_matches_definition(torch, merf, case):
    print(f"distance grid: {case}", flush=True)
    rng = np.random.default_rng(7)
    if case == "pyramid":            # a max-pool pyramid 4 / 16 / 32
        fine = (rng.random((32, 32, 32)) < 0.003).astype(np.uint8)
        levels = [synth.maxpool(fine, 8), synth.maxpool(fine, 2), fine]
    elif case == "and_of_levels":    # coarse levels that are not max-pools: the AND decides
        fine = (rng.random((24, 24, 24)) < 0.02).astype(np.uint8)
        levels = [(rng.random((6, 6, 6)) < 0.5).astype(np.uint8), (rng.random((12, 12, 12)) < 0.7).astype(np.uint8),
                  fine]
    elif case == "empty":
        levels = [np.zeros((4, 4, 4), np.uint8), np.zeros((16, 16, 16), np.uint8)]
    else:                            # distances beyond 255 are capped
        fine = np.zeros((320, 320, 320), np.uint8)
        fine[3, 5, 7] = 1
        levels = [fine]
    want = chebyshev_brute(levels)
    got = merf.distance_grid([torch.from_numpy(np.ascontiguousarray(o)).cuda() for o in levels])
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]


def octant_brute(levels):
    """Octant extents by definition: for each finest cell and octant o (bit 0:
    -x, bit 1: -y, bit 2: -z), the largest k <= 255 such that the k-cell cube
    with a corner at the cell, extending in o's directions and clipped to the
    grid, has no cell occupied at every level; 0 for such a cell."""
    rf = levels[-1].shape[0]
    comb = np.ones((rf,) * 3, bool)
    for o in levels:
        k = rf // o.shape[0]
        comb &= np.repeat(np.repeat(np.repeat(o > 0, k, 0), k, 1), k, 2)
    out = np.zeros((8, rf, rf, rf), np.uint8)
    for o in range(8):
        for z in range(rf):
            for y in range(rf):
                for x in range(rf):
                    if comb[z, y, x]:
                        continue
                    k = 1
                    while k < 255:
                        lo = [c - k if (o >> a) & 1 else c for a, c in enumerate((x, y, z))]
                        hi = [c + 1 if (o >> a) & 1 else c + k + 1 for a, c in enumerate((x, y, z))]
                        sl = comb[max(lo[2], 0):min(hi[2], rf), max(lo[1], 0):min(hi[1], rf),
                                  max(lo[0], 0):min(hi[0], rf)]
                        if sl.any():
                            break
                        k += 1
                    out[o, z, y, x] = k
    return out


@pytest.mark.parametrize("case", ["pyramid", "and_of_levels", "empty"])
def test_octant_extent_grid_matches_definition(torch, merf, case):
    print(f"octant extent grid: {case}", flush=True)
    rng = np.random.default_rng(11)
    if case == "pyramid":
        fine = (rng.random((16, 16, 16)) < 0.01).astype(np.uint8)
        levels = [synth.maxpool(fine, 4), synth.maxpool(fine, 2), fine]
    elif case == "and_of_levels":
        fine = (rng.random((12, 12, 12)) < 0.05).astype(np.uint8)
        levels = [(rng.random((3, 3, 3)) < 0.6).astype(np.uint8), fine]
    else:
        levels = [np.zeros((2, 2, 2), np.uint8), np.zeros((8, 8, 8), np.uint8)]
    want = octant_brute(levels)
    got = merf.distance_grid([torch.from_numpy(np.ascontiguousarray(o)).cuda() for o in levels], octants=True)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]
