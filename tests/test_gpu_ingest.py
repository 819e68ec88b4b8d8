"""GPU tests of device-side ingest: the occupancy max-pool entry point
matches a numpy max-pool bit for bit, and the same pyramid drives the
renderer to the oracle's image."""
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
    print("tiny scene with a device-built occupancy pyramid", flush=True)
    fine = tiny_scene.occ[-1][1]
    outs = merf.occupancy_pyramid(torch.from_numpy(np.ascontiguousarray(fine)).cuda(), (2, 1))
    torch.cuda.synchronize()
    import dataclasses
    sc = dataclasses.replace(tiny_scene, occ=[(o.shape[0], o.cpu().numpy()) for o in outs])
    assert all(np.array_equal(a[1], b[1]) for a, b in zip(sc.occ, tiny_scene.occ))
    r = merf.Renderer(sc)
    try:
        gpu = r.render(tiny_cams)
        torch.cuda.synchronize()
        gpu = gpu.cpu().numpy().astype(np.float64)
    finally:
        r.close()
    ref, st = oracle.render(tiny_scene, tiny_cams)
    ok = st["fragile"] == 0
    assert np.abs(gpu - ref)[ok].max() <= 2.0 / 255.0
