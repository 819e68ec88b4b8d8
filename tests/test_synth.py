"""Invariants of the seeded scene generator."""
import numpy as np

import synth


def test_tiny_scene_structure(tiny_scene):
    s = tiny_scene
    nb = s.L // s.B
    assert s.block_index.shape == (nb ** 3,)
    assert s.blocks.shape == (s.num_blocks, 8, 8, 8, 8)
    assert s.planes.shape == (3, s.R, s.R, 8)
    present = s.block_index >= 0
    assert present.sum() == s.num_blocks
    assert np.array_equal(np.sort(s.block_index[present]), np.arange(s.num_blocks))
    (rc, coarse), (rf, fine) = s.occ
    assert rf == s.L // 4 and rc == s.L // 8
    assert np.array_equal(coarse, synth.maxpool(fine, 2))
    # the block mask is the L/8 occupancy level
    assert np.array_equal(coarse.reshape(-1).astype(bool), present)
    frac = s.num_blocks / nb ** 3
    assert 0.10 <= frac < 0.25


def test_occupancy_only_in_reachable_cells(tiny_scene):
    rf, fine = tiny_scene.occ[-1]
    assert not np.any(fine[~synth.reachable_mask(rf)])


def test_deterministic_and_seed_dependent():
    a = synth.preset_scene("tiny")
    b = synth.preset_scene("tiny")
    c = synth.preset_scene("tiny", seed=5)
    assert np.array_equal(a.blocks, b.blocks) and np.array_equal(a.planes, b.planes)
    assert np.array_equal(a.mlp, b.mlp)
    assert not np.array_equal(a.planes, c.planes)


def test_cameras():
    c = synth.tiny_camera()
    assert len(c) == 1 and c.num_pixels() == 128 * 128
    R = c.c2w[0, :, :3].astype(np.float64)
    assert np.allclose(R.T @ R, np.eye(3), atol=1e-6)
    assert abs(np.linalg.norm(c.c2w[0, :, 3]) - 3.0) < 1e-5
    # forward axis points at the origin
    f = R[:, 2]
    assert np.allclose(f, -c.c2w[0, :, 3] / 3.0, atol=1e-6)
    o = synth.orbit_cameras(4, w=64, h=32)
    assert o.num_pixels() == 4 * 64 * 32
