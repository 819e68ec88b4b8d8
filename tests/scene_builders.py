"""Hand-built scenes with known content for closed-form tests (CPU only)."""
import numpy as np

import synth


def dense_scene(L=16, R=16, fill_grid=None, fill_planes=None, occ_fine=None, seed=0, pools=(2, 1),
                mlp=None):
    """All blocks stored.  fill_grid(z, y, x, c) / fill_planes(plane, v, u, c)
    give byte values (broadcast index grids); default random."""
    rng = np.random.default_rng(seed)
    B, C = 8, 8
    nb = L // B
    if fill_grid is None:
        grid = rng.integers(0, 256, (L, L, L, C), dtype=np.uint8)
    else:
        z, y, x, c = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), np.arange(C), indexing="ij")
        grid = np.asarray(fill_grid(z, y, x, c)).astype(np.uint8) * np.ones((L, L, L, C), np.uint8)
    blocks = grid.reshape(nb, B, nb, B, nb, B, C).transpose(0, 2, 4, 1, 3, 5, 6).reshape(nb ** 3, B, B, B, C)
    block_index = np.arange(nb ** 3, dtype=np.int32)
    if fill_planes is None:
        planes = rng.integers(0, 256, (3, R, R, C), dtype=np.uint8)
    else:
        pl, v, u, c = np.meshgrid(np.arange(3), np.arange(R), np.arange(R), np.arange(C), indexing="ij")
        planes = np.asarray(fill_planes(pl, v, u, c)).astype(np.uint8) * np.ones((3, R, R, C), np.uint8)
    rf = L // 4
    if occ_fine is None:
        occ_fine = np.ones((rf, rf, rf), np.uint8)
    occ = [(rf // p, synth.maxpool(occ_fine, p) if p > 1 else occ_fine.copy()) for p in pools]
    if mlp is None:
        mlp = np.random.default_rng(seed + 7).normal(0, 0.1, synth.mlp_param_count()).astype(np.float32)
    return synth.Scene(name="dense", seed=seed, L=L, R=R, block_index=block_index,
                       blocks=np.ascontiguousarray(blocks), planes=planes, occ=occ, mlp=mlp, step=4.0 / R)


def grid_bytes(scene):
    """Dense [L, L, L, C] byte grid (z, y, x, c) with zeros for absent blocks."""
    L, B, C = scene.L, scene.B, scene.C
    nb = L // B
    g = np.zeros((nb ** 3, B, B, B, C), np.uint8)
    present = scene.block_index >= 0
    g[present] = scene.blocks[scene.block_index[present]]
    return g.reshape(nb, nb, nb, B, B, B, C).transpose(0, 3, 1, 4, 2, 5, 6).reshape(L, L, L, C)
