"""Seeded synthetic MERF scenes and cameras.

This module only *draws inputs*: random bytes, sphere-shaped occupancy,
max-pooled occupancy levels, random MLP weights and pinhole cameras.  It
contains none of the rendering arithmetic (no contraction, no
interpolation, no compositing), so both the FP64 oracle and the GPU path can
consume the same scenes without sharing any of the method's code.

Scene layout (the baked representation of MERF, Sec. 4.1 and Sec. 5.3):

* ``block_index``  int32 ``[(L/B)^3]``, z-major (``(bz*nb + by)*nb + bx``);
  ``-1`` marks an absent block, otherwise the slot in ``blocks``.
* ``blocks``       uint8 ``[num_blocks, B, B, B, C]`` indexed ``[z, y, x, c]``.
* ``planes``       uint8 ``[3, R, R, C]``; plane 0 is P_x indexed ``[z][y]``,
  plane 1 is P_y indexed ``[z][x]``, plane 2 is P_z indexed ``[y][x]``
  (row = second in-plane axis, column = first in-plane axis).
* ``occ``          list of ``(res, uint8[res, res, res])`` coarse to fine,
  z-major; a cell of level ``res`` covers an axis-aligned box of edge
  ``4/res`` tiling the contracted domain ``[-2, 2]^3``.
* channel order ``[density, diffuse r, g, b, feature 0..3]`` (C = 8, K = 4).
* ``mlp``          float32 parameters of the deferred MLP (App. B: 3 layers,
  16 hidden units): ``W0[in][h], b0[h], W1[h][h], b1[h], W2[h][3], b2[3]``.

Occupancy is drawn as random spheres placed directly in contracted space.
The finest level has resolution L/4; coarser levels are max-pools of it
(Sec. 6 builds its hierarchy by max-pooling a binary mask).  The level at
resolution L/B is the block mask: a block is stored iff its cell is occupied.
Cells that the piecewise-projective contraction cannot reach (boxes lying
outside [-1, 1] on two or more axes, Sec. 4.2) are left empty.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

BLOCK = 8
CHANNELS = 8
MLP_IN = 34      # 3 diffuse + 4 features + 3 direction + 24 sin/cos terms
MLP_HIDDEN = 16
MLP_OUT = 3


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    L: int
    R: int
    block_index: np.ndarray          # int32 [(L/B)^3]
    blocks: np.ndarray               # uint8 [nb, B, B, B, C]
    planes: np.ndarray               # uint8 [3, R, R, C]
    occ: List[Tuple[int, np.ndarray]]
    mlp: np.ndarray                  # float32 flat parameter vector
    m_density: float = 14.0
    m_feature: float = 7.0
    B: int = BLOCK
    C: int = CHANNELS
    mlp_in: int = MLP_IN
    mlp_hidden: int = MLP_HIDDEN
    step: float = 0.0                # default contracted step (4/R)

    @property
    def num_blocks(self) -> int:
        return int(self.blocks.shape[0])

    def nbytes(self) -> int:
        return int(self.block_index.nbytes + self.blocks.nbytes + self.planes.nbytes
                   + sum(o.nbytes for _, o in self.occ) + self.mlp.nbytes)

    def mlp_split(self):
        """Return (W0, b0, W1, b1, W2, b2) views of the flat parameter vector."""
        i, h = self.mlp_in, self.mlp_hidden
        shapes = [(i, h), (h,), (h, h), (h,), (h, MLP_OUT), (MLP_OUT,)]
        out, off = [], 0
        for s in shapes:
            n = int(np.prod(s))
            out.append(self.mlp[off:off + n].reshape(s))
            off += n
        return tuple(out)


@dataclasses.dataclass
class Cameras:
    """Pinhole cameras, OpenCV axes (x right, y down, z forward).

    ``c2w[i]`` is a 3x4 row-major camera-to-world matrix whose first three
    columns are the camera axes in world space and whose last column is the
    camera centre.  ``intr[i] = (fx, fy, cx, cy)`` in pixels; ``size[i] =
    (width, height)``.
    """
    c2w: np.ndarray   # float32 [n, 3, 4]
    intr: np.ndarray  # float32 [n, 4]
    size: np.ndarray  # int32 [n, 2]

    def __len__(self):
        return int(self.c2w.shape[0])

    def num_pixels(self) -> int:
        return int(np.sum(self.size[:, 0].astype(np.int64) * self.size[:, 1]))

    def subset(self, idx) -> "Cameras":
        idx = np.atleast_1d(idx)
        return Cameras(self.c2w[idx].copy(), self.intr[idx].copy(), self.size[idx].copy())


def mlp_param_count(mlp_in: int = MLP_IN, hidden: int = MLP_HIDDEN) -> int:
    return mlp_in * hidden + hidden + hidden * hidden + hidden + hidden * MLP_OUT + MLP_OUT


# ----------------------------------------------------------------------------
# occupancy drawing
# ----------------------------------------------------------------------------

def _axis_cells(res: int):
    """Lower/upper box bounds of the cells of one axis at resolution ``res``."""
    h = 4.0 / res
    lo = -2.0 + h * np.arange(res)
    return lo, lo + h


def reachable_mask(res: int) -> np.ndarray:
    """Cells that meet the image of the contraction (at most one axis outside [-1, 1])."""
    lo, hi = _axis_cells(res)
    outside = (lo >= 1.0) | (hi <= -1.0)                     # per axis, box misses [-1, 1]
    cnt = (outside[:, None, None].astype(np.int8) + outside[None, :, None]
           + outside[None, None, :])
    return cnt <= 1


def maxpool(a: np.ndarray, f: int) -> np.ndarray:
    r = a.shape[0]
    assert r % f == 0
    n = r // f
    return a.reshape(n, f, n, f, n, f).max(axis=(1, 3, 5))


def _mark_sphere(occ: np.ndarray, center: np.ndarray, rad: float, extent: float,
                 reach: np.ndarray):
    """Mark the cells meeting the sphere; returns the touched index box (lo, hi) per axis (x, y, z)."""
    res = occ.shape[0]
    h = 4.0 / res
    lo_i = np.clip(np.floor((center - rad + 2.0) / h).astype(int), 0, res - 1)
    hi_i = np.clip(np.floor((center + rad + 2.0) / h).astype(int), 0, res - 1)
    ax = []
    for a in range(3):   # a = 0:x, 1:y, 2:z
        idx = np.arange(lo_i[a], hi_i[a] + 1)
        blo = -2.0 + idx * h
        bhi = blo + h
        gap = np.maximum(np.maximum(blo - center[a], center[a] - bhi), 0.0)
        inside_ext = (blo < extent) & (bhi > -extent)
        ax.append((idx, gap, inside_ext))
    (ix, gx, ex), (iy, gy, ey), (iz, gz, ez) = ax
    d2 = gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2
    hit = (d2 <= rad * rad) & ez[:, None, None] & ey[None, :, None] & ex[None, None, :]
    sub = np.ix_(iz, iy, ix)
    occ[sub] |= (hit & reach[sub]).astype(np.uint8)
    return lo_i, hi_i


def draw_occupancy(L: int, target_block_frac: float, extent: float, r_lo: float, r_hi: float,
                   rng: np.random.Generator, max_spheres: int = 100000) -> Tuple[np.ndarray, int]:
    """Add random spheres until the block-mask occupancy reaches the target.

    The block count is checked after every sphere for small targets and after
    every 8th sphere otherwise.  Returns the finest occupancy level
    (resolution L/4, uint8 0/1) and the number of spheres drawn.
    """
    rf = L // 4
    nb = L // BLOCK
    occ = np.zeros((rf, rf, rf), np.uint8)
    blocks = np.zeros((nb, nb, nb), np.uint8)     # max-pool x2 of occ, kept up to date
    count = 0
    reach = reachable_mask(rf)
    target = target_block_frac * nb ** 3
    n = 0
    while n < max_spheres:
        center = rng.uniform(-extent, extent, 3)
        rad = rng.uniform(r_lo, r_hi)
        lo_i, hi_i = _mark_sphere(occ, center, rad, extent, reach)
        b0, b1 = lo_i // 2, hi_i // 2 + 1           # touched blocks, (x, y, z)
        sub = occ[2 * b0[2]:2 * b1[2], 2 * b0[1]:2 * b1[1], 2 * b0[0]:2 * b1[0]]
        new = maxpool_box(sub)
        old = blocks[b0[2]:b1[2], b0[1]:b1[1], b0[0]:b1[0]]
        count += int(new.sum()) - int(old.sum())
        blocks[b0[2]:b1[2], b0[1]:b1[1], b0[0]:b1[0]] = new
        n += 1
        if n % 8 == 0 or target < 4096:
            if count >= target:
                break
    return occ, n


def maxpool_box(a: np.ndarray) -> np.ndarray:
    """Max-pool by 2 along every axis of a box with even extents."""
    z, y, x = a.shape
    return a.reshape(z // 2, 2, y // 2, 2, x // 2, 2).max(axis=(1, 3, 5))


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

SCENE_PRESETS = {
    # name: (L, R, block occupancy, extent c, r_lo, r_hi, occupancy pools coarse->fine, mlp seed)
    "tiny": dict(L=64, R=256, frac=0.10, extent=2.0, r_lo=0.15, r_hi=0.5, pools=(2, 1), mlp_seed=11),
    "full": dict(L=512, R=2048, frac=0.05, extent=1.99, r_lo=0.05, r_hi=0.25, pools=(8, 2, 1), mlp_seed=12),
}


def make_scene(L: int, R: int, frac: float, extent: float, r_lo: float, r_hi: float,
               pools=(8, 2, 1), seed: int = 0, mlp_seed: Optional[int] = None,
               name: str = "custom") -> Scene:
    """Draw a scene: spheres -> occupancy pyramid -> stored blocks -> random bytes."""
    assert L % BLOCK == 0 and (L // 4) % max(pools) == 0
    rng = np.random.default_rng(seed)
    fine, _ = draw_occupancy(L, frac, extent, r_lo, r_hi, rng)
    occ = [(fine.shape[0] // p, maxpool(fine, p) if p > 1 else fine.copy()) for p in pools]
    mask = maxpool(fine, 2).reshape(-1)              # resolution L/8 == block grid
    nb = L // BLOCK
    block_index = np.full(nb ** 3, -1, np.int32)
    stored = np.nonzero(mask)[0]
    block_index[stored] = np.arange(stored.size, dtype=np.int32)
    blocks = rng.integers(0, 256, size=(stored.size, BLOCK, BLOCK, BLOCK, CHANNELS), dtype=np.uint8)
    planes = rng.integers(0, 256, size=(3, R, R, CHANNELS), dtype=np.uint8)
    mrng = np.random.default_rng(seed + 1000 if mlp_seed is None else mlp_seed)
    mlp = mrng.normal(0.0, 0.1, size=mlp_param_count()).astype(np.float32)
    return Scene(name=name, seed=seed, L=L, R=R, block_index=block_index, blocks=blocks,
                 planes=planes, occ=occ, mlp=mlp, step=4.0 / max(R, L))


def planes_only(scene: Scene) -> Scene:
    """The same scene without its 3D grid (L = 0): the paper's ablation of MERF
    without the low-resolution voxel grid (Sec. 7)."""
    return dataclasses.replace(scene, name=scene.name + "-planes", L=0,
                               block_index=np.zeros(0, np.int32),
                               blocks=np.zeros((0, BLOCK, BLOCK, BLOCK, CHANNELS), np.uint8))


def grid_only_scene(L: int, frac: float, seed: int, extent: float = 1.99, r_lo: float = 0.05,
                    r_hi: float = 0.25, mlp_seed: Optional[int] = None) -> Scene:
    """A block-sparse grid with no planes (R = 0), e.g. a high-resolution grid in
    the spirit of the paper's SNeRG++ comparison."""
    sc = make_scene(L, 0, frac, extent, r_lo, r_hi, pools=(8, 2, 1), seed=seed, mlp_seed=mlp_seed,
                    name=f"grid{L}")
    return sc


def preset_scene(name: str, seed: Optional[int] = None) -> Scene:
    """The tiny (seed 1) and full-size (seed 2) plain scenes."""
    p = SCENE_PRESETS[name]
    if seed is None:
        seed = {"tiny": 1, "full": 2}[name]
    return make_scene(p["L"], p["R"], p["frac"], p["extent"], p["r_lo"], p["r_hi"],
                      pools=p["pools"], seed=seed, mlp_seed=p["mlp_seed"], name=name)


def serving_scenes(seeds=range(100, 108)) -> List[Scene]:
    """Resident scene mix: occupancy U[2%, 15%], (L, R) in {(256, 1024), (512, 2048)}."""
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        frac = float(rng.uniform(0.02, 0.15))
        L, R = [(256, 1024), (512, 2048)][int(rng.integers(0, 2))]
        out.append(make_scene(L, R, frac, 1.99, 0.05, 0.25, pools=(8, 2, 1), seed=s,
                              mlp_seed=s + 5000, name=f"serve{s}"))
    return out


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def _look_at(pos: np.ndarray, forward: np.ndarray, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    f = forward / np.linalg.norm(forward)
    up = np.asarray(up, np.float64)
    if abs(np.dot(f, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    m = np.zeros((3, 4))
    m[:, 0], m[:, 1], m[:, 2], m[:, 3] = right, down, f, pos
    return m


def _intrinsics(w: int, h: int, hfov_deg: float = 60.0):
    fx = (w / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return (fx, fx, w / 2.0, h / 2.0)


def make_cameras(poses: List[np.ndarray], sizes: List[Tuple[int, int]], hfov_deg: float = 60.0) -> Cameras:
    n = len(poses)
    c2w = np.stack([np.asarray(p, np.float64) for p in poses]).astype(np.float32).reshape(n, 3, 4)
    intr = np.array([_intrinsics(w, h, hfov_deg) for (w, h) in sizes], np.float32)
    size = np.array(sizes, np.int32).reshape(n, 2)
    return Cameras(c2w, intr, size)


def _unit(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def tiny_camera(seed: int = 21, w: int = 128, h: int = 128) -> Cameras:
    """Camera at radius 3 (world units) looking at the origin, up +z."""
    rng = np.random.default_rng(seed)
    pos = 3.0 * _unit(rng)
    return make_cameras([_look_at(pos, -pos)], [(w, h)])


def full_camera(seed: int = 22, w: int = 1920, h: int = 1080) -> Cameras:
    """Camera inside the unit cube (U[-0.5, 0.5]^3) with a random look direction."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-0.5, 0.5, 3)
    return make_cameras([_look_at(pos, _unit(rng))], [(w, h)])


def orbit_cameras(n: int = 16, seed: int = 23, radius: float = 0.5, w: int = 1920, h: int = 1080) -> Cameras:
    """Cameras on a horizontal orbit about the origin, looking outward with yaw/pitch jitter."""
    rng = np.random.default_rng(seed)
    poses = []
    for i in range(n):
        th = 2.0 * math.pi * i / n
        pos = np.array([radius * math.cos(th), radius * math.sin(th), 0.0])
        yaw = th + rng.uniform(-0.5, 0.5)
        pitch = rng.uniform(-0.3, 0.3)
        fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
        poses.append(_look_at(pos, fwd))
    return make_cameras(poses, [(w, h)] * n)


def random_cameras(n: int, seed: int, sizes: List[Tuple[int, int]], inside: float = 0.5) -> Cameras:
    """Cameras at U[-inside, inside]^3 with random look directions (serving requests)."""
    rng = np.random.default_rng(seed)
    poses = [_look_at(rng.uniform(-inside, inside, 3), _unit(rng)) for _ in range(n)]
    return make_cameras(poses, sizes)


def concat_cameras(cams: List[Cameras]) -> Cameras:
    return Cameras(np.concatenate([c.c2w for c in cams]), np.concatenate([c.intr for c in cams]),
                   np.concatenate([c.size for c in cams]))
