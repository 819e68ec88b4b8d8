"""Cameras whose rays have exactly zero or exactly equal direction
components, for parity cases at the breakpoints of Eq. 7 (Sec. 4.2).

With an odd image size, cx = W/2 and cy = H/2, the centre column has
(j + 1/2 - cx) = 0 and the centre row (i + 1/2 - cy) = 0 exactly; with
fx = fy, pixels on the image diagonals through the centre have equal
|vx| = |vy|.  An axis-aligned pose (entries 0 and +-1) therefore gives rays
with d_j = +-0 and rays with |d_j| = |d_k|; a pose whose entries are
+-float32(sqrt(1/2)) gives rays with d_x = +-d_y exactly, and a pose with
equal float32 entries on the 3-D diagonal gives d_x = d_y = d_z.  The origins
put rays across the cube faces and the outer seams |x_j| = |x_k|, and some run
along a seam or through a cube edge.
"""
import numpy as np

import synth

H2 = float(np.float32(np.sqrt(0.5)))
H3 = float(np.float32(np.sqrt(1.0 / 3.0)))


def _pose(right, down, fwd, pos):
    m = np.zeros((3, 4))
    m[:, 0], m[:, 1], m[:, 2], m[:, 3] = right, down, fwd, pos
    return m


def edge_poses():
    """(name, 3x4 pose, (width, height)) of each edge-case camera."""
    x, y, z = np.eye(3)
    return [
        # inside the cube, looking +x: rays leave through x = 1 into region +x
        ("axis +x inside", _pose(-y, -z, x, [0.05, -0.3, 0.2]), (33, 33)),
        # outside, looking -x: region +x, the cube, region -x
        ("axis -x outside", _pose(y, -z, -x, [2.5, 0.3, -0.2]), (33, 33)),
        # inside, looking +z, non-square odd frame
        ("axis +z inside", _pose(x, y, z, [0.1, 0.2, -0.1]), (31, 17)),
        # far outside below, looking +z through the whole cube
        ("axis +z outside", _pose(x, -y, z, [-0.2, 0.1, -3.0]), (33, 33)),
        # 45 degrees in x-y from a point on the seam x = y: the centre column
        # runs along that seam, and through the cube edge x = y = 1
        ("diagonal x=y on seam", _pose([H2, -H2, 0.0], -z, [H2, H2, 0.0], [0.3, 0.3, 0.1]), (33, 33)),
        # 45 degrees in x-y from off the seam, outside the cube
        ("diagonal x=-y outside", _pose([H2, H2, 0.0], -z, [-H2, H2, 0.0], [1.5, -1.5, 0.2]), (33, 33)),
        # along the 3-D diagonal from a point on it: all three seams at once
        ("3-D diagonal", _pose([H2, -H2, 0.0], [0.40824829, 0.40824829, -0.81649658], [H3, H3, H3],
                               [-0.2, -0.2, -0.2]), (33, 33)),
        # a single ray, the optical axis of the first camera
        ("single axis ray", _pose(-y, -z, x, [0.05, -0.3, 0.2]), (1, 1)),
    ]


def edge_cameras():
    poses = edge_poses()
    cams = synth.make_cameras([p for _, p, _ in poses], [s for _, _, s in poses])
    # exact principal points and equal focal lengths
    cams.intr[:, 2] = cams.size[:, 0] / 2.0
    cams.intr[:, 3] = cams.size[:, 1] / 2.0
    cams.intr[:, 1] = cams.intr[:, 0]
    return [n for n, _, _ in poses], cams


def special_pixels(w, h):
    """Flat indices of the centre row, centre column and both diagonals
    through the centre of a w x h frame (odd sizes)."""
    cx, cy = (w - 1) // 2, (h - 1) // 2
    idx = set()
    for j in range(w):
        idx.add(cy * w + j)
    for i in range(h):
        idx.add(i * w + cx)
    for k in range(-min(cx, cy), min(cx, cy) + 1):
        idx.add((cy + k) * w + cx + k)
        idx.add((cy + k) * w + cx - k)
    return sorted(idx)
