"""The edge-case cameras really produce the rays they are meant to: exact
zero and exactly equal direction components (checked on the oracle's own
FP64 rays from the float32 poses)."""
import numpy as np

import oracle
from edge_cameras import edge_cameras


def ray(cams, c, i, j):
    _, d = oracle.camera_rays(cams, c, [i], [j])
    return d[0]


def test_axis_camera_has_zero_and_equal_components():
    names, cams = edge_cameras()
    c = names.index("axis +x inside")
    assert np.array_equal(ray(cams, c, 16, 16), [1.0, 0.0, 0.0])
    d = ray(cams, c, 16, 3)                # centre row: no vertical component
    assert d[2] == 0.0 and d[1] != 0.0
    d = ray(cams, c, 3, 3)                 # diagonal pixel: |d_y| = |d_z|
    assert abs(d[1]) == abs(d[2]) and d[1] != 0.0


def test_diagonal_cameras_have_equal_components():
    names, cams = edge_cameras()
    d = ray(cams, names.index("diagonal x=y on seam"), 16, 16)
    assert d[0] == d[1] and d[2] == 0.0
    d = ray(cams, names.index("diagonal x=-y outside"), 16, 16)
    assert d[0] == -d[1] and d[2] == 0.0
    d = ray(cams, names.index("3-D diagonal"), 16, 16)
    assert d[0] == d[1] == d[2]


def test_seam_camera_centre_ray_lies_on_the_seam():
    names, cams = edge_cameras()
    c = names.index("diagonal x=y on seam")
    o, d = oracle.camera_rays(cams, c, [16], [16])
    for t in (0.5, 1.0, 3.0, 10.0):
        x = o[0] + t * d[0]
        assert x[0] == x[1]
