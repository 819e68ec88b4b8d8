"""Positive and negative pins of the oracle's fragility flags.

A pixel is flagged when an FP32 renderer may legitimately take a different
discrete decision than the FP64 oracle (a sample on an occupancy cell face
whose two sides differ, a segment whose length is an integer number of steps
with an occupied end, or two region breakpoints that coincide at an occupied
point).  These tests place rays so that each condition holds exactly, or
clearly fails, and check the flag (Sec. 6 occupancy test; Sec. 4.2 Eq. 7
breakpoints; sample lattice of the contracted march).
"""
import numpy as np

import oracle
from test_oracle_render import box_scene

# box_scene(L=64): planes R = 64, step 4/64 = 1/16; finest occupancy level
# 16^3 (cell edge 1/4), coarse level 8^3; a box of cells is occupied.
STEP = 1.0 / 16.0


def flag(scene, o, d):
    _, st, log = oracle.render_ray(scene, np.asarray(o, float), np.asarray(d, float), step=STEP)
    return int(st["fragile"]), log


def test_sample_on_a_deciding_face_is_flagged():
    # occupied x in [0, 1]; x = 0 separates an empty and an occupied cell.
    sc = box_scene(np.array([0.0, -0.5, -0.5]), np.array([1.0, 0.5, 0.5]))
    # inside the cube contracted = world; samples at x0 + (k + 1/2)/16, so
    # x0 = -3.5/16 puts sample k = 3 exactly on x = 0
    o = [-3.5 / 16.0, 0.01, 0.02]
    f, log = flag(sc, o, [1.0, 0.0, 0.0])
    assert np.any(log["p"][:, 0] == 0.0)
    assert f == 1


def test_samples_away_from_faces_are_not_flagged():
    sc = box_scene(np.array([0.0, -0.5, -0.5]), np.array([1.0, 0.5, 0.5]))
    # x0 = -0.234375: samples at odd multiples of 1/64 from the faces, and the
    # cube segment is 19.75 steps long
    o = [-0.234375, 0.01, 0.02]
    f, log = flag(sc, o, [1.0, 0.0, 0.0])
    assert log["evaluated"].sum() > 0
    assert f == 0


def test_sample_on_a_face_between_two_occupied_cells_is_not_flagged():
    sc = box_scene(np.array([0.0, -0.5, -0.5]), np.array([1.0, 0.5, 0.5]))
    # samples land exactly on x = 0.5 and x = 0.75, faces between occupied
    # cells: moving across them changes nothing
    o = [0.5 - 3.5 / 16.0, 0.01, 0.02]
    f, log = flag(sc, o, [1.0, 0.0, 0.0])
    xs = log["p"][:, 0]
    assert np.any(xs == 0.5) and np.any(xs == 0.75)
    assert f == 0


def test_integer_interval_count_with_occupied_end_is_flagged():
    # occupied x in [0, 1.25]: the cube face x = 1 lies inside occupied space
    sc = box_scene(np.array([0.0, -0.5, -0.5]), np.array([1.2, 0.5, 0.5]))
    # the cube segment from x = -0.25 to x = 1 is exactly 20 steps
    f, _ = flag(sc, [-0.25, 0.01, 0.02], [1.0, 0.0, 0.0])
    assert f == 1
    # 19.75 steps: no flag
    f, _ = flag(sc, [-0.234375, 0.01, 0.02], [1.0, 0.0, 0.0])
    assert f == 0


def test_ray_through_a_cube_edge_at_an_occupied_point_is_flagged():
    # occupied box around the cube edge x = y = 1
    sc = box_scene(np.array([0.5, 0.5, -0.5]), np.array([1.5, 1.5, 0.5]))
    d = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
    # x = 1 and y = 1 are reached at the same t: two coinciding breakpoints
    c = oracle.candidates([0.5, 0.5, 0.1], d)
    assert np.min(np.diff(np.sort(c))) == 0.0
    f, _ = flag(sc, [0.5, 0.5, 0.1], d)
    assert f == 1
    # shifted off the edge, the breakpoints are 0.05 apart
    f, _ = flag(sc, [0.5, 0.45, 0.1], d)
    assert f == 0
