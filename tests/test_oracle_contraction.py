"""Pins of the oracle's contraction and ray segmentation (Sec. 4.2, Eq. 7).

Checked against hand-evaluated values, the invariants the paper states
(identity on the unit cube; seven regions, each a projective map, so rays
stay straight inside a region) and an inverse map derived separately from
Eq. 7 in this file.
"""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "contraction_eq7.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b = line.split("|")
        rows.append((np.array(a.split(), float), np.array(b.split(), float)))
    return rows


def inverse_eq7(reg, y):
    """Preimage of y under the region map, solved from Eq. 7 by hand:
    |x_j| = 1 / (2 - s y_j), x_j = s |x_j|, x_k = y_k |x_j|."""
    y = np.asarray(y, float)
    if reg == 0:
        return y.copy()
    j, s = (reg - 1) // 2, (-1.0 if (reg - 1) % 2 else 1.0)
    a = 1.0 / (2.0 - s * y[j])
    x = y * a
    x[j] = s * a
    return x


def test_golden_values():
    for x, y in _golden():
        assert np.allclose(oracle.contract(x), y, rtol=0, atol=1e-15), (x, oracle.contract(x), y)


def test_identity_inside_unit_cube():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, (500, 3))
    assert np.array_equal(oracle.contract(x), x)


def test_image_is_seven_regions():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2000, 3)) * np.exp(rng.uniform(-2, 8, (2000, 1)))
    y = oracle.contract(x)
    assert np.all(np.abs(y).max(axis=1) < 2.0)
    # at most one coordinate outside [-1, 1], and it lies on the max axis of x
    outside = np.abs(y) > 1.0
    assert np.all(outside.sum(axis=1) <= 1)
    r = np.abs(x).max(axis=1)
    far = r > 1.0
    assert np.array_equal(outside.any(axis=1), far & (r > 1.0) & (np.abs(y).max(axis=1) > 1.0))
    # each point's image is on the same side of the origin per axis
    assert np.all(np.sign(y) == np.sign(x))


def test_continuous_across_cube_faces():
    rng = np.random.default_rng(2)
    for _ in range(200):
        p = rng.uniform(-1, 1, 3)
        j = rng.integers(0, 3)
        p[j] = rng.choice([-1.0, 1.0])
        n = np.zeros(3)
        n[j] = np.sign(p[j])
        a = oracle.contract(p - 1e-9 * n)
        b = oracle.contract(p + 1e-9 * n)
        assert np.abs(a - b).max() < 1e-8


def test_mirror_jump_across_outer_seams():
    # (2+e, 2, 1/2) and (2, 2+e, 1/2) approach the same seam point from its two
    # sides; Eq. 7 sends them to mirror images (1.5, 1, .25) and (1, 1.5, .25).
    e = 1e-10
    a = oracle.contract([2 + e, 2, 0.5])
    b = oracle.contract([2, 2 + e, 0.5])
    assert np.allclose(a, [1.5, 1.0, 0.25], atol=1e-9)
    assert np.allclose(b, [1.0, 1.5, 0.25], atol=1e-9)


def test_projective_within_region_keeps_lines_straight():
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(400):
        o = rng.normal(size=3) * 3
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ts = np.sort(rng.uniform(0, 20, 3))
        xs = o + ts[:, None] * d
        regs = [oracle.region(x) for x in xs]
        if len(set(regs)) != 1:
            continue
        ys = oracle.contract(xs)
        c = np.cross(ys[1] - ys[0], ys[2] - ys[0])
        assert np.linalg.norm(c) < 1e-12 * max(1.0, np.linalg.norm(ys[1] - ys[0]) * np.linalg.norm(ys[2] - ys[0])) + 1e-14
        checked += 1
    assert checked > 50


def _rays(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        scale = [0.5, 3.0, 30.0][i % 3]
        o = rng.uniform(-scale, scale, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        out.append((o, d))
    # axis-aligned and diagonal special cases
    out.append((np.zeros(3), np.array([1.0, 0, 0])))
    out.append((np.array([0.3, -0.2, 0.1]), np.array([0.0, 0.0, -1.0])))
    out.append((np.zeros(3), np.ones(3) / np.sqrt(3)))
    out.append((np.array([5.0, 0.0, 0.0]), np.array([-1.0, 0.0, 0.0])))
    return out


def test_segments_tile_the_ray_and_are_regions():
    for o, d in _rays(300, 4):
        ta, tb, reg, ya, yb = oracle.segments(o, d)
        n = len(ta)
        assert 1 <= n <= 7
        assert ta[0] == 0.0 and np.isinf(tb[-1])
        assert np.all(tb[:-1] == ta[1:])
        assert np.all(reg[:-1] != reg[1:])
        for i in range(n):
            # the region of interior points is the segment's region
            hi = tb[i] if np.isfinite(tb[i]) else ta[i] + 1e6
            for f in (0.25, 0.5, 0.75):
                t = ta[i] + f * (hi - ta[i])
                assert oracle.region(o + t * d) == reg[i]
            # segment ends are contracted points of the ray (or its limit)
            assert np.allclose(inverse_eq7(reg[i], ya[i]), o + ta[i] * d, atol=1e-9 * max(1, ta[i]))
            if np.isfinite(tb[i]):
                assert np.allclose(inverse_eq7(reg[i], yb[i]), o + tb[i] * d, atol=1e-9 * max(1, tb[i]))
            else:
                far = oracle.contract(o + 1e9 * d)
                assert np.allclose(far, yb[i], atol=1e-7)


def test_breakpoints_lie_on_region_boundaries():
    for o, d in _rays(300, 5):
        ta, tb, reg, ya, yb = oracle.segments(o, d)
        for t in tb[:-1]:
            x = o + t * d
            r = np.abs(x).max()
            on_face = abs(r - 1.0) < 1e-9 * max(1, t)
            ax = np.sort(np.abs(x))
            on_seam = r > 1 and abs(ax[2] - ax[1]) < 1e-9 * max(1, t)
            assert on_face or on_seam


def test_samples_lie_on_world_ray(tiny_scene):
    """Every sample of the oracle's lattice maps back onto the world ray."""
    rng = np.random.default_rng(6)
    for _ in range(40):
        o = rng.uniform(-3, 3, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        _, st, log = oracle.render_ray(tiny_scene, o, d, t_min=0.0)
        ta, tb, reg, ya, yb = oracle.segments(o, d)
        for s in log[:: max(1, len(log) // 50)]:
            x = inverse_eq7(reg[s["segment"]], s["p"])
            t = np.dot(x - o, d)
            assert np.linalg.norm(x - (o + t * d)) < 1e-9 * max(1.0, abs(t))
            assert ta[s["segment"]] - 1e-9 <= t <= tb[s["segment"]] * (1 + 1e-9) + 1e-9


def test_limit_point_of_last_segment():
    for o, d in _rays(100, 7):
        ta, tb, reg, ya, yb = oracle.segments(o, d)
        j = int(np.argmax(np.abs(d)))
        assert reg[-1] == 1 + 2 * j + (1 if d[j] < 0 else 0)
        assert abs(abs(yb[-1][j]) - 2.0) < 1e-15
